"""ctypes declarations of libteuk's C ABI (include/teuk.h).  Marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# TEUK_LIB selects another build of the same ABI (e.g. an installed copy).
LIB_PATH = os.environ.get("TEUK_LIB") or os.path.join(HERE, "libteuk.so")

OK, EINVAL, ESTATE, EDEVICE, EUNSTABLE, ENOTSUP = 0, -1, -2, -3, -4, -5
FP64, FP32, FP32S = 64, 32, 48   # FP32S: FP32 storage, FP64 arithmetic
PARAM_A, PARAM_M, PARAM_R0, PARAM_AMP = 0, 1, 2, 3   # parameters of teuk_param_gradient


class TeukGrid(ctypes.Structure):
    _fields_ = [("n_rstar", ctypes.c_int64), ("n_theta", ctypes.c_int64),
                ("rstar_min", ctypes.c_double), ("rstar_max", ctypes.c_double)]


class TeukError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        super().__init__(f"{_strerror(code)}{': ' + msg if msg else ''}")


class TeukDesc(ctypes.Structure):
    _fields_ = [("grid", TeukGrid), ("a", ctypes.c_double), ("M", ctypes.c_double), ("m", ctypes.c_int32),
                ("s", ctypes.c_int32), ("dt", ctypes.c_double), ("r0", ctypes.c_double), ("amp", ctypes.c_double),
                ("sigma_r_cells", ctypes.c_double), ("sigma_th_cells", ctypes.c_double),
                ("rstar_obs", ctypes.c_double)]


_P = ctypes.c_void_p
_D = ctypes.c_double
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SIGS = {
    "teuk_create": (ctypes.c_int, [ctypes.POINTER(TeukGrid), _D, _D, _I32, _I32, _D, _I32, _P,
                                   ctypes.POINTER(_P)]),
    "teuk_destroy": (ctypes.c_int, [_P]),
    "teuk_bind_state": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "teuk_set_source": (ctypes.c_int, [_P, _D, _D, _D, _D]),
    "teuk_set_observer": (ctypes.c_int, [_P, _D, _P, _I64]),
    "teuk_set_trajectory": (ctypes.c_int, [_P, _P, _I64]),
    "teuk_step": (ctypes.c_int, [_P, _I64]),
    "teuk_extract": (ctypes.c_int, [_P, _D, _P]),
    "teuk_get_time": (ctypes.c_int, [_P, ctypes.POINTER(_D), ctypes.POINTER(_I64)]),
    "teuk_set_time": (ctypes.c_int, [_P, _D, _I64]),
    "teuk_get_clock": (ctypes.c_int, [_P, ctypes.POINTER(_D), ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "teuk_set_clock": (ctypes.c_int, [_P, _D, _I64, _I64]),
    "teuk_current": (ctypes.c_int, [_P]),
    "teuk_set_tiling": (ctypes.c_int, [_P, _I32, _I32]),
    "teuk_get_tiling": (ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "teuk_set_blocking": (ctypes.c_int, [_P, _I32]),
    "teuk_get_blocking": (ctypes.c_int, [_P]),
    "teuk_adjoint_workspace_bytes": (_I64, [_P]),
    "teuk_adjoint": (ctypes.c_int, [_P, _D, _P, _I64, _D, _P, _I64, _P, _P, ctypes.POINTER(_D),
                                    ctypes.POINTER(_D)]),
    "teuk_adjoint_noalloc_max_bytes": (_I64, []),
    "teuk_adjoint_noalloc": (ctypes.c_int, [_P, _D, _P, _I64, _D, _P, _P, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "teuk_autotune": (ctypes.c_int, [_P, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "teuk_set_adjoint_tiling": (ctypes.c_int, [_P, _I32, _I32]),
    "teuk_param_gradient_workspace_bytes": (_I64, [_P, _I64, _I64]),
    "teuk_param_gradient": (ctypes.c_int, [_P, _I32, ctypes.c_double, ctypes.c_double, _P, _I64, ctypes.c_double,
                                           _P, _P, _I64, _P, _I64, ctypes.POINTER(ctypes.c_double), _P, _P]),
    "teuk_adjoint_moving": (ctypes.c_int, [_P, ctypes.c_double, _P, _I64, _P, _I64, _P, _P, _P,
                                           ctypes.POINTER(ctypes.c_double)]),
    "teuk_get_adjoint_tiling": (ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "teuk_adjoint_autotune": (ctypes.c_int, [_P, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "teuk_batch_create": (ctypes.c_int, [_I32, ctypes.POINTER(TeukDesc), _I64, _P, ctypes.POINTER(_P)]),
    "teuk_batch_destroy": (ctypes.c_int, [_P]),
    "teuk_batch_bind": (ctypes.c_int, [_P, _I32, _P, _P, _P, _P, _P, _I64]),
    "teuk_batch_set_trajectory": (ctypes.c_int, [_P, _I32, _P, _I64]),
    "teuk_batch_step": (ctypes.c_int, [_P, _I64]),
    "teuk_batch_capture_graph": (ctypes.c_int, [_P, _I64]),
    "teuk_batch_set_tiling": (ctypes.c_int, [_P, _I32, _I32, _I32]),
    "teuk_batch_autotune": (ctypes.c_int, [_P, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                           ctypes.POINTER(_I32)]),
    "teuk_batch_current": (ctypes.c_int, [_P]),
    "teuk_batch_get_step": (ctypes.c_int, [_P, ctypes.POINTER(_I64)]),
    "teuk_batch_status": (ctypes.c_int, [_P]),
    "teuk_batch_last_error": (ctypes.c_char_p, [_P]),
    "teuk_batch_set_watchdog": (ctypes.c_int, [_P, _I32, ctypes.c_double]),
    "teuk_check_finite": (ctypes.c_int, [_P]),
    "teuk_set_watchdog": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_double]),
    "teuk_status": (ctypes.c_int, [_P]),
    "teuk_last_error": (ctypes.c_char_p, [_P]),
    "teuk_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "teuk_suggest_dt": (ctypes.c_int, [ctypes.POINTER(TeukGrid), _D, _D, _I32, _I32, _I64,
                                       ctypes.POINTER(_D)]),
    "teuk_stream_copy": (ctypes.c_int, [_P, _P, _I64, _P]),
    "teuk_rstar_of_r": (_D, [_D, _D, _D]),
    "teuk_delta_of_rstar": (_D, [_D, _D, _D]),
}

_lib = None


def lib():
    """Load libteuk.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libteuk.so not found at {LIB_PATH}; build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        # PyTorch ships its own HIP and HSA runtimes under the same sonames as
        # the system's.  Importing it first makes the library bind to those, so
        # the process holds one runtime; loaded the other way round, torch
        # would bring up a second runtime beside the library's on the same GPU.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _strerror(code):
    try:
        return lib().teuk_strerror(code).decode()
    except Exception:
        return f"teuk error {code}"


def check(code, ctx=None):
    if code != OK:
        msg = ""
        if ctx:
            msg = lib().teuk_last_error(ctx).decode()
        raise TeukError(code, msg)
    return code
