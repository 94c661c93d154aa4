"""Plain FP64 CPU oracle for the m-mode 2+1 Teukolsky Lax-Wendroff step.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's
CPU-baseline leg use it to check the GPU library.  The product path never
imports it.  It shares no code with the HIP library; its arithmetic lives in
``teuk_oracle.c`` (written from the paper's Eqs. (1)-(14) and the boundary
conditions stated after Eq. (14)); this module only marshals numpy arrays.

Functions that have no external pin are named in ``PARITY_UNPINNED``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "teuk_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Kerr (a != 0) pointwise field values have no printed value to compare
# with.  They are pinned indirectly: by the l = m = 2 ringdown frequencies at
# a = 0.5, 0.9 and 0.99 (tests/golden, Leaver's values), which depend on
# every a-dependent coefficient, and by the invariants (convergence order,
# mirror symmetry, linearity, a -> 0 continuity, adjoint identity).  No
# function of the oracle is left without a pin.
PARITY_UNPINNED = ()


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain IEEE FP64: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fcx-fortran-rules", "-fno-fast-math",
               _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nr", ctypes.c_int64), ("nth", ctypes.c_int64),
        ("rstar_min", ctypes.c_double), ("rstar_max", ctypes.c_double),
        ("i0", ctypes.c_int64), ("ni", ctypes.c_int64),
        ("j0", ctypes.c_int64), ("nj", ctypes.c_int64),
        ("a", ctypes.c_double), ("M", ctypes.c_double),
        ("m", ctypes.c_int32), ("s", ctypes.c_int32),
        ("dt", ctypes.c_double),
        ("r0", ctypes.c_double), ("amp", ctypes.c_double),
        ("sigma_r_cells", ctypes.c_double), ("sigma_th_cells", ctypes.c_double),
        ("rstar_obs", ctypes.c_double),
    ]


_lib = None


def _L():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        D, I64, P, I32 = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32
        sig = {
            "teuko_rstar_of_delta": (D, [D, D, D]),
            "teuko_rstar_of_r": (D, [D, D, D]),
            "teuko_delta_of_rstar": (D, [D, D, D]),
            "teuko_coeffs": (None, [D, D, D, D, ctypes.c_int, ctypes.c_int, P]),
            "teuko_create": (P, [ctypes.POINTER(_Params)]),
            "teuko_destroy": (None, [P]),
            "teuko_angular_apply": (None, [I64, I32, I32, P, P]),
            "teuko_step": (ctypes.c_int, [P, P, P, P, P, D]),
            "teuko_extract": (ctypes.c_int, [P, P, P]),
            "teuko_run": (ctypes.c_int, [P, P, P, I64, D, P]),
            "teuko_adjoint_step": (ctypes.c_int, [P, P, P, P, P, P, P]),
            "teuko_adjoint_run": (ctypes.c_int, [P, P, I64, D, P, P,
                                                 ctypes.POINTER(D), ctypes.POINTER(D)]),
            "teuko_dr": (D, [P]), "teuko_dth": (D, [P]), "teuko_rstar0": (D, [P]),
            "teuko_Omega": (D, [P]), "teuko_iobs": (I64, [P]), "teuko_alpha": (D, [P]),
            "teuko_max_DoS2": (D, [P]),
            "teuko_set_trajectory": (ctypes.c_int, [P, P, I64, D]),
            "teuko_adjoint_run_moving": (ctypes.c_int, [P, P, I64, P, P, P, ctypes.POINTER(D)]),
            "teuko_threads": (ctypes.c_int, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


# ------------------------------------------------------------ Eq. (2)

def threads() -> int:
    """OpenMP threads the oracle's step loops use."""
    return _L().teuko_threads()


def rstar_of_r(r: float, a: float, M: float = 1.0) -> float:
    """Tortoise coordinate r*(r), Eq. (2) integrated with the standard constant."""
    return _L().teuko_rstar_of_r(r, a, M)


def delta_of_rstar(rstar: float, a: float, M: float = 1.0) -> float:
    """Inverse of Eq. (2): delta = r - r+ at the given r*."""
    return _L().teuko_delta_of_rstar(rstar, a, M)


def coeffs(delta: float, theta: float, a: float, M: float, m: int, s: int) -> dict:
    """Coefficients of the first-order system (Eqs. 5-12) at r = r+ + delta, theta."""
    out = np.zeros(11)
    _L().teuko_coeffs(delta, theta, a, M, m, s, _ptr(out))
    return {"b": out[0], "bstar": out[1], "ct": out[2] + 1j * out[3], "cr": out[4] + 1j * out[5],
            "V": out[6] + 1j * out[7], "mu": out[8] + 1j * out[9], "DoS2": out[10]}


def angular_apply(f: np.ndarray, m: int, s: int) -> np.ndarray:
    """Discrete Lth (centred differences, cell-centred grid, pole ghosts) on one column."""
    f = np.ascontiguousarray(f, dtype=np.complex128)
    out = np.zeros_like(f)
    _L().teuko_angular_apply(f.shape[0], m, s, _ptr(f), _ptr(out))
    return out


def angular_matrix(nth: int, m: int, s: int) -> np.ndarray:
    """The nth x nth matrix of the discrete Lth, assembled column by column."""
    A = np.zeros((nth, nth))
    for k in range(nth):
        e = np.zeros(nth, dtype=np.complex128)
        e[k] = 1.0
        A[:, k] = angular_apply(e, m, s).real
    return A


class Oracle:
    """One m-mode problem on an (r*, theta) grid, or a window of it."""

    def __init__(self, nr, nth, rstar_min, rstar_max, a, M, m, s, dt,
                 r0=0.0, amp=0.0, sigma_r_cells=2.0, sigma_th_cells=2.0,
                 rstar_obs=None, window=None):
        if rstar_obs is None:
            rstar_obs = 0.5 * (rstar_min + rstar_max)
        i0, ni, j0, nj = window if window is not None else (0, nr, 0, nth)
        self.p = _Params(nr, nth, rstar_min, rstar_max, i0, ni, j0, nj, a, M, m, s, dt,
                         r0, amp, sigma_r_cells, sigma_th_cells, rstar_obs)
        self.shape = (nj, ni)
        self._c = _L().teuko_create(ctypes.byref(self.p))
        if not self._c:
            raise ValueError("oracle: invalid parameters")

    def __del__(self):
        c = getattr(self, "_c", None)
        if c and _lib is not None:
            _lib.teuko_destroy(c)
            self._c = None

    dr = property(lambda self: _L().teuko_dr(self._c))
    dth = property(lambda self: _L().teuko_dth(self._c))
    rstar0 = property(lambda self: _L().teuko_rstar0(self._c))
    Omega = property(lambda self: _L().teuko_Omega(self._c))
    iobs = property(lambda self: _L().teuko_iobs(self._c))
    alpha = property(lambda self: _L().teuko_alpha(self._c))
    max_DoS2 = property(lambda self: _L().teuko_max_DoS2(self._c))

    def _arr(self, x):
        x = np.ascontiguousarray(x, dtype=np.complex128)
        assert x.shape == self.shape, (x.shape, self.shape)
        return x

    def set_trajectory(self, r0_phi, t0=0.0):
        """Moving source: r0_phi[k] = (r0, phi) at t = t0 + k dt/2 (None: static source)."""
        if r0_phi is None:
            _L().teuko_set_trajectory(self._c, None, 0, 0.0)
            self._traj = None
            return
        self._traj = np.ascontiguousarray(r0_phi, dtype=np.float64)
        assert self._traj.ndim == 2 and self._traj.shape[1] == 2
        if _L().teuko_set_trajectory(self._c, _ptr(self._traj), self._traj.shape[0], float(t0)) != 0:
            raise ValueError("oracle: invalid trajectory")

    def step(self, phi, pi, t):
        """One Lax-Wendroff step (Eqs. 13-14) from time t."""
        phi, pi = self._arr(phi), self._arr(pi)
        o1, o2 = np.empty_like(phi), np.empty_like(pi)
        if _L().teuko_step(self._c, _ptr(phi), _ptr(pi), _ptr(o1), _ptr(o2), float(t)) != 0:
            raise ValueError("oracle: step outside the trajectory table")
        return o1, o2

    def extract(self, phi):
        phi = self._arr(phi)
        out = np.empty(self.shape[0], dtype=np.complex128)
        if _L().teuko_extract(self._c, _ptr(phi), _ptr(out)) != 0:
            raise ValueError("observer columns not held")
        return out

    def run(self, phi, pi, n, t_start=0.0, record=True):
        """n steps from t_start; returns (phi, pi, wave) with wave = w^0..w^n."""
        phi = self._arr(phi).copy()
        pi = self._arr(pi).copy()
        wave = np.zeros((n + 1, self.shape[0]), dtype=np.complex128) if record else None
        rc = _L().teuko_run(self._c, _ptr(phi), _ptr(pi), int(n), float(t_start),
                            _ptr(wave) if record else None)
        if rc != 0:
            raise ValueError("oracle run failed")
        return phi, pi, wave

    def adjoint_step(self, lphi, lpi):
        """K^H applied to (lphi, lpi) plus the source adjoints (half, integer points)."""
        lphi, lpi = self._arr(lphi), self._arr(lpi)
        o = [np.empty_like(lphi) for _ in range(4)]
        _L().teuko_adjoint_step(self._c, _ptr(lphi), _ptr(lpi), *[_ptr(x) for x in o])
        return tuple(o)

    def adjoint_run(self, g, n, t_start=0.0):
        """Reverse sweep: g = dL/dw (n+1, nth).  Returns dphi0, dpi0, dL/dr0, dL/damp."""
        g = np.ascontiguousarray(g, dtype=np.complex128)
        assert g.shape == (n + 1, self.shape[0])
        d1, d2 = np.empty(self.shape, np.complex128), np.empty(self.shape, np.complex128)
        r0 = ctypes.c_double(0.0)
        am = ctypes.c_double(0.0)
        rc = _L().teuko_adjoint_run(self._c, _ptr(g), int(n), float(t_start), _ptr(d1), _ptr(d2),
                                    ctypes.byref(r0), ctypes.byref(am))
        if rc != 0:
            raise ValueError("oracle adjoint failed")
        return d1, d2, r0.value, am.value


    def adjoint_run_moving(self, g, n):
        """Reverse sweep for the orbit table of ``set_trajectory``, the forward
        run starting at its first entry: returns dphi0, dpi0, dL/dtraj
        ((2n, 2): dL/dr0_e, dL/dphi_e for entries e < 2n) and dL/damp."""
        g = np.ascontiguousarray(g, dtype=np.complex128)
        assert g.shape == (n + 1, self.shape[0])
        d1, d2 = np.empty(self.shape, np.complex128), np.empty(self.shape, np.complex128)
        dtraj = np.zeros((2 * n, 2), dtype=np.float64)
        am = ctypes.c_double(0.0)
        rc = _L().teuko_adjoint_run_moving(self._c, _ptr(g), int(n), _ptr(d1), _ptr(d2), _ptr(dtraj),
                                           ctypes.byref(am))
        if rc != 0:
            raise ValueError("oracle moving-source adjoint failed (no table, or it is too short)")
        return d1, d2, dtraj, am.value


def param_gradient_fd(nr, nth, rstar_min, rstar_max, a, M, m, s, dt, r0, amp, rstar_obs, param, h, G, n, phi0,
                      pi0, t_start=0.0) -> float:
    """dL/dp for L = Re sum conj(G) w (w^0..w^n at rstar_obs) by the central
    difference of two complete oracle runs, p + h and p - h, for p one of
    "a", "M", "r0", "amp": the definition of the derivative, to O(h^2)."""
    base = dict(a=a, M=M, r0=r0, amp=amp)
    Ls = []
    for sign in (1.0, -1.0):
        q = dict(base)
        q[param] += sign * h
        o = Oracle(nr, nth, rstar_min, rstar_max, q["a"], q["M"], m, s, dt, r0=q["r0"], amp=q["amp"],
                   rstar_obs=rstar_obs)
        _, _, w = o.run(phi0, pi0, n, t_start)
        Ls.append(float(np.sum((np.conj(G) * w).real)))
    return (Ls[0] - Ls[1]) / (2.0 * h)


def stable_dt(nr, nth, rstar_min, rstar_max, a, M, m, s, n_steps) -> float:
    """Time step rule for the explicit scheme.

    For data smooth in r*, both Lax-Wendroff stages apply the angular terms of
    S, so a theta-mode with frequency w sees the explicit midpoint map, whose
    amplification obeys |G|^2 = 1 + (w dt)^4 / 4.  Limiting the growth of the
    stiffest mode to one e-fold over the run gives
    dt_theta = (8 / n_steps)^(1/4) / w_max, with
    w_max^2 = max eig(-Lth) * max(Delta/Sigma^2); the r* direction needs
    dt <= dr*/2 (b ~ 1).
    """
    A = angular_matrix(nth, m, s)
    lam = np.max(np.abs(np.linalg.eigvals(A)))
    # Delta/Sigma^2 grows with sin^2(theta): the two rows next to the equator bound it
    jm = nth // 2 - 1
    o = Oracle(nr, nth, rstar_min, rstar_max, a, M, m, s, 1.0, window=(0, nr, jm, 2))
    wmax = np.sqrt(lam * o.max_DoS2)
    dr = (rstar_max - rstar_min) / (nr - 1)
    return float(min(0.5 * dr, (8.0 / n_steps) ** 0.25 / wmax))
