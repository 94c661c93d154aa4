"""MI355X-native Teukolsky time stepper (paper: Khanna & McKennon, Cell/CUDA EMRI code).

The compute path is libteuk.so (HIP kernels for gfx950 behind a C ABI,
include/teuk.h); ``Solver`` is its thin PyTorch/ctypes binding.  The
``inputs`` and ``workloads`` modules only describe synthetic inputs.
"""
from ._lib import FP32, FP64, TeukError  # noqa: F401


def __getattr__(name):
    if name in ("Solver", "suggest_dt", "rstar_of_r", "delta_of_rstar"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
