"""Build libteuk.so in-tree with hipcc for gfx950, and the C example that
drives it through the C ABI alone."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libteuk.so")
SOURCES = ["teuk_api.cpp", "teuk_geom.cpp", "teuk_batch.cpp", "teuk_kernels.hip", "teuk_adjoint.hip",
           "teuk_watch.hip", "teuk_probe.hip", "teuk_noalloc.hip"]
ARCH = os.environ.get("TEUK_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit multiply-add contraction: the kernels write each FMA out
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-function", "-pthread",
]


def build(verbose: bool = False, extra_flags=None) -> str:
    """Compile every source into LIB; always recompiles."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *FLAGS, *(extra_flags or []), *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libteuk.so")
    if verbose and r.stderr:
        sys.stderr.write("\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l) + "\n")
    os.replace(tmp, LIB)
    return LIB




ROOT = os.path.dirname(HERE)
EXAMPLE_SRC = os.path.join(ROOT, "examples", "teuk_run.c")
EXAMPLE_BIN = os.path.join(ROOT, "examples", "teuk_run")


def build_example(verbose: bool = False, out: str = EXAMPLE_BIN) -> str:
    """Compile examples/teuk_run.c (plain C99) against LIB and the HIP runtime
    into out; always recompiles.  The binary finds libteuk.so next to the
    package through its run path."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           f"-I{rocm}/include", f"-I{os.path.join(ROOT, 'include')}", EXAMPLE_SRC,
           f"-L{HERE}", "-lteuk", f"-L{rocm}/lib", "-lamdhip64",
           f"-Wl,-rpath,{HERE}", "-Wl,-rpath,$ORIGIN/../paper_0909_4039_amd", f"-Wl,-rpath,{rocm}/lib",
           "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("gcc failed building examples/teuk_run")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_example(verbose=True))
