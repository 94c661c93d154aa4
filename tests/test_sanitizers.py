"""Host-side memory and undefined-behaviour checks (AddressSanitizer and
UBSan, host code only; no GPU code is instrumented):

- libteuk's host code (geometry tables, argument checks, create/destroy and
  their failure paths), built with the sanitizers on the host side of hipcc
  and driven by a small C program;
- the oracle, built with the sanitizers and run from Python with the
  sanitizer runtime preloaded, over forward, reverse, moving-source and
  window runs.

A report from either sanitizer fails the test.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0909_4039_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang"
HIPCC = "/opt/rocm/bin/hipcc"
REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")

DRIVER = r"""
#include <stdio.h>
#include "teuk.h"
int main(void) {
    teuk_grid g = {300, 37, -100.0, 400.0}, tiny = {5, 4, -10.0, 10.0}, bad = {3, 4, 1.0, 0.0};
    double dt = 0.0;
    int ok = 1;
    ok &= teuk_suggest_dt(&g, 0.9, 1.0, 2, -2, 1000, &dt) == TEUK_OK && dt > 0.0;
    ok &= teuk_suggest_dt(&tiny, 0.99, 1.0, 7, 2, 10, &dt) == TEUK_OK;
    ok &= teuk_suggest_dt(&bad, 0.5, 1.0, 2, -2, 10, &dt) == TEUK_EINVAL;
    ok &= teuk_rstar_of_r(10.0, 0.9, 1.0) > 10.0;
    for (int s = -2; s <= 2; ++s) {
        teuk_ctx* c = NULL;
        int rc = teuk_create(&g, 0.9, 1.0, 3, s, 0.01, 64, NULL, &c);
        /* without a GPU the tables are built and the device allocation fails */
        ok &= (rc == TEUK_OK && c) || (rc == TEUK_EDEVICE && !c);
        if (c) teuk_destroy(c);
    }
    teuk_ctx* c = NULL;
    ok &= teuk_create(&g, 1.5, 1.0, 2, -2, 0.01, 64, NULL, &c) == TEUK_EINVAL && !c;
    ok &= teuk_create(&g, 0.5, 1.0, 2, 3, 0.01, 64, NULL, &c) == TEUK_EINVAL;
    ok &= teuk_create(&g, 0.5, 1.0, 2, -2, 0.01, 16, NULL, &c) == TEUK_EINVAL;
    teuk_desc d[2];
    for (int i = 0; i < 2; ++i) {
        d[i].grid = g; d[i].a = 0.5; d[i].M = 1.0; d[i].m = 2; d[i].s = -2; d[i].dt = 0.01;
        d[i].r0 = 8.0; d[i].amp = 1.0; d[i].sigma_r_cells = 2.0; d[i].sigma_th_cells = 2.0; d[i].rstar_obs = 100.0;
    }
    teuk_batch* b = NULL;
    int rc = teuk_batch_create(2, d, 10, NULL, &b);
    ok &= (rc == TEUK_OK && b) || rc == TEUK_EDEVICE || rc == TEUK_EINVAL;
    if (b) teuk_batch_destroy(b);
    printf("%s\n", ok ? "driver ok" : "driver FAILED");
    return ok ? 0 : 1;
}
"""


def _need(*tools):
    for t in tools:
        if not os.path.exists(t) and shutil.which(t) is None:
            pytest.skip(f"{t} not found")


def _clean(r):
    out = r.stdout + r.stderr
    assert not any(s in out for s in REPORTS), out[-4000:]
    return out


def test_host_library_under_asan_ubsan(tmp_path):
    _need(HIPCC, CLANG)
    lib = tmp_path / "libteuk_san.so"
    srcs = [os.path.join(CSRC, f) for f in ("teuk_api.cpp", "teuk_geom.cpp", "teuk_batch.cpp", "teuk_kernels.hip",
                                             "teuk_adjoint.hip", "teuk_watch.hip")]
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=off",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", *srcs, "-o", str(lib)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    drv_c = tmp_path / "drv.c"
    drv_c.write_text(DRIVER)
    drv = tmp_path / "drv"
    r = subprocess.run([CLANG, "-g", "-fsanitize=address,undefined", "-I", os.path.join(ROOT, "include"),
                        str(drv_c), f"-L{tmp_path}", "-lteuk_san", f"-Wl,-rpath,{tmp_path}", "-o", str(drv)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([str(drv)], capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"))
    out = _clean(r)
    assert r.returncode == 0 and "driver ok" in out, out[-3000:]


ORACLE_RUN = r"""
import sys
sys.path.insert(0, {root!r})
import numpy as np
import oracle
oracle._LIB = {lib!r}
from paper_0909_4039_amd import inputs
for (nr, nth, a, m, s) in [(40, 9, 0.9, 2, -2), (33, 8, 0.6, 1, -1), (25, 5, 0.3, 3, 2), (20, 4, 0.0, 0, 0)]:
    dt = oracle.stable_dt(nr, nth, -30.0, 50.0, a, 1.0, m, s, 100)
    phi, pi = inputs.random_state(nr, nth, 1)
    o = oracle.Oracle(nr, nth, -30.0, 50.0, a, 1.0, m, s, dt, r0=8.0, amp=1.0, rstar_obs=10.0)
    p, q, w = o.run(phi, pi, 7)
    g = np.random.default_rng(2).standard_normal(w.shape) + 0j
    o.adjoint_run(g, 7)
    o.set_trajectory(inputs.inspiral_trajectory(8.0, a, 1.0, 0.05, dt, 7))
    o.run(phi, pi, 7)
    o.adjoint_run_moving(g, 7)
    o.set_trajectory(None)
    ni = min(15, nr - 5)
    ow = oracle.Oracle(nr, nth, -30.0, 50.0, a, 1.0, m, s, dt, r0=8.0, amp=1.0, rstar_obs=10.0,
                       window=(5, ni, 1, nth - 2))
    ow.run(phi[1:nth - 1, 5:5 + ni], pi[1:nth - 1, 5:5 + ni], 2, record=False)
    oracle.angular_matrix(nth, m, s)
    oracle.coeffs(0.5, 1.0, a, 1.0, m, s)
print("oracle ok")
"""


def test_oracle_under_asan_ubsan(tmp_path):
    _need(CLANG)
    rt = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    if not os.path.exists(rt):
        pytest.skip("no clang ASan runtime")
    lib = tmp_path / "liboracle_san.so"
    r = subprocess.run([CLANG, "-O1", "-g", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                        "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                        os.path.join(ROOT, "oracle", "teuk_oracle.c"), "-o", str(lib), "-lm"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    script = tmp_path / "run.py"
    script.write_text(ORACLE_RUN.format(root=ROOT, lib=str(lib)))
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, timeout=300, env=env)
    out = _clean(r)
    assert r.returncode == 0 and "oracle ok" in out, out[-3000:]
