"""CPU-side checks of libteuk: the C ABI loads, exports what include/teuk.h
declares, validates arguments, and its host geometry agrees with the oracle."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "teuk.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(teuk_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_0909_4039_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libteuk.so is not built (run __graft_entry__.build())")
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n


def test_bindings_cover_header():
    from paper_0909_4039_amd import _lib
    missing = [n for n in declared_functions() if n not in _lib._SIGS]
    assert not missing, missing


def test_strerror(L):
    from paper_0909_4039_amd import _lib
    for code in (0, -1, -2, -3, -4, -5):
        assert L.teuk_strerror(code).decode().startswith("TEUK_")
    assert b"unknown" in L.teuk_strerror(-99)


def test_create_rejects_bad_arguments(L):
    from paper_0909_4039_amd._lib import TeukGrid, EINVAL
    ctx = ctypes.c_void_p()
    good = TeukGrid(64, 16, -50.0, 150.0)
    bad_grids = [TeukGrid(3, 16, -50.0, 150.0), TeukGrid(64, 3, -50.0, 150.0), TeukGrid(64, 16, 10.0, 10.0)]
    for g in bad_grids:
        assert L.teuk_create(ctypes.byref(g), 0.5, 1.0, 2, -2, 0.01, 64, None, ctypes.byref(ctx)) == EINVAL
        assert not ctx.value
    cases = [(1.0, 1.0, 2, -2, 0.01, 64),    # a = M
             (-0.1, 1.0, 2, -2, 0.01, 64),   # a < 0
             (0.5, 0.0, 2, -2, 0.01, 64),    # M = 0
             (0.5, 1.0, 2, -3, 0.01, 64),    # |s| > 2
             (0.5, 1.0, 2, -2, 0.0, 64),     # dt = 0
             (0.5, 1.0, 2, -2, float("nan"), 64),
             (0.5, 1.0, 2, -2, 0.01, 16)]    # precision
    for a, M, m, s, dt, prec in cases:
        assert L.teuk_create(ctypes.byref(good), a, M, m, s, dt, prec, None, ctypes.byref(ctx)) == EINVAL
    assert L.teuk_create(None, 0.5, 1.0, 2, -2, 0.01, 64, None, ctypes.byref(ctx)) == EINVAL
    assert L.teuk_create(ctypes.byref(good), 0.5, 1.0, 2, -2, 0.01, 64, None, None) == EINVAL


def test_null_context_calls(L):
    from paper_0909_4039_amd._lib import EINVAL
    assert L.teuk_step(None, 1) == EINVAL
    assert L.teuk_destroy(None) == EINVAL
    assert L.teuk_status(None) == EINVAL
    assert L.teuk_current(None) == EINVAL
    assert L.teuk_extract(None, 1.0, None) == EINVAL


@pytest.mark.parametrize("a", [0.0, 0.3, 0.9, 0.99])
def test_host_geometry_matches_oracle(L, oracle_mod, a):
    # same Eq. (2), independent code: bisection (oracle) vs Newton (library)
    for rs in (-100.0, -10.0, 0.0, 12.5, 100.0, 400.0):
        d1 = L.teuk_delta_of_rstar(rs, a, 1.0)
        d2 = oracle_mod.delta_of_rstar(rs, a, 1.0)
        assert d1 == pytest.approx(d2, rel=1e-13)
    for r in (2.5, 6.0, 10.0, 80.0):
        assert L.teuk_rstar_of_r(r, a, 1.0) == pytest.approx(oracle_mod.rstar_of_r(r, a, 1.0), rel=1e-14, abs=1e-13)


@pytest.mark.parametrize("cfg", [(256, 64, -50.0, 150.0, 0.0, 2, 2000),
                                 (8192, 256, -100.0, 400.0, 0.9, 2, 50000),
                                 (512, 128, -100.0, 400.0, 0.6, 3, 1000)])
def test_suggested_dt_is_conservative(L, oracle_mod, cfg):
    from paper_0909_4039_amd.solver import suggest_dt
    nr, nth, r0, r1, a, m, n = cfg
    mine = suggest_dt(nr, nth, r0, r1, a, 1.0, m, -2, n)
    ref = oracle_mod.stable_dt(nr, nth, r0, r1, a, 1.0, m, -2, n)
    assert 0.5 * ref < mine <= ref * (1 + 1e-12)


def test_header_is_plain_c(tmp_path):
    # include/teuk.h is the boundary: it must compile as C99 on its own and
    # declare every entry point with a C prototype
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    names = declared_functions()
    src = tmp_path / "uses_header.c"
    src.write_text("#include \"teuk.h\"\n"
                   "typedef void (*entry)(void);\n"
                   "entry entry_points[] = {\n" + ",\n".join(f"    (entry)&{n}" for n in names) + "\n};\n"
                   "int main(void) { return entry_points[0] == 0; }\n")
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only",
                        "-I", os.path.dirname(HEADER), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_header_compiles_as_cpp(tmp_path):
    # the same header from C++: extern "C" linkage, no C-only constructs
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    src = tmp_path / "uses_header.cpp"
    src.write_text("#include \"teuk.h\"\n"
                   "static_assert(sizeof(teuk_grid) == 32, \"teuk_grid layout\");\n"
                   "int main() { return teuk_strerror(TEUK_OK) == nullptr; }\n")
    r = subprocess.run([gxx, "-std=c++17", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only",
                        "-I", os.path.dirname(HEADER), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_constants_match_header():
    from paper_0909_4039_amd import _lib
    src = open(HEADER).read()
    defs = {k: int(v) for k, v in re.findall(r"#define\s+(TEUK_\w+)\s+\(?(-?\d+)\)?", src)}
    want = {"TEUK_OK": _lib.OK, "TEUK_EINVAL": _lib.EINVAL, "TEUK_ESTATE": _lib.ESTATE,
            "TEUK_EDEVICE": _lib.EDEVICE, "TEUK_EUNSTABLE": _lib.EUNSTABLE, "TEUK_ENOTSUP": _lib.ENOTSUP,
            "TEUK_FP64": _lib.FP64, "TEUK_FP32": _lib.FP32, "TEUK_PARAM_A": _lib.PARAM_A,
            "TEUK_PARAM_M": _lib.PARAM_M, "TEUK_PARAM_R0": _lib.PARAM_R0, "TEUK_PARAM_AMP": _lib.PARAM_AMP}
    for k, v in want.items():
        assert defs.get(k) == v, (k, defs.get(k), v)


def test_null_handles_on_later_entry_points(L):
    from paper_0909_4039_amd._lib import EINVAL
    d = ctypes.c_double()
    i = ctypes.c_int32()
    assert L.teuk_set_adjoint_tiling(None, 0, 1) == EINVAL
    assert L.teuk_get_adjoint_tiling(None, ctypes.byref(i), ctypes.byref(i)) == EINVAL
    assert L.teuk_adjoint_autotune(None, 1, None, None) == EINVAL
    assert L.teuk_adjoint_moving(None, 1.0, None, 1, None, 0, None, None, None, None) == EINVAL
    assert L.teuk_param_gradient_workspace_bytes(None, 1, 0) == EINVAL
    assert L.teuk_param_gradient(None, 0, 1e-6, 1.0, None, 1, 0.0, None, None, 0, None, 0, ctypes.byref(d),
                                 None, None) == EINVAL
    assert L.teuk_set_trajectory(None, None, 0) == EINVAL
    assert L.teuk_batch_set_trajectory(None, 0, None, 0) == EINVAL
    assert L.teuk_set_watchdog(None, 10, 1.0) == EINVAL
    assert L.teuk_batch_set_watchdog(None, 1, 1.0) == EINVAL
    assert L.teuk_batch_step(None, 1) == EINVAL


def test_c_example_builds_and_prints_usage(tmp_path):
    # examples/teuk_run.c is plain C99 over the header and the library; with
    # no arguments it prints its usage before any HIP call
    from paper_0909_4039_amd import build as B
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = B.build_example(out=str(tmp_path / "teuk_run"))
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "usage:" in r.stderr
