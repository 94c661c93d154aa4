"""GPU parity of the fused Lax-Wendroff step (libteuk through its C ABI) against the oracle.

Bar: FP64 relative L2 error <= 1e-12 on the state and on the recorded
waveform; tile shapes bitwise identical; FP32 waveform within 1e-5 of the
FP64 oracle where the run is short enough for FP32 storage to allow it.
"""
import numpy as np
import pytest

from paper_0909_4039_amd import inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def rel(a, b):
    """The larger of the relative L2 error and the largest element error
    relative to the largest reference element (a local error shows in the
    second even on a large grid)."""
    a = np.asarray(a)
    b = np.asarray(b)
    l2 = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
    el = np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300) if b.size else 0.0
    return float(max(l2, el))


def run_gpu(case, phi, pi, n, prec=64, rows=None, dt=None, order=0, kb=None):
    import torch
    from paper_0909_4039_amd.solver import Solver
    s = Solver(case["nr"], case["nth"], case["rmin"], case["rmax"], case["a"], 1.0, case["m"], case["s"],
               dt if dt is not None else case["dt"], prec=prec)
    if rows:
        s.set_tiling(rows, order)
    if kb is not None:            # None: the library default (two steps per launch)
        s.set_blocking(kb)
    if case.get("amp", 0.0) != 0.0 or case.get("r0"):
        s.set_source(case.get("r0", 10.0), case.get("amp", 0.0))
    s.set_state(phi, pi)
    s.set_observer(case["robs"], n + 1)
    s.step(n)
    torch.cuda.synchronize()
    s.check_finite()
    out = (s.phi.cpu().numpy(), s.pi.cpu().numpy(), s.wave.cpu().numpy())
    s.close()
    return out


def run_oracle(oracle_mod, case, phi, pi, n, dt=None):
    o = oracle_mod.Oracle(case["nr"], case["nth"], case["rmin"], case["rmax"], case["a"], 1.0, case["m"],
                          case["s"], dt if dt is not None else case["dt"], r0=case.get("r0", 0.0),
                          amp=case.get("amp", 0.0), rstar_obs=case["robs"])
    return o.run(phi, pi, n)


SMALL = [
    dict(name="min_4x4", nr=4, nth=4, rmin=-10.0, rmax=10.0, a=0.0, m=2, s=-2, robs=1.0, n=7),
    dict(name="strip_edge_63x5", nr=63, nth=5, rmin=-20.0, rmax=40.0, a=0.9, m=1, s=-2, robs=19.99,
         r0=7.0, amp=1.0, n=40),
    dict(name="strip_64x16", nr=64, nth=16, rmin=-30.0, rmax=60.0, a=0.6, m=2, s=-2, robs=12.0, n=60),
    dict(name="ragged_125x33_s+2", nr=125, nth=33, rmin=-50.0, rmax=80.0, a=0.3, m=3, s=2, robs=40.0,
         r0=9.0, amp=0.7, n=50),
    dict(name="kerr_200x70_m-2", nr=200, nth=70, rmin=-60.0, rmax=140.0, a=0.99, m=-2, s=-2, robs=100.0,
         r0=8.0, amp=1.0, n=60),
    dict(name="odd_s_129x8", nr=129, nth=8, rmin=-40.0, rmax=90.0, a=0.5, m=0, s=-1, robs=0.0, n=50),
    dict(name="m8_300x37", nr=300, nth=37, rmin=-100.0, rmax=400.0, a=0.9, m=8, s=-2, robs=300.0,
         r0=11.0, amp=1.0, n=40),
    dict(name="s0_97x12", nr=97, nth=12, rmin=-40.0, rmax=80.0, a=0.7, m=1, s=0, robs=20.0, r0=8.0, amp=1.0,
         n=40),
    dict(name="s+1_111x10", nr=111, nth=10, rmin=-40.0, rmax=80.0, a=0.4, m=2, s=1, robs=30.0, n=40),
]


def _dt(oracle_mod, c, nsteps=None):
    return oracle_mod.stable_dt(c["nr"], c["nth"], c["rmin"], c["rmax"], c["a"], 1.0, c["m"], c["s"],
                                nsteps or 10000)


@pytest.mark.parametrize("kb", [1, 2])
@pytest.mark.parametrize("case", SMALL, ids=[c["name"] for c in SMALL])
def test_parity_random_data(oracle_mod, case, kb):
    case = dict(case, dt=_dt(oracle_mod, case))
    print(f"[gpu] parity {case['name']} n={case['n']} kb={kb}", flush=True)
    phi, pi = inputs.random_state(case["nr"], case["nth"], seed=sum(map(ord, case["name"])) % 1000)
    gp, gq, gw = run_gpu(case, phi, pi, case["n"], kb=kb)
    op, oq, ow = run_oracle(oracle_mod, case, phi, pi, case["n"])
    assert rel(gp, op) <= TOL64 and rel(gq, oq) <= TOL64, (rel(gp, op), rel(gq, oq))
    assert rel(gw, ow) <= TOL64, rel(gw, ow)
    # Dirichlet columns exactly zero
    assert not np.any(gp[:, 0]) and not np.any(gp[:, -1])


@pytest.mark.parametrize("prec", [64, 32])
def test_tiling_bitwise_invariant(oracle_mod, prec):
    # FP32 two-step launches on one wavefront carry each point's coefficients
    # from the first step to the second through a ring unrolled four times:
    # 20 steps at these chunk heights end the row loop at every phase of it
    case = dict(SMALL[4])
    case["dt"] = _dt(oracle_mod, case)
    print(f"[gpu] tiling invariance fp{prec}", flush=True)
    phi, pi = inputs.random_state(case["nr"], case["nth"], seed=3)
    for kb in (1, 2):
        ref = run_gpu(case, phi, pi, 20, prec=prec, rows=1, kb=kb)
        for rows, order in ((2, 0), (3, 1), (7, 0), (16, 1), (64, 0), (4096, 1), (1, 2), (5, 2), (64, 2), (4096, 2)):
            got = run_gpu(case, phi, pi, 20, prec=prec, rows=rows, order=order, kb=kb)
            for x, y in zip(got, ref):
                assert np.array_equal(x, y), (rows, order, kb)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("idx", [0, 1, 3, 4, 6])
def test_temporal_blocking_bitwise(oracle_mod, idx, prec):
    # two steps per launch reproduce single steps bit for bit (odd step
    # counts end with a single step; the recorder sees every state)
    case = dict(SMALL[idx])
    case["dt"] = _dt(oracle_mod, case)
    phi, pi = inputs.random_state(case["nr"], case["nth"], seed=40 + idx)
    for n, rows in ((21, None), (8, 5), (3, 64)):
        ref = run_gpu(case, phi, pi, n, prec=prec, rows=rows, kb=1)
        got = run_gpu(case, phi, pi, n, prec=prec, rows=rows, kb=2)
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), (case["name"], n, rows)
        # the fused pair on two wavefronts
        got = run_gpu(case, phi, pi, n, prec=prec, rows=rows or 16, order=2, kb=2)
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), (case["name"], n, rows, "pair")


@pytest.mark.parametrize("robs_index", [59, 60, 61, 119, 120])
def test_blocked_observer_on_strip_boundaries(oracle_mod, robs_index):
    # with two steps per launch the strips are 60 columns wide
    case = dict(name="obs2", nr=250, nth=12, rmin=0.0, rmax=249.0, a=0.6, m=2, s=-2, r0=20.0, amp=1.0)
    case["robs"] = robs_index + 0.61
    case["dt"] = _dt(oracle_mod, case)
    phi, pi = inputs.random_state(250, 12, seed=robs_index)
    gp, gq, gw = run_gpu(case, phi, pi, 14, kb=2)
    op, oq, ow = run_oracle(oracle_mod, case, phi, pi, 14)
    assert rel(gw, ow) <= TOL64 and rel(gp, op) <= TOL64


def test_schwarzschild_pulse_256x64(oracle_mod):
    # a = 0, s = -2, m = 2, sourceless; pulse at r* = 20 (width 4), seeded
    # amplitude; 2000 steps; waveform at r* = 100
    case = dict(name="c1", nr=256, nth=64, rmin=-50.0, rmax=150.0, a=0.0, m=2, s=-2, robs=100.0)
    n = 2000
    case["dt"] = _dt(oracle_mod, case, n)
    print(f"[gpu] schwarzschild 256x64 n={n} dt={case['dt']}", flush=True)
    phi, pi = inputs.pulse(256, 64, -50.0, 150.0, 2, 20.0, 4.0, inputs.seeded_amplitude(1))
    gp, gq, gw = run_gpu(case, phi, pi, n)
    op, oq, ow = run_oracle(oracle_mod, case, phi, pi, n)
    assert rel(gp, op) <= TOL64 and rel(gq, oq) <= TOL64, (rel(gp, op), rel(gq, oq))
    assert rel(gw, ow) <= TOL64, rel(gw, ow)


def test_kerr_source_full_grid_8192x256(oracle_mod):
    # full-size Kerr a = 0.9 grid with the source on, smooth seeded data, 12 steps
    case = dict(name="c2", nr=8192, nth=256, rmin=-100.0, rmax=400.0, a=0.9, m=2, s=-2, robs=300.0,
                r0=10.0, amp=1.0)
    n = 12
    case["dt"] = _dt(oracle_mod, case, 50000)
    print(f"[gpu] kerr 8192x256 n={n}", flush=True)
    phi, pi = inputs.smooth_random_state(8192, 256, -100.0, 400.0, seed=21)
    gp, gq, gw = run_gpu(case, phi, pi, n)
    op, oq, ow = run_oracle(oracle_mod, case, phi, pi, n)
    assert rel(gp, op) <= TOL64 and rel(gq, oq) <= TOL64, (rel(gp, op), rel(gq, oq))
    assert rel(gw, ow) <= TOL64, rel(gw, ow)


def test_large_grid_sampled_windows(oracle_mod):
    # 32768 x 1024 (a = 0.99, source at r0 = 8) in the benchmark's launch
    # configuration; the oracle evaluates windows and the domain of dependence
    # of each is compared point by point
    nr, nth, rmin, rmax, a, m = 32768, 1024, -100.0, 400.0, 0.99, 2
    n = 6
    dt = _dt(oracle_mod, dict(nr=nr, nth=nth, rmin=rmin, rmax=rmax, a=a, m=m, s=-2), 100000)
    case = dict(name="c5", nr=nr, nth=nth, rmin=rmin, rmax=rmax, a=a, m=m, s=-2, robs=100.0, r0=8.0,
                amp=1.0, dt=dt)
    print(f"[gpu] large 32768x1024 n={n}", flush=True)
    phi, pi = inputs.smooth_random_state(nr, nth, rmin, rmax, seed=55)
    gp, gq, gw = run_gpu(case, phi, pi, n)
    checked = 0
    for (i0, ni, j0, nj) in [(0, 90, 0, 40), (32768 - 90, 90, 1024 - 40, 40), (6500, 200, 480, 64),
                             (199 * 62 - 20, 80, 300, 50), (15000, 128, 1000, 24)]:
        o = oracle_mod.Oracle(nr, nth, rmin, rmax, a, 1.0, m, -2, dt, r0=8.0, amp=1.0, rstar_obs=100.0,
                              window=(i0, ni, j0, nj))
        sl = (slice(j0, j0 + nj), slice(i0, i0 + ni))
        op, oq, _ = o.run(phi[sl], pi[sl], n, record=False)
        ok = np.isfinite(op)
        assert ok.sum() > 0.3 * ok.size
        assert rel(gp[sl][ok], op[ok]) <= TOL64 and rel(gq[sl][ok], oq[ok]) <= TOL64
        checked += int(ok.sum())
    assert checked > 20000


@pytest.mark.parametrize("robs_index", [61, 62, 123, 124])
def test_observer_on_strip_boundaries(oracle_mod, robs_index):
    # the recorder's column pair may straddle the 62-column strips
    case = dict(name="obs", nr=250, nth=12, rmin=0.0, rmax=249.0, a=0.6, m=2, s=-2, r0=20.0, amp=1.0)
    case["robs"] = robs_index + 0.37
    case["dt"] = _dt(oracle_mod, case)
    phi, pi = inputs.random_state(250, 12, seed=robs_index)
    gp, gq, gw = run_gpu(case, phi, pi, 15, kb=1)
    op, oq, ow = run_oracle(oracle_mod, case, phi, pi, 15)
    assert rel(gw, ow) <= TOL64


def test_zero_steps_and_resume(oracle_mod):
    import torch
    from paper_0909_4039_amd.solver import Solver
    case = dict(SMALL[2])
    dt = _dt(oracle_mod, case)
    phi, pi = inputs.random_state(case["nr"], case["nth"], seed=8)
    s = Solver(case["nr"], case["nth"], case["rmin"], case["rmax"], case["a"], 1.0, case["m"], case["s"], dt)
    s.set_source(10.0, 1.0)
    s.set_state(phi, pi)
    w = s.set_observer(case["robs"], 1)
    s.step(0)
    torch.cuda.synchronize()
    o = oracle_mod.Oracle(case["nr"], case["nth"], case["rmin"], case["rmax"], case["a"], 1.0, case["m"],
                          case["s"], dt, r0=10.0, amp=1.0, rstar_obs=case["robs"])
    assert rel(w.cpu().numpy()[0], o.extract(phi)) <= 1e-15
    s.clear_observer()
    # 2n in one go == n, save, restore into a fresh solver, n
    s.step(30)
    t_mid, n_mid = s.get_time()
    saved = (s.phi.clone(), s.pi.clone())
    s.step(30)
    full = s.phi.cpu().numpy()
    s2 = Solver(case["nr"], case["nth"], case["rmin"], case["rmax"], case["a"], 1.0, case["m"], case["s"], dt)
    s2.set_source(10.0, 1.0)
    s2.set_state(*saved)
    s2.set_time(t_mid, n_mid)
    s2.step(30)
    torch.cuda.synchronize()
    assert np.array_equal(s2.phi.cpu().numpy(), full)
    assert s2.get_time()[1] == 60
    s.close()
    s2.close()


def test_nonfinite_is_reported():
    import torch
    from paper_0909_4039_amd import TeukError
    from paper_0909_4039_amd.solver import Solver
    s = Solver(64, 8, -20.0, 40.0, 0.5, 1.0, 2, -2, 0.01)
    phi = np.zeros((8, 64), complex)
    phi[3, 20] = np.nan
    s.set_state(phi, np.zeros_like(phi))
    s.step(2)
    torch.cuda.synchronize()
    with pytest.raises(TeukError) as e:
        s.check_finite()
    assert e.value.code == -4
    assert s.status() == -4
    s.close()


@pytest.mark.parametrize("prec", [32, 48], ids=["fp32", "fp32s"])
def test_fp32_waveform_error(oracle_mod, prec):
    # FP32 storage (with FP32 or FP64 arithmetic) vs the FP64 oracle on the
    # Schwarzschild pulse
    case = dict(name="c1", nr=256, nth=64, rmin=-50.0, rmax=150.0, a=0.0, m=2, s=-2, robs=100.0)
    n = 2000
    case["dt"] = _dt(oracle_mod, case, n)
    phi, pi = inputs.pulse(256, 64, -50.0, 150.0, 2, 20.0, 4.0, inputs.seeded_amplitude(1))
    # read further in so that the pulse reaches the observer within the run
    case["robs"] = 30.0
    gp, gq, gw = run_gpu(case, phi, pi, n, prec=prec)
    op, oq, ow = run_oracle(oracle_mod, case, phi, pi, n)
    err_w = rel(gw, ow)
    err_s = rel(gp, op)
    print(f"[gpu] prec {prec} waveform rel err {err_w:.3e}, state {err_s:.3e}", flush=True)
    assert err_w <= 1e-5, err_w


def test_autotune_keeps_state_and_results(oracle_mod):
    import torch
    from paper_0909_4039_amd.solver import Solver
    case = dict(SMALL[4])
    dt = _dt(oracle_mod, case)
    phi, pi = inputs.random_state(case["nr"], case["nth"], seed=77)
    n = 25
    ref = run_gpu(dict(case, dt=dt), phi, pi, n)
    s = Solver(case["nr"], case["nth"], case["rmin"], case["rmax"], case["a"], 1.0, case["m"], case["s"], dt)
    s.set_source(case["r0"], case["amp"])
    s.set_state(phi, pi)
    s.set_observer(case["robs"], n + 1)
    s.step(5)
    torch.cuda.synchronize()
    before = (s.phi.clone(), s.pi.clone(), s.wave.clone(), s.get_time())
    rows, kb = s.autotune(3)
    print(f"[gpu] autotune picked rows={rows} kb={kb}", flush=True)
    torch.cuda.synchronize()
    assert torch.equal(s.phi, before[0]) and torch.equal(s.pi, before[1]) and torch.equal(s.wave, before[2])
    assert s.get_time() == before[3]
    assert s.get_tiling()[0] == rows and s.get_blocking() == kb
    s.step(n - 5)
    torch.cuda.synchronize()
    got = (s.phi.cpu().numpy(), s.pi.cpu().numpy(), s.wave.cpu().numpy())
    for x, y in zip(got, ref):
        assert np.array_equal(x, y)
    s.close()


@pytest.mark.parametrize("prec", [32, 48], ids=["fp32", "fp32s"])
def test_fp32_waveform_error_kerr_8192x256(oracle_mod, prec):
    # FP32 storage and arithmetic on the full Kerr a = 0.9 source grid against
    # the FP64 oracle: smooth seeded data, 300 steps, waveform at r* = 20
    nr, nth, rmin, rmax, a, m = 8192, 256, -100.0, 400.0, 0.9, 2
    case = dict(name="c2_fp32", nr=nr, nth=nth, rmin=rmin, rmax=rmax, a=a, m=m, s=-2, robs=20.0, r0=10.0, amp=1.0)
    case["dt"] = _dt(oracle_mod, case, 50000)
    n = 300
    phi, pi = inputs.smooth_random_state(nr, nth, rmin, rmax, seed=23)
    print(f"[gpu] fp32 8192x256 n={n}", flush=True)
    gp, gq, gw = run_gpu(case, phi, pi, n, prec=prec)
    op, oq, ow = run_oracle(oracle_mod, case, phi, pi, n)
    err_w = rel(gw, ow)
    print(f"[gpu] prec {prec} 8192x256 waveform rel err {err_w:.3e}, state {rel(gp, op):.3e}", flush=True)
    assert err_w <= 1e-5, err_w


def _random_cases(k=16, seed=2027):
    """Seeded random grids, spins, modes, sources, tilings and blocking, all
    within the documented limits."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(k):
        rmin, rmax = float(rng.uniform(-80.0, -10.0)), float(rng.uniform(30.0, 300.0))
        case = dict(name=f"rand{i}", nr=int(rng.integers(4, 400)), nth=int(rng.integers(4, 80)), rmin=rmin,
                    rmax=rmax, a=float(rng.choice([0.0, rng.uniform(0.0, 0.99)])), m=int(rng.integers(-4, 7)),
                    s=int(rng.integers(-2, 3)), robs=rmin + (rmax - rmin) * float(rng.uniform(0.05, 0.95)),
                    n=int(rng.integers(5, 31)), rows=int(rng.choice([1, 2, 3, 5, 8, 13, 32, 64])),
                    kb=int(rng.integers(1, 3)))
        if rng.integers(0, 2):
            case.update(r0=float(rng.uniform(6.0, 12.0)), amp=float(rng.uniform(0.5, 2.0)))
        case["order"] = 2 * (i % 2)   # every other case: a fused pair on two wavefronts
        out.append(case)
    return out


@pytest.mark.parametrize("case", _random_cases(), ids=lambda c: c["name"])
def test_parity_seeded_random_configurations(oracle_mod, case):
    case = dict(case, dt=_dt(oracle_mod, case, 1000))
    print(f"[gpu] random parity {case}", flush=True)
    phi, pi = inputs.random_state(case["nr"], case["nth"], seed=int(case["name"][4:]) + 100)
    gp, gq, gw = run_gpu(case, phi, pi, case["n"], rows=case["rows"], kb=case["kb"], order=case["order"])
    op, oq, ow = run_oracle(oracle_mod, case, phi, pi, case["n"])
    assert rel(gp, op) <= TOL64 and rel(gq, oq) <= TOL64, (rel(gp, op), rel(gq, oq))
    assert rel(gw, ow) <= TOL64, rel(gw, ow)


def test_fp32_storage_fp64_arithmetic_tilings(oracle_mod):
    # FP32 storage with FP64 arithmetic: bitwise equal across tilings and
    # launch forms at fixed steps per launch; one or two steps per launch
    # differ only by where the state is rounded to FP32
    case = dict(SMALL[4])
    case["dt"] = _dt(oracle_mod, case)
    phi, pi = inputs.random_state(case["nr"], case["nth"], seed=48)
    for kb in (1, 2):
        ref = run_gpu(case, phi, pi, 20, prec=48, rows=1, kb=kb)
        for rows, order in ((3, 1), (16, 0), (64, 0)) + (((5, 2), (4096, 2)) if kb == 2 else ()):
            got = run_gpu(case, phi, pi, 20, prec=48, rows=rows, order=order, kb=kb)
            for x, y in zip(got, ref):
                assert np.array_equal(x, y), (rows, order, kb)
        if kb == 1:
            one = ref
    for x, y in zip(ref, one):
        assert rel(x, y) <= 1e-6
    op, oq, ow = run_oracle(oracle_mod, case, phi, pi, 20)
    assert rel(ref[2], ow) <= 1e-6
