"""GPU reverse sweep (teuk_adjoint through the C ABI) against the oracle's
hand-written reverse sweep, the adjoint identity, central finite
differences of GPU forward runs, and the autograd Function.

Bars: FP64 relative L2 <= 1e-12 for dL/du^0 against the oracle; source
gradients within 1e-11 relative; bitwise dL/du^0 across tilings and steps
per launch; finite differences (h = 1e-6) within 1e-5 relative.
"""
import numpy as np
import pytest

from paper_0909_4039_amd import inputs, workloads

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


def rel_scalar(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def make_solver(case, dt, kb=None, rows=None, order=0):
    from paper_0909_4039_amd.solver import Solver
    s = Solver(case["nr"], case["nth"], case["rmin"], case["rmax"], case["a"], 1.0, case["m"], case["s"], dt)
    if kb is not None:
        s.set_blocking(kb)
    if rows:
        s.set_tiling(rows, order)
    if kb is not None or rows:
        # the reverse sweep's own tiling: these rows (0 follows the forward's)
        s.set_adjoint_tiling(rows or 0, kb or 1)
    if case.get("r0"):
        s.set_source(case["r0"], case.get("amp", 0.0))
    return s


def seeded_g(n, nth, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n + 1, nth)) + 1j * rng.standard_normal((n + 1, nth))


def gpu_adjoint(case, dt, g, n, kb=None, rows=None, order=0, t_start=0.0):
    s = make_solver(case, dt, kb, rows, order)
    dphi, dpi, dr0, damp = s.adjoint(g, n, case["robs"], t_start)
    out = (dphi.cpu().numpy(), dpi.cpu().numpy(), dr0, damp)
    s.close()
    return out


def oracle_adjoint(oracle_mod, case, dt, g, n, t_start=0.0):
    o = oracle_mod.Oracle(case["nr"], case["nth"], case["rmin"], case["rmax"], case["a"], 1.0, case["m"],
                          case["s"], dt, r0=case.get("r0", 0.0), amp=case.get("amp", 0.0),
                          rstar_obs=case["robs"])
    return o.adjoint_run(g, n, t_start)


CASES = [
    dict(name="min_4x4", nr=4, nth=4, rmin=-10.0, rmax=10.0, a=0.0, m=2, s=-2, robs=1.0, n=7),
    dict(name="strip_edge_63x5", nr=63, nth=5, rmin=-20.0, rmax=40.0, a=0.9, m=1, s=-2, robs=19.99,
         r0=7.0, amp=1.0, n=40),
    dict(name="ragged_125x33_s+2", nr=125, nth=33, rmin=-50.0, rmax=80.0, a=0.3, m=3, s=2, robs=40.0,
         r0=9.0, amp=0.7, n=50),
    dict(name="kerr_200x70_m-2", nr=200, nth=70, rmin=-60.0, rmax=140.0, a=0.99, m=-2, s=-2, robs=10.0,
         r0=8.0, amp=1.0, n=60),
    dict(name="odd_s_129x8", nr=129, nth=8, rmin=-40.0, rmax=90.0, a=0.5, m=0, s=-1, robs=0.0, n=50),
    dict(name="src_reach_150x24", nr=150, nth=24, rmin=-20.0, rmax=55.0, a=0.6, m=2, s=-2, robs=14.0,
         r0=10.0, amp=0.0, n=90),
]


def _dt(oracle_mod, c, nsteps=10000):
    return oracle_mod.stable_dt(c["nr"], c["nth"], c["rmin"], c["rmax"], c["a"], 1.0, c["m"], c["s"], nsteps)


@pytest.mark.parametrize("kb", [1, 2])
@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_adjoint_parity(oracle_mod, case, kb):
    dt = _dt(oracle_mod, case)
    n = case["n"]
    print(f"[gpu] adjoint parity {case['name']} n={n} kb={kb}", flush=True)
    g = seeded_g(n, case["nth"], seed=sum(map(ord, case["name"])) % 1000)
    t0 = 0.37
    gp, gq, gr0, gamp = gpu_adjoint(case, dt, g, n, kb=kb, t_start=t0)
    op, oq, or0, oamp = oracle_adjoint(oracle_mod, case, dt, g, n, t_start=t0)
    assert rel(gp, op) <= TOL64 and rel(gq, oq) <= TOL64, (rel(gp, op), rel(gq, oq))
    if case.get("r0"):
        # every sourced case puts the source within reach of the observer
        assert oamp != 0.0
        assert rel_scalar(gamp, oamp) <= 1e-11, (gamp, oamp)
        if case.get("amp", 0.0) != 0.0:
            assert rel_scalar(gr0, or0) <= 1e-11, (gr0, or0)
        else:
            assert gr0 == 0.0
    else:
        assert gr0 == 0.0 and gamp == 0.0


def test_adjoint_zero_steps(oracle_mod):
    case = CASES[3]
    dt = _dt(oracle_mod, case)
    g = seeded_g(0, case["nth"], seed=5)
    gp, gq, gr0, gamp = gpu_adjoint(case, dt, g, 0)
    op, oq, _, _ = oracle_adjoint(oracle_mod, case, dt, g, 0)
    assert np.array_equal(gp, op) and not np.any(gq)
    assert gr0 == 0.0 and gamp == 0.0


def test_adjoint_bitwise_across_tilings(oracle_mod):
    case = CASES[3]
    dt = _dt(oracle_mod, case)
    n = 33
    g = seeded_g(n, case["nth"], seed=9)
    print("[gpu] adjoint tiling invariance", flush=True)
    ref = gpu_adjoint(case, dt, g, n, kb=1, rows=1)
    for kb, rows, order in ((1, 7, 0), (2, 5, 0), (2, 64, 0), (2, 4096, 0), (1, 16, 0), (2, None, 0)):
        got = gpu_adjoint(case, dt, g, n, kb=kb, rows=rows, order=order)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (kb, rows)
        # the source-gradient sums group their terms by tile: equal to rounding
        assert rel_scalar(got[2], ref[2]) <= 1e-13 and rel_scalar(got[3], ref[3]) <= 1e-13


def test_adjoint_tiling_setters_and_autotune(oracle_mod):
    import torch
    case = CASES[3]
    dt = _dt(oracle_mod, case)
    n = 33
    g = seeded_g(n, case["nth"], seed=9)
    ref = gpu_adjoint(case, dt, g, n, kb=1, rows=1)
    s = make_solver(case, dt)
    assert s.get_adjoint_tiling() == (s.get_tiling()[0], 1)     # defaults: forward rows, one step
    s.set_tiling(12)
    assert s.get_adjoint_tiling() == (12, 1)
    ws0 = s.adjoint_workspace_bytes()
    s.set_adjoint_tiling(3, 2)
    assert s.get_adjoint_tiling() == (3, 2) and s.adjoint_workspace_bytes() == ws0
    from paper_0909_4039_amd import TeukError
    for bad in ((-1, 1), (4097, 1), (8, 0), (8, 3)):
        with pytest.raises(TeukError):
            s.set_adjoint_tiling(*bad)
    assert s.get_adjoint_tiling() == (3, 2)
    # the trials read the current pair and write the other: the state stays
    phi, pi = inputs.random_state(case["nr"], case["nth"], seed=4)
    s.set_state(phi, pi)
    s.step(3)
    torch.cuda.synchronize()
    keep = (s.phi.clone(), s.pi.clone(), s.get_time())
    rows, kb = s.adjoint_autotune(2)
    print(f"[gpu] adjoint autotune picked rows={rows} kb={kb}", flush=True)
    assert s.get_adjoint_tiling() == (rows, kb) and 1 <= kb <= 2
    torch.cuda.synchronize()
    assert torch.equal(s.phi, keep[0]) and torch.equal(s.pi, keep[1]) and s.get_time() == keep[2]
    dphi, dpi, dr0, damp = s.adjoint(g, n, case["robs"])
    assert np.array_equal(dphi.cpu().numpy(), ref[0]) and np.array_equal(dpi.cpu().numpy(), ref[1])
    assert rel_scalar(dr0, ref[2]) <= 1e-13 and rel_scalar(damp, ref[3]) <= 1e-13
    s.close()


@pytest.mark.parametrize("robs_index", [59, 60, 61, 62, 119, 120])
def test_adjoint_observer_on_strip_boundaries(oracle_mod, robs_index):
    case = dict(name="obs", nr=250, nth=12, rmin=0.0, rmax=249.0, a=0.6, m=2, s=-2, r0=20.0, amp=1.0,
                robs=robs_index + 0.61)
    dt = _dt(oracle_mod, case)
    n = 14
    g = seeded_g(n, 12, seed=robs_index)
    for kb in (1, 2):
        gp, gq, _, _ = gpu_adjoint(case, dt, g, n, kb=kb)
        op, oq, _, _ = oracle_adjoint(oracle_mod, case, dt, g, n)
        assert rel(gp, op) <= TOL64 and rel(gq, oq) <= TOL64


W = workloads.ADJOINT


def _adjoint_case():
    return dict(name=W.name, nr=W.nr, nth=W.nth, rmin=W.rstar_min, rmax=W.rstar_max, a=W.a, m=W.m, s=W.s,
                robs=W.rstar_obs, r0=W.r0, amp=W.amp)


def test_adjoint_full_grid_parity_4096x256(oracle_mod):
    # the adjoint workload's full grid, a few reverse steps, oracle element by element
    case = _adjoint_case()
    dt = _dt(oracle_mod, case, W.steps)
    n = 10
    print(f"[gpu] adjoint parity 4096x256 n={n}", flush=True)
    g = seeded_g(n, case["nth"], seed=12)
    gp, gq, _, _ = gpu_adjoint(case, dt, g, n)
    op, oq, _, _ = oracle_adjoint(oracle_mod, case, dt, g, n)
    assert rel(gp, op) <= TOL64 and rel(gq, oq) <= TOL64, (rel(gp, op), rel(gq, oq))


def test_adjoint_identity_full_run_4096x256(oracle_mod):
    # <g, E K^k du0> summed over the recorded steps equals <lambda^0, du0>:
    # the GPU reverse sweep is the transpose of the GPU forward map over the
    # whole 20000-step run (source off: the linear part)
    import torch
    case = _adjoint_case()
    dt = _dt(oracle_mod, case, W.steps)
    n = W.steps
    print(f"[gpu] adjoint identity 4096x256 n={n}", flush=True)
    s = make_solver(dict(case, r0=None), dt)
    phi, pi = inputs.smooth_random_state(W.nr, W.nth, W.rstar_min, W.rstar_max, seed=31)
    s.set_state(phi, pi)
    s.set_observer(W.rstar_obs, n + 1)
    s.step(n)
    torch.cuda.synchronize()
    s.check_finite()
    w = s.wave.cpu().numpy()
    g = seeded_g(n, W.nth, seed=32)
    dphi, dpi, _, _ = s.adjoint(g, n, W.rstar_obs)
    lhs = float(np.sum((np.conj(g) * w).real))
    rhs = float(np.sum((np.conj(dphi.cpu().numpy()) * phi).real) + np.sum((np.conj(dpi.cpu().numpy()) * pi).real))
    print(f"[gpu] identity lhs={lhs:.15e} rhs={rhs:.15e}", flush=True)
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
    s.close()


def test_adjoint_central_differences_full_run_4096x256():
    # the adjoint workload: a = 0.6, m = 2, 4096 x 256, 20000 steps, waveform
    # misfit against a target from perturbed (r0, amp, pulse); gradients for
    # r0, amp and 3 random directions of Phi0 vs central differences
    # (h = 1e-6) of GPU forward runs.  At the stable dt the run covers
    # T = 21.6 M, while the signal needs ~280 M to reach r* = 300 from the
    # source (r* = 12.8) and the pulse (r* = 20): the misfit is read at
    # r* = 30, which both reach within the run.
    import torch
    from paper_0909_4039_amd.solver import Solver, suggest_dt
    n = W.steps
    robs = W.extra["rstar_obs_reached"]
    dt = suggest_dt(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, 1.0, W.m, W.s, n)
    s = Solver(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, 1.0, W.m, W.s, dt)
    amp0 = inputs.seeded_amplitude(W.pulse["seed"])
    phi, pi = inputs.pulse(W.nr, W.nth, W.rstar_min, W.rstar_max, W.m, W.pulse["center"], W.pulse["width"], amp0)
    er, ea, ep = workloads.adjoint_perturbation()

    def wave(ph, pq, r0, amp):
        s.set_source(r0, amp)
        s.set_state(ph, pq)
        s.set_time(0.0, 0)
        s.set_observer(robs, n + 1)
        s.step(n)
        torch.cuda.synchronize()
        return s.wave.cpu().numpy()

    print(f"[gpu] adjoint FD 4096x256 n={n}", flush=True)
    target = wave(phi * (1 + ep), pi * (1 + ep), W.r0 * (1 + er), W.amp * (1 + ea))

    def loss(ph, pq, r0, amp):
        return float(np.sum(np.abs(wave(ph, pq, r0, amp) - target) ** 2))

    w0 = wave(phi, pi, W.r0, W.amp)
    L0 = float(np.sum(np.abs(w0 - target) ** 2))
    print(f"[gpu] misfit {L0:.6e}, |w| max {np.abs(w0).max():.3e}", flush=True)
    assert L0 > 0.0
    g = 2.0 * (w0 - target)
    s.set_source(W.r0, W.amp)
    dphi, dpi, dr0, damp = s.adjoint(g, n, robs)
    dphi = dphi.cpu().numpy()
    h = 1e-6
    fd_r0 = (loss(phi, pi, W.r0 + h, W.amp) - loss(phi, pi, W.r0 - h, W.amp)) / (2 * h)
    fd_amp = (loss(phi, pi, W.r0, W.amp + h) - loss(phi, pi, W.r0, W.amp - h)) / (2 * h)
    print(f"[gpu] dL/dr0 adjoint {dr0:.12e} fd {fd_r0:.12e}; dL/damp {damp:.12e} fd {fd_amp:.12e}", flush=True)
    assert dr0 == pytest.approx(fd_r0, rel=1e-5)
    assert damp == pytest.approx(fd_amp, rel=1e-5)
    # Directions of unit size per point: L is exactly quadratic in the
    # initial data, and a direction of unit total norm over 10^6 points
    # would move L by ~1e-9 of itself at h = 1e-6, below its rounding.
    rng = np.random.default_rng(7)
    for k in range(3):
        d = (rng.standard_normal(phi.shape) + 1j * rng.standard_normal(phi.shape)) / np.sqrt(2.0)
        fd = (loss(phi + h * d, pi, W.r0, W.amp) - loss(phi - h * d, pi, W.r0, W.amp)) / (2 * h)
        ad = float(np.sum((np.conj(dphi) * d).real))
        print(f"[gpu] direction {k}: adjoint {ad:.12e} fd {fd:.12e}", flush=True)
        assert ad == pytest.approx(fd, rel=1e-5)
    s.close()


def test_fp32_context_has_no_adjoint():
    from paper_0909_4039_amd import TeukError
    from paper_0909_4039_amd.solver import Solver
    s = Solver(64, 8, -20.0, 40.0, 0.5, 1.0, 2, -2, 0.01, prec=32)
    with pytest.raises(TeukError) as e:
        s.adjoint(np.zeros((3, 8), complex), 2, 1.0)
    assert e.value.code == -5
    s.close()


def test_autograd_waveform(oracle_mod):
    import torch
    from paper_0909_4039_amd.autograd import waveform
    from paper_0909_4039_amd.solver import Solver
    case = CASES[5]
    dt = _dt(oracle_mod, case)
    n = 80
    s = Solver(case["nr"], case["nth"], case["rmin"], case["rmax"], case["a"], 1.0, case["m"], case["s"], dt)
    phi, pi = inputs.pulse(case["nr"], case["nth"], case["rmin"], case["rmax"], case["m"], 3.0, 2.5, 1.0)
    dev = torch.device("cuda:0")
    p0 = torch.tensor(phi, device=dev, requires_grad=True)
    q0 = torch.tensor(pi, device=dev, requires_grad=True)
    r0 = torch.tensor(10.0, dtype=torch.float64, device=dev, requires_grad=True)
    amp = torch.tensor(0.8, dtype=torch.float64, device=dev, requires_grad=True)
    w = waveform(s, p0, q0, r0, amp, n, case["robs"])
    target = torch.zeros_like(w)
    L = (w - target).abs().pow(2).sum()
    L.backward()
    # forward against the oracle, gradients against the oracle's reverse sweep
    o = oracle_mod.Oracle(case["nr"], case["nth"], case["rmin"], case["rmax"], case["a"], 1.0, case["m"],
                          case["s"], dt, r0=10.0, amp=0.8, rstar_obs=case["robs"])
    _, _, ow = o.run(phi, pi, n)
    assert rel(w.detach().cpu().numpy(), ow) <= TOL64
    op, oq, or0, oamp = o.adjoint_run(2.0 * ow, n)
    assert rel(p0.grad.cpu().numpy(), op) <= 1e-11 and rel(q0.grad.cpu().numpy(), oq) <= 1e-11
    assert rel_scalar(float(r0.grad), or0) <= 1e-10 and rel_scalar(float(amp.grad), oamp) <= 1e-10
    s.close()


def _random_adjoint_cases():
    from test_gpu_step import _random_cases
    return _random_cases(k=12, seed=3031)


@pytest.mark.parametrize("case", _random_adjoint_cases(), ids=lambda c: c["name"])
def test_adjoint_parity_seeded_random_configurations(oracle_mod, case):
    """Seeded random grids, spins, modes, sources and tilings (forward and
    reverse-sweep tiling both set), against the oracle's reverse sweep."""
    dt = _dt(oracle_mod, case, 1000)
    n = case["n"]
    print(f"[gpu] random adjoint parity {case}", flush=True)
    g = seeded_g(n, case["nth"], seed=int(case["name"][4:]) + 200)
    gp, gq, gr0, gamp = gpu_adjoint(case, dt, g, n, kb=case["kb"], rows=case["rows"], t_start=0.21)
    op, oq, or0, oamp = oracle_adjoint(oracle_mod, case, dt, g, n, t_start=0.21)
    assert rel(gp, op) <= TOL64 and rel(gq, oq) <= TOL64, (rel(gp, op), rel(gq, oq))
    if not case.get("r0"):
        assert gr0 == 0.0 and gamp == 0.0          # no source: both gradients are 0 by contract
        return
    for got, want in ((gamp, oamp), (gr0, or0)):
        # a source at the edge of the observer's reach gives values near the
        # underflow of the sums; those are compared absolutely
        assert abs(got - want) <= 1e-11 * abs(want) + 1e-25, (got, want)
