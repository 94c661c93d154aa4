"""Checkpointed parameter gradients on the GPU (teuk_param_gradient through
the C ABI): dL/da, dL/dM, dL/dr0 and dL/damp of a waveform loss.

Bars: against the oracle's central differences of complete runs, 1e-7
relative (both sides are O(h^2) differences of the same derivative; 2e-8
and less seen); for r0 and amp against the GPU's exact reverse sweep
(teuk_adjoint), 1e-7 and 1e-9;
results bitwise identical for every checkpoint interval; dL/du^0 equal bit
for bit to teuk_adjoint's; on the adjoint workload's full 4096 x 256 grid,
dL/da against central differences of GPU forward runs.
"""
import numpy as np
import pytest

from paper_0909_4039_amd import inputs, workloads

pytestmark = pytest.mark.gpu

CASE = dict(nr=150, nth=24, rmin=-20.0, rmax=55.0, a=0.6, M=1.0, m=2, s=-2, r0=10.0, amp=1.0, robs=14.0)
N = 45


def _dt(oracle_mod, c):
    return oracle_mod.stable_dt(c["nr"], c["nth"], c["rmin"], c["rmax"], c["a"], 1.0, c["m"], c["s"], 10000)


def _solver(c, dt, prec=64):
    from paper_0909_4039_amd.solver import Solver
    s = Solver(c["nr"], c["nth"], c["rmin"], c["rmax"], c["a"], c["M"], c["m"], c["s"], dt, prec=prec)
    s.set_source(c["r0"], c["amp"])
    return s


def _inputs(c, n, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n + 1, c["nth"])) + 1j * rng.standard_normal((n + 1, c["nth"]))
    phi0, pi0 = inputs.random_state(c["nr"], c["nth"], seed=seed + 1)
    return G, phi0, pi0


@pytest.mark.parametrize("param,h", [("a", 1e-5), ("M", 1e-5), ("r0", 1e-5), ("amp", 1e-3)])
def test_param_gradient_against_oracle_differences(oracle_mod, param, h):
    c = CASE
    dt = _dt(oracle_mod, c)
    G, phi0, pi0 = _inputs(c, N, 101)
    print(f"[gpu] param gradient {param} vs oracle", flush=True)
    s = _solver(c, dt)
    got = s.param_gradient(param, G, N, c["robs"], phi0, pi0, h=h, checkpoint_interval=7)
    s.close()
    ref = oracle_mod.param_gradient_fd(c["nr"], c["nth"], c["rmin"], c["rmax"], c["a"], c["M"], c["m"], c["s"], dt,
                                       c["r0"], c["amp"], c["robs"], param, h, G, N, phi0, pi0)
    print(f"[gpu] {param}: gpu {got:.12e} oracle {ref:.12e}", flush=True)
    assert abs(ref) > 0
    assert got == pytest.approx(ref, rel=1e-7)


@pytest.mark.parametrize("nr,nth,rows", [(61, 4, 2), (190, 7, 4), (47, 33, 64)])
def test_param_gradient_ragged_grids(oracle_mod, nr, nth, rows):
    """Grids of one or a few partial strips (a ragged last strip), with the
    context's tiling at 2, 4 and 64 rows (a chunk taller than the grid) for
    the checkpointing pass and the sweep's one-step launches at their own
    height, against the oracle's central differences."""
    c = dict(CASE, nr=nr, nth=nth, rmin=-20.0, rmax=40.0, robs=13.0)
    dt = _dt(oracle_mod, c)
    n = 12
    G, phi0, pi0 = _inputs(c, n, 121)
    s = _solver(c, dt)
    s.set_tiling(rows)
    print(f"[gpu] param gradient a on {nr}x{nth}, {rows} rows", flush=True)
    got = s.param_gradient("a", G, n, c["robs"], phi0, pi0, h=1e-5, checkpoint_interval=5)
    s.close()
    ref = oracle_mod.param_gradient_fd(c["nr"], c["nth"], c["rmin"], c["rmax"], c["a"], c["M"], c["m"], c["s"], dt,
                                       c["r0"], c["amp"], c["robs"], "a", 1e-5, G, n, phi0, pi0)
    print(f"[gpu] gpu {got:.12e} oracle {ref:.12e}", flush=True)
    assert abs(ref) > 0
    assert got == pytest.approx(ref, rel=1e-6)


def test_source_parameters_match_the_exact_sweep(oracle_mod):
    c = CASE
    dt = _dt(oracle_mod, c)
    G, phi0, pi0 = _inputs(c, N, 102)
    s = _solver(c, dt)
    dphi, dpi, dr0, damp = s.adjoint(G, N, c["robs"])
    g_r0 = s.param_gradient("r0", G, N, c["robs"], phi0, pi0, h=1e-5)
    g_amp, lp, lq = s.param_gradient("amp", G, N, c["robs"], phi0, pi0, h=1e-3, want_initial=True)
    assert g_r0 == pytest.approx(dr0, rel=1e-7)
    assert g_amp == pytest.approx(damp, rel=1e-9)
    # lambda^0 comes out of the same reverse steps
    assert np.array_equal(lp.cpu().numpy(), dphi.cpu().numpy()) and np.array_equal(lq.cpu().numpy(), dpi.cpu().numpy())
    s.close()


def test_checkpoint_interval_does_not_change_the_result(oracle_mod):
    c = CASE
    dt = _dt(oracle_mod, c)
    G, phi0, pi0 = _inputs(c, N, 103)
    s = _solver(c, dt)
    ref = s.param_gradient("a", G, N, c["robs"], phi0, pi0, h=1e-5, checkpoint_interval=1)
    for C in (0, 2, 7, 44, 45, 1000):
        assert s.param_gradient("a", G, N, c["robs"], phi0, pi0, h=1e-5, checkpoint_interval=C) == ref, C
    # zero steps: only lambda^0 = E^H g^0, and no parameter dependence
    g0, lp, lq = s.param_gradient("a", G[:1], 0, c["robs"], phi0, pi0, h=1e-5, want_initial=True)
    assert g0 == 0.0 and np.count_nonzero(lp.cpu().numpy()) > 0 and not np.any(lq.cpu().numpy())
    s.close()


def test_param_gradient_does_not_depend_on_the_context_tiling(oracle_mod):
    # the sweep's one-step launches take a chunk height of their own, and its
    # checkpointing pass the context's launches, whose two fused steps equal
    # single steps bit for bit: the context's tiling changes no bit
    c = CASE
    dt = _dt(oracle_mod, c)
    G, phi0, pi0 = _inputs(c, N, 104)
    s = _solver(c, dt)
    s.set_blocking(1)
    ref = s.param_gradient("a", G, N, c["robs"], phi0, pi0, h=1e-5, checkpoint_interval=8)
    for rows, order, kb in ((2, 0, 1), (5, 1, 2), (16, 0, 2), (12, 2, 2), (64, 0, 2)):
        s.set_tiling(rows, order)
        s.set_blocking(kb)
        print(f"[gpu] param gradient a, context tiling {rows}:{order}, {kb} steps per launch", flush=True)
        got = s.param_gradient("a", G, N, c["robs"], phi0, pi0, h=1e-5, checkpoint_interval=8)
        assert got == ref, (rows, order, kb)
    s.close()


def test_param_gradient_errors(oracle_mod):
    from paper_0909_4039_amd import TeukError
    c = CASE
    dt = _dt(oracle_mod, c)
    G, phi0, pi0 = _inputs(c, 4, 104)
    s = _solver(c, dt)
    with pytest.raises(ValueError):
        s.param_gradient("s", G, 4, c["robs"], phi0, pi0)
    with pytest.raises(TeukError) as e:          # a + h beyond M
        s.param_gradient("a", G, 4, c["robs"], phi0, pi0, h=0.5)
    assert e.value.code == -1
    with pytest.raises(TeukError) as e:
        s.param_gradient("a", G, 4, c["robs"], phi0, pi0, h=-1e-5)
    assert e.value.code == -1
    s.set_trajectory(inputs.inspiral_trajectory(c["r0"], c["a"], 1.0, 0.1, dt, 4))
    with pytest.raises(TeukError) as e:          # fixed orbits only
        s.param_gradient("a", G, 4, c["robs"], phi0, pi0)
    assert e.value.code == -5
    s.close()
    s32 = _solver(c, dt, prec=32)
    with pytest.raises(TeukError) as e:
        s32.param_gradient("a", G, 4, c["robs"], phi0, pi0)
    assert e.value.code == -5
    s32.close()
    from paper_0909_4039_amd.solver import Solver
    s0 = Solver(c["nr"], c["nth"], c["rmin"], c["rmax"], c["a"], 1.0, c["m"], c["s"], dt)
    with pytest.raises(TeukError) as e:          # no source to move
        s0.param_gradient("r0", G, 4, c["robs"], phi0, pi0, h=1e-5)
    assert e.value.code == -2
    s0.close()


def test_spin_gradient_full_grid_4096x256():
    # the adjoint workload's grid and source, 2000 steps, observer at r* = 14
    # next to the source: dL/da against central differences of GPU forward
    # runs of solvers built at a +- h
    import torch
    from paper_0909_4039_amd.solver import Solver, suggest_dt
    W = workloads.ADJOINT
    n = 2000
    robs = 14.0
    dt = suggest_dt(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, 1.0, W.m, W.s, W.steps)
    phi0, pi0 = inputs.pulse(W.nr, W.nth, W.rstar_min, W.rstar_max, W.m, W.pulse["center"], W.pulse["width"],
                             inputs.seeded_amplitude(W.pulse["seed"]))
    rng = np.random.default_rng(105)
    G = rng.standard_normal((n + 1, W.nth)) + 1j * rng.standard_normal((n + 1, W.nth))

    def loss(a):
        s = Solver(W.nr, W.nth, W.rstar_min, W.rstar_max, a, 1.0, W.m, W.s, dt)
        s.set_source(W.r0, W.amp)
        s.set_state(phi0, pi0)
        s.set_observer(robs, n + 1)
        s.step(n)
        torch.cuda.synchronize()
        w = s.wave.cpu().numpy()
        s.close()
        return float(np.sum((np.conj(G) * w).real))

    print(f"[gpu] spin gradient 4096x256 n={n}", flush=True)
    s = Solver(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, 1.0, W.m, W.s, dt)
    s.set_source(W.r0, W.amp)
    got = s.param_gradient("a", G, n, robs, phi0, pi0, h=1e-5)
    s.close()
    h = 1e-5
    fd = (loss(W.a + h) - loss(W.a - h)) / (2 * h)
    print(f"[gpu] dL/da checkpointed {got:.12e} fd {fd:.12e}", flush=True)
    assert abs(fd) > 0
    assert got == pytest.approx(fd, rel=1e-5)


def test_autograd_through_the_spin(oracle_mod):
    # L = sum |w - target|^2; dL/dspin by autograd (checkpointed sweep) and by
    # central differences of forward runs of solvers built at spin +- h
    import torch
    from paper_0909_4039_amd.autograd import waveform
    from paper_0909_4039_amd.solver import Solver
    c = CASE
    dt = _dt(oracle_mod, c)
    G, phi0, pi0 = _inputs(c, N, 106)
    p0 = torch.as_tensor(phi0, device="cuda:0")
    q0 = torch.as_tensor(pi0, device="cuda:0")
    target = torch.as_tensor(G, device="cuda:0") * 1e-3

    def solver_at(a):
        s = Solver(c["nr"], c["nth"], c["rmin"], c["rmax"], a, c["M"], c["m"], c["s"], dt)
        s.set_source(c["r0"], c["amp"])
        return s

    s = solver_at(c["a"])
    spin = torch.tensor(c["a"], dtype=torch.float64, requires_grad=True)
    r0 = torch.tensor(c["r0"], dtype=torch.float64, requires_grad=True)
    w = waveform(s, p0, q0, r0, c["amp"], N, c["robs"], spin=spin, spin_h=1e-5)
    L = torch.sum(torch.abs(w - target) ** 2)
    L.backward()

    def loss(a):
        sa = solver_at(a)
        with torch.no_grad():
            v = torch.sum(torch.abs(waveform(sa, p0, q0, c["r0"], c["amp"], N, c["robs"]) - target) ** 2).item()
        sa.close()
        return v

    h = 1e-5
    fd = (loss(c["a"] + h) - loss(c["a"] - h)) / (2 * h)
    print(f"[gpu] autograd dL/dspin {spin.grad.item():.12e} fd {fd:.12e}; dL/dr0 {r0.grad.item():.6e}", flush=True)
    assert abs(fd) > 0 and r0.grad is not None
    assert spin.grad.item() == pytest.approx(fd, rel=1e-6)
    with pytest.raises(ValueError):
        waveform(s, p0, q0, c["r0"], c["amp"], N, c["robs"], spin=torch.tensor(c["a"] + 0.1))
    s.close()
