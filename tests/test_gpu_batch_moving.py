"""Batched inspirals (teuk_batch_set_trajectory through the C ABI): the m
modes of one inspiralling orbit, plus other instances, stepped together.
Every instance must equal, bit for bit, a single-mode run given the same
orbit table (single-mode moving runs are parity-tested against the
oracle), whatever the tiling, steps per launch, launch form or graph
replays; one instance is also compared with the oracle directly (1e-12).
"""
import numpy as np
import pytest

from paper_0909_4039_amd import inputs

pytestmark = pytest.mark.gpu

MAX_STEPS = 60
N = 37

SPECS = [
    # nr, nth, rmin, rmax, a, m, s, r0, amp, robs, q (None: fixed orbit)
    (257, 33, -50.0, 100.0, 0.9, 1, -2, 8.0, 1.0, 12.0, 0.2),
    (257, 33, -50.0, 100.0, 0.9, 2, -2, 8.0, 1.0, 12.0, 0.2),
    (257, 33, -50.0, 100.0, 0.9, 3, -2, 8.0, 1.0, 12.0, 0.2),
    (130, 40, -40.0, 90.0, 0.3, -2, -2, 9.0, 0.7, 20.0, None),
    (150, 24, -20.0, 55.0, 0.6, 2, -2, 10.0, 1.0, 14.0, 0.05),
]


def _dt(oracle_mod, sp):
    nr, nth, rmin, rmax, a, m, s = sp[:7]
    return oracle_mod.stable_dt(nr, nth, rmin, rmax, a, 1.0, m, s, 10000)


def _setup(oracle_mod):
    from paper_0909_4039_amd.batch import make_desc
    descs, tables = [], []
    for sp in SPECS:
        nr, nth, rmin, rmax, a, m, s, r0, amp, robs, q = sp
        dt = _dt(oracle_mod, sp)
        descs.append(make_desc(nr, nth, rmin, rmax, a, m, dt, s=s, r0=r0, amp=amp, rstar_obs=robs))
        tables.append(None if q is None else inputs.inspiral_trajectory(r0, a, 1.0, q, dt, MAX_STEPS))
    return descs, tables


def _data(i):
    return inputs.random_state(SPECS[i][0], SPECS[i][1], seed=200 + i)


def single_mode(d, table, phi, pi, n):
    import torch
    from paper_0909_4039_amd.solver import Solver
    g = d.grid
    s = Solver(g.n_rstar, g.n_theta, g.rstar_min, g.rstar_max, d.a, d.M, d.m, d.s, d.dt)
    s.set_source(d.r0, d.amp, d.sigma_r_cells, d.sigma_th_cells)
    if table is not None:
        s.set_trajectory(table)
    s.set_state(phi, pi)
    s.set_observer(d.rstar_obs, n + 1)
    s.step(n)
    torch.cuda.synchronize()
    out = (s.phi.cpu().numpy(), s.pi.cpu().numpy(), s.wave.cpu().numpy())
    s.close()
    return out


def make_batch(descs, tables):
    from paper_0909_4039_amd.batch import Batch
    b = Batch(descs, MAX_STEPS)
    for i, t in enumerate(tables):
        b.set_state(i, *_data(i))
        if t is not None:
            b.set_trajectory(i, t)
    return b


def result(b, i, rows):
    b.synchronize()
    return b.phi(i).cpu().numpy(), b.pi(i).cpu().numpy(), b.waves[i][:rows].cpu().numpy()


def same(got, ref):
    return all(np.array_equal(x, y) for x, y in zip(got, ref))


@pytest.fixture(scope="module")
def reference(oracle_mod):
    descs, tables = _setup(oracle_mod)
    return descs, tables, [single_mode(d, tables[i], *_data(i), N) for i, d in enumerate(descs)]


@pytest.mark.parametrize("rows,kb,persistent", [(0, 2, True), (0, 1, True), (5, 2, False), (3, 1, False),
                                               (64, 2, True)])
def test_batched_inspiral_bitwise_equals_single_mode(reference, rows, kb, persistent):
    descs, tables, ref = reference
    print(f"[gpu] batched inspiral rows={rows} kb={kb} persistent={persistent}", flush=True)
    b = make_batch(descs, tables)
    b.set_tiling(rows, kb, persistent)
    b.step(N)
    for i in range(len(descs)):
        assert same(result(b, i, N + 1), ref[i]), (i, rows, kb, persistent)
    b.close()


def test_batched_inspiral_graph_replays(reference):
    import torch
    descs, tables, ref = reference
    print("[gpu] batched inspiral graph replays", flush=True)
    b = make_batch(descs, tables)
    b.capture_graph(8)
    for _ in range(4):
        b.step(8)
        b.synchronize()
        (torch.randn(1000, device="cuda:0") * 2).sum().item()
    b.step(5)
    for i in range(len(descs)):
        assert same(result(b, i, N + 1), ref[i]), i
    b.close()


def test_batched_inspiral_instance_against_oracle(oracle_mod, reference):
    descs, tables, _ = reference
    b = make_batch(descs, tables)
    b.step(N)
    i = 1
    d, g = descs[i], descs[i].grid
    o = oracle_mod.Oracle(g.n_rstar, g.n_theta, g.rstar_min, g.rstar_max, d.a, 1.0, d.m, d.s, d.dt, r0=d.r0,
                          amp=d.amp, rstar_obs=d.rstar_obs)
    o.set_trajectory(tables[i])
    op, oq, ow = o.run(*_data(i), N)
    gp, gq, gw = result(b, i, N + 1)
    rel = lambda x, y: max(np.linalg.norm(x - y) / np.linalg.norm(y),   # relative L2 and per element
                           np.max(np.abs(x - y)) / np.max(np.abs(y)))
    assert rel(gp, op) <= 1e-12 and rel(gq, oq) <= 1e-12 and rel(gw, ow) <= 1e-12
    b.close()


def test_batched_trajectory_clear_and_errors(oracle_mod, reference):
    from paper_0909_4039_amd import TeukError
    from paper_0909_4039_amd.batch import Batch, make_desc
    descs, tables, ref = reference
    # a table set and cleared again leaves the fixed orbit
    b = make_batch(descs, tables)
    b.set_trajectory(3, inputs.inspiral_trajectory(9.0, 0.3, 1.0, 0.1, descs[3].dt, MAX_STEPS))
    b.set_trajectory(3, None)
    b.step(N)
    assert same(result(b, 3, N + 1), ref[3])
    with pytest.raises(TeukError) as e:          # shorter than 2 max_steps
        b.set_trajectory(0, tables[0][: 2 * MAX_STEPS - 1])
    assert e.value.code == -1
    bad = tables[0].copy()
    bad[5, 0] = 0.5                              # inside the horizon
    with pytest.raises(TeukError) as e:
        b.set_trajectory(0, bad)
    assert e.value.code == -1
    b.close()
    d = descs[4]
    g = d.grid
    nosrc = make_desc(g.n_rstar, g.n_theta, g.rstar_min, g.rstar_max, d.a, d.m, d.dt, s=d.s, rstar_obs=d.rstar_obs)
    b = Batch([nosrc], MAX_STEPS)
    with pytest.raises(TeukError) as e:          # no source to move
        b.set_trajectory(0, tables[4])
    assert e.value.code == -2
    b.close()


def test_graph_dropped_when_the_kernel_build_changes(reference):
    descs, tables, ref = reference
    print("[gpu] batched inspiral: graph captured before the tables", flush=True)
    b = make_batch(descs, [None] * len(descs))
    b.capture_graph(4)
    for i, t in enumerate(tables):               # switches to the moving build: the graph goes
        if t is not None:
            b.set_trajectory(i, t)
    b.step(N)
    for i in range(len(descs)):
        assert same(result(b, i, N + 1), ref[i]), i
    b.close()
