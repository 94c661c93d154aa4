"""Batched stepping (teuk_batch_* through the C ABI): every instance of a
batch must equal, bit for bit, a single-mode run with the same parameters,
whatever the tiling, the steps per launch or the graph replays; single-mode
runs are themselves parity-tested against the oracle.  One instance is also
compared with the oracle directly.
"""
import numpy as np
import pytest

from paper_0909_4039_amd import inputs, workloads

pytestmark = pytest.mark.gpu

SPECS = [
    # nr, nth, rmin, rmax, a, m, s, r0, amp, robs
    (257, 33, -50.0, 100.0, 0.9, 2, -2, 8.0, 1.0, 30.0),
    (64, 5, -20.0, 40.0, 0.0, 1, -2, 0.0, 0.0, 10.0),
    (1000, 70, -100.0, 300.0, 0.6, 3, 2, 10.0, 0.5, 50.0),
    (130, 128, -40.0, 90.0, 0.3, -2, -2, 9.0, 1.0, 20.0),
    (4, 4, -10.0, 10.0, 0.5, 0, -1, 0.0, 0.0, 1.0),
    (3001, 12, -100.0, 400.0, 0.99, 8, -2, 7.0, 1.0, 100.0),
]


def _descs(oracle_mod):
    from paper_0909_4039_amd.batch import make_desc
    out = []
    for (nr, nth, rmin, rmax, a, m, s, r0, amp, robs) in SPECS:
        dt = oracle_mod.stable_dt(nr, nth, rmin, rmax, a, 1.0, m, s, 10000)
        out.append(make_desc(nr, nth, rmin, rmax, a, m, dt, s=s, r0=r0, amp=amp, rstar_obs=robs))
    return out


def _data(i):
    nr, nth = SPECS[i][0], SPECS[i][1]
    return inputs.random_state(nr, nth, seed=100 + i)


def single_mode(d, phi, pi, n):
    import torch
    from paper_0909_4039_amd.solver import Solver
    g = d.grid
    s = Solver(g.n_rstar, g.n_theta, g.rstar_min, g.rstar_max, d.a, d.M, d.m, d.s, d.dt)
    if d.r0 != 0.0:
        s.set_source(d.r0, d.amp, d.sigma_r_cells, d.sigma_th_cells)
    s.set_state(phi, pi)
    s.set_observer(d.rstar_obs, n + 1)
    s.step(n)
    torch.cuda.synchronize()
    out = (s.phi.cpu().numpy(), s.pi.cpu().numpy(), s.wave.cpu().numpy())
    s.close()
    return out


def make_batch(descs, max_steps):
    from paper_0909_4039_amd.batch import Batch
    b = Batch(descs, max_steps)
    for i in range(len(descs)):
        b.set_state(i, *_data(i))
    return b


def batch_result(b, i, rows):
    b.synchronize()
    return b.phi(i).cpu().numpy(), b.pi(i).cpu().numpy(), b.waves[i][:rows].cpu().numpy()


def assert_same(got, ref, what):
    for x, y, name in zip(got, ref, ("phi", "pi", "wave")):
        assert np.array_equal(x, y), (what, name)


@pytest.fixture(scope="module")
def reference(oracle_mod):
    descs = _descs(oracle_mod)
    n = 37
    return descs, n, [single_mode(d, *_data(i), n) for i, d in enumerate(descs)]


@pytest.mark.parametrize("rows,kb,persistent", [(0, 2, True), (0, 1, True), (5, 2, True), (1, 1, True),
                                               (64, 2, True), (0, 2, False), (3, 1, False), (16, 2, False)])
def test_batch_bitwise_equals_single_mode(reference, rows, kb, persistent):
    descs, n, ref = reference
    print(f"[gpu] batch vs single mode rows={rows} kb={kb} persistent={persistent}", flush=True)
    b = make_batch(descs, 100)
    b.set_tiling(rows, kb, persistent)
    b.step(n)
    for i in range(len(descs)):
        assert_same(batch_result(b, i, n + 1), ref[i], (i, rows, kb))
    assert b.get_step() == n
    b.close()


def test_batch_graph_replays(reference):
    import torch
    descs, n, ref = reference
    print("[gpu] batch graph replays", flush=True)
    b = make_batch(descs, 100)
    b.set_tiling(0, 2, False)
    b.capture_graph(8)
    # 37 = 4 replays of 8 steps + a direct remainder of 5; eager work and
    # synchronisations between the replays
    for k in range(4):
        b.step(8)
        b.synchronize()
        x = torch.randn(1000, device="cuda:0")
        (x * 2).sum().item()
    b.step(5)
    for i in range(len(descs)):
        assert_same(batch_result(b, i, n + 1), ref[i], i)
    b.close()


def test_batch_graph_each_replay(oracle_mod):
    # every replay checked against direct launches of the same batch
    descs = _descs(oracle_mod)
    print("[gpu] batch graph: each replay", flush=True)
    g = make_batch(descs, 60)
    e = make_batch(descs, 60)
    g.capture_graph(4)
    for k in range(5):
        g.step(4)
        e.step(4)
        for i in range(len(descs)):
            assert np.array_equal(batch_result(g, i, 1)[0], batch_result(e, i, 1)[0]), (k, i)
    g.close()
    e.close()


def test_batch_autotune_keeps_state(reference):
    descs, n, ref = reference
    b = make_batch(descs, 100)
    b.step(10)
    b.synchronize()
    before = [b.phi(i).clone() for i in range(len(descs))]
    rows, kb, persistent = b.autotune(2)
    print(f"[gpu] batch autotune picked rows={rows} kb={kb} persistent={persistent}", flush=True)
    b.synchronize()
    for i in range(len(descs)):
        assert torch_equal(b.phi(i), before[i])
    b.step(n - 10)
    for i in range(len(descs)):
        assert_same(batch_result(b, i, n + 1), ref[i], i)
    b.close()


def torch_equal(x, y):
    import torch
    return bool(torch.equal(x, y))


def test_batch_instance_against_oracle(oracle_mod):
    descs = _descs(oracle_mod)
    b = make_batch(descs, 50)
    n = 21
    b.step(n)
    i = 2
    d = descs[i]
    g = d.grid
    o = oracle_mod.Oracle(g.n_rstar, g.n_theta, g.rstar_min, g.rstar_max, d.a, 1.0, d.m, d.s, d.dt, r0=d.r0,
                          amp=d.amp, rstar_obs=d.rstar_obs)
    op, oq, ow = o.run(*_data(i), n)
    gp, gq, gw = batch_result(b, i, n + 1)
    rel = lambda x, y: max(np.linalg.norm(x - y) / np.linalg.norm(y),   # relative L2 and per element
                           np.max(np.abs(x - y)) / np.max(np.abs(y)))
    assert rel(gp, op) <= 1e-12 and rel(gq, oq) <= 1e-12 and rel(gw, ow) <= 1e-12
    b.close()


def test_batch_errors(oracle_mod):
    from paper_0909_4039_amd import TeukError
    from paper_0909_4039_amd.batch import Batch
    descs = _descs(oracle_mod)[:2]
    b = Batch(descs, 6)
    b.step(6)
    with pytest.raises(TeukError) as e:
        b.step(1)
    assert e.value.code == -1
    with pytest.raises(TeukError):
        b.capture_graph(3)           # not a multiple of the two steps per launch
    b.close()


def test_batched_workload_sampled(oracle_mod):
    # the 32-instance batch (m = 1..8 x a in {0, 0.3, 0.6, 0.9}, uneven grids
    # from seed 3), a few steps; four instances against single-mode runs
    import torch
    from paper_0909_4039_amd.batch import Batch, make_desc
    from paper_0909_4039_amd.solver import suggest_dt
    ws = workloads.batched_instances()
    descs = []
    for w in ws:
        dt = suggest_dt(w.nr, w.nth, w.rstar_min, w.rstar_max, w.a, 1.0, w.m, w.s, w.steps)
        descs.append(make_desc(w.nr, w.nth, w.rstar_min, w.rstar_max, w.a, w.m, dt, s=w.s, r0=w.r0, amp=w.amp,
                               rstar_obs=w.rstar_obs))
    n = 6
    print(f"[gpu] batched workload: {len(descs)} instances, "
          f"{sum(w.nr * w.nth for w in ws) / 1e6:.1f} M points, n={n}", flush=True)
    b = Batch(descs, n)
    for i, w in enumerate(ws):
        p = w.pulse
        b.set_state(i, *inputs.pulse(w.nr, w.nth, w.rstar_min, w.rstar_max, w.m, p["center"], p["width"],
                                     p["amplitude"]))
    b.capture_graph(2)
    b.step(n)
    b.synchronize()
    for i in (0, 7, 19, 31):
        w = ws[i]
        p = w.pulse
        ph, pq = inputs.pulse(w.nr, w.nth, w.rstar_min, w.rstar_max, w.m, p["center"], p["width"], p["amplitude"])
        ref = single_mode(descs[i], ph, pq, n)
        assert_same(batch_result(b, i, n + 1), ref, i)
    b.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("seed", [7, 11, 13])
def test_batch_of_seeded_random_instances_is_bitwise(oracle_mod, seed):
    """A batch of 5 seeded random instances (grid, spin, mode, source; see the
    step's random parity cases) with a random tiling, steps per launch and
    launch form equals 5 single-mode runs bit for bit."""
    import torch
    from paper_0909_4039_amd.batch import Batch, make_desc
    from test_gpu_step import _random_cases
    cases = _random_cases(k=5, seed=seed)
    rng = np.random.default_rng(seed)
    n = 12
    descs, data = [], []
    for i, c in enumerate(cases):
        dt = oracle_mod.stable_dt(c["nr"], c["nth"], c["rmin"], c["rmax"], c["a"], 1.0, c["m"], c["s"], 1000)
        descs.append(make_desc(c["nr"], c["nth"], c["rmin"], c["rmax"], c["a"], c["m"], dt, s=c["s"],
                               r0=c.get("r0", 0.0), amp=c.get("amp", 0.0), rstar_obs=c["robs"]))
        data.append(inputs.random_state(c["nr"], c["nth"], seed=seed * 10 + i))
    rows, kb, persistent = int(rng.choice([0, 1, 3, 8, 32])), int(rng.integers(1, 3)), bool(rng.integers(0, 2))
    print(f"[gpu] random batch seed={seed} rows={rows} kb={kb} persistent={persistent}", flush=True)
    b = Batch(descs, n)
    for i, (p, q) in enumerate(data):
        b.set_state(i, p, q)
    b.set_tiling(rows, kb, persistent)
    b.step(n)
    torch.cuda.synchronize()
    for i, d in enumerate(descs):
        got = batch_result(b, i, n + 1)
        assert_same(got, single_mode(d, *data[i], n), f"instance {i}")
    b.close()
