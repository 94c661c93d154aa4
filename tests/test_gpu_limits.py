"""The largest grids the C ABI accepts, stepped on the GPU and compared with
the oracle on windows next to the far ends of the grid (where the 32-bit
byte offsets and the chunk counts are largest): n_rstar = 2^26 with
n_theta = 4, and n_theta = 2^20 with n_rstar = 4.  Also the rejections just
past the limits.
"""
import numpy as np
import pytest

from paper_0909_4039_amd import inputs

pytestmark = pytest.mark.gpu


def _run(nr, nth, rmin, rmax, a, m, window, n, seed):
    import torch
    import oracle
    from paper_0909_4039_amd.solver import Solver, suggest_dt
    i0, ni, j0, nj = window
    dt = suggest_dt(nr, nth, rmin, rmax, a, 1.0, m, -2, 1000)
    # random data on the window only, zero elsewhere
    wp, wq = inputs.random_state(ni, nj, seed=seed)
    s = Solver(nr, nth, rmin, rmax, a, 1.0, m, -2, dt)
    s.phi[j0:j0 + nj, i0:i0 + ni] = torch.as_tensor(wp, device="cuda:0")
    s.pi[j0:j0 + nj, i0:i0 + ni] = torch.as_tensor(wq, device="cuda:0")
    torch.cuda.synchronize()
    s.step(n)
    torch.cuda.synchronize()
    s.check_finite()
    gp = s.phi[j0:j0 + nj, i0:i0 + ni].cpu().numpy()
    gq = s.pi[j0:j0 + nj, i0:i0 + ni].cpu().numpy()
    rest = float(s.phi.abs().sum()) - float(np.abs(gp).sum())
    s.close()
    torch.cuda.empty_cache()
    o = oracle.Oracle(nr, nth, rmin, rmax, a, 1.0, m, -2, dt, window=window)
    op, oq, _ = o.run(wp, wq, n, record=False)
    ok = np.isfinite(op)
    assert ok.sum() > 0.3 * ok.size
    for g, r in ((gp, op), (gq, oq)):
        assert np.linalg.norm(g[ok] - r[ok]) <= 1e-12 * np.linalg.norm(r[ok])
        assert np.max(np.abs(g[ok] - r[ok])) <= 1e-12 * np.max(np.abs(r[ok]))
    return rest


def test_max_rstar_grid():
    nr, nth = 1 << 26, 4
    print(f"[gpu] {nr} x {nth}", flush=True)
    # window touching the last column (Dirichlet) and the pole rows
    rest = _run(nr, nth, -100.0, 400.0, 0.7, 2, (nr - 160, 160, 0, nth), 8, seed=90)
    assert rest < 1e30


def test_max_theta_grid():
    nr, nth = 4, 1 << 20
    print(f"[gpu] {nr} x {nth}", flush=True)
    _run(nr, nth, -10.0, 10.0, 0.3, 1, (0, nr, nth - 48, 48), 6, seed=91)


def test_limits_rejected():
    from paper_0909_4039_amd import TeukError
    from paper_0909_4039_amd.solver import Solver
    for nr, nth in (((1 << 26) + 1, 4), (4, (1 << 20) + 1)):
        with pytest.raises(TeukError):
            Solver(nr, nth, -10.0, 10.0, 0.3, 1.0, 2, -2, 0.01)
