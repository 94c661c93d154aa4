"""Pins for the oracle's moving source (an inspiralling orbit given as an
(r0, phi) table at every half step).

A fixed orbit with phi = Omega t must reproduce the static source; the
response stays linear in the amplitude; and a decaying orbit moves the
source inwards and raises its frequency, as the table says.
"""
import numpy as np
import pytest

from paper_0909_4039_amd import inputs


def _case(oracle_mod, r0, amp, q, n, nr=120, nth=12):
    a, m = 0.6, 2
    rmin, rmax = -30.0, 60.0
    dt = oracle_mod.stable_dt(nr, nth, rmin, rmax, a, 1.0, m, -2, 5000)
    o = oracle_mod.Oracle(nr, nth, rmin, rmax, a, 1.0, m, -2, dt, r0=r0, amp=amp, rstar_obs=20.0)
    traj = inputs.inspiral_trajectory(r0, a, 1.0, q, dt, n)
    return o, traj, dt


def test_fixed_orbit_is_the_static_source(oracle_mod):
    n = 60
    o, traj, dt = _case(oracle_mod, 9.0, 1.0, 0.0, n)
    phi, pi = inputs.random_state(120, 12, seed=61)
    ps, qs, ws = o.run(phi, pi, n)
    o.set_trajectory(traj)
    pm, qm, wm = o.run(phi, pi, n)
    rel = lambda x, y: np.linalg.norm(x - y) / np.linalg.norm(y)
    assert rel(pm, ps) < 1e-13 and rel(qm, qs) < 1e-13 and rel(wm, ws) < 1e-13


def test_moving_source_is_affine_in_amp(oracle_mod):
    n = 50
    phi = np.zeros((12, 120), complex)    # zero data: the response is the source's alone
    pi = np.zeros_like(phi)
    out = []
    for amp in (0.0, 1.0, 2.0):
        o, traj, dt = _case(oracle_mod, 9.0, amp, 0.02, n)
        o.set_trajectory(traj)
        out.append(o.run(phi, pi, n))
    for k in range(3):
        assert not np.any(out[0][k])
        d1, d2 = out[1][k], out[2][k]
        assert np.linalg.norm(d1) > 0
        assert np.linalg.norm(d2 - 2 * d1) <= 1e-14 * np.linalg.norm(d2)


def test_trajectory_follows_the_orbit_law():
    dt, n = 0.05, 400
    tr = inputs.inspiral_trajectory(10.0, 0.0, 1.0, 0.5, dt, n)
    t = np.arange(tr.shape[0]) * 0.5 * dt
    r_exact = (10.0 ** 4 - 256.0 / 5.0 * 0.5 * t) ** 0.25
    assert np.allclose(tr[:, 0], np.maximum(r_exact, 6.0), rtol=1e-14)
    # phase: closed form for a = 0, int sqrt(M) r^{-3/2} dt with r^4 = r_i^4 - k t
    k = 256.0 / 5.0 * 0.5
    phi_exact = (10.0 ** 2.5 - (10.0 ** 4 - k * t) ** 0.625) / (0.625 * k)
    assert np.allclose(tr[:, 1], phi_exact, rtol=1e-6)
    assert inputs.isco_radius(0.0) == pytest.approx(6.0, rel=1e-14)
    assert inputs.isco_radius(0.999999) == pytest.approx(1.0, abs=0.02)


def test_trajectory_outside_table_is_refused(oracle_mod):
    o, traj, dt = _case(oracle_mod, 9.0, 1.0, 0.0, 5)
    o.set_trajectory(traj)
    phi, pi = inputs.random_state(120, 12, seed=63)
    o.run(phi, pi, 5)
    with pytest.raises(ValueError):
        o.run(phi, pi, 6)
    with pytest.raises(ValueError):
        o.adjoint_run(np.zeros((3, 12), complex), 2)
