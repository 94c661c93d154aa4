"""Pins for the oracle's reverse sweep with a moving source.

The forward run is pinned separately; here the gradients of a loss with
respect to every orbit-table entry (r0_e, phi_e) and the amplitude are
checked against central differences of the oracle's forward run, and a
fixed orbit (phi = Omega t) must give back, through the chain rule, the
static source's dL/dr0 and dL/damp.  The adjoint of the initial data does
not depend on the source, so it must equal the static sweep's bit for bit.
"""
import numpy as np
import pytest

from paper_0909_4039_amd import inputs

NR, NTH = 48, 10
RMIN, RMAX = -12.0, 24.0
A, M_AZ, S = 0.6, 2, -2


def _oracle(oracle_mod, amp=1.0, r0=7.0, robs=None):
    dt = oracle_mod.stable_dt(NR, NTH, RMIN, RMAX, A, 1.0, M_AZ, S, 5000)
    o = oracle_mod.Oracle(NR, NTH, RMIN, RMAX, A, 1.0, M_AZ, S, dt, r0=r0, amp=amp,
                          rstar_obs=robs if robs is not None else 6.3)
    return o, dt


def _loss(o, traj, G, n, phi0, pi0):
    # L = Re sum conj(G) w: its waveform gradient dL/dRe w + i dL/dIm w is G
    o.set_trajectory(traj)
    _, _, w = o.run(phi0, pi0, n)
    return float(np.sum((np.conj(G) * w).real))


def _setup(oracle_mod, n, seed):
    o, dt = _oracle(oracle_mod)
    # a decaying orbit that crosses the observer's neighbourhood in r*
    traj = inputs.inspiral_trajectory(7.0, A, 1.0, 0.3, dt, n)
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n + 1, NTH)) + 1j * rng.standard_normal((n + 1, NTH))
    phi0, pi0 = inputs.random_state(NR, NTH, seed=seed + 1)
    return o, dt, traj, G, phi0, pi0


def test_moving_adjoint_matches_central_differences(oracle_mod):
    n = 16
    o, dt, traj, G, phi0, pi0 = _setup(oracle_mod, n, seed=71)
    o.set_trajectory(traj)
    _, _, dtraj, damp = o.adjoint_run_moving(G, n)
    assert dtraj.shape == (2 * n, 2)
    scale = np.abs(dtraj).max(axis=0)
    assert np.all(scale > 0)
    for e in (0, 1, 2, 9, 2 * n - 2, 2 * n - 1):
        for k, h in ((0, 1e-5), (1, 1e-5)):
            tp, tm = traj.copy(), traj.copy()
            tp[e, k] += h
            tm[e, k] -= h
            fd = (_loss(o, tp, G, n, phi0, pi0) - _loss(o, tm, G, n, phi0, pi0)) / (2 * h)
            assert abs(fd - dtraj[e, k]) <= 1e-7 * scale[k], (e, k, fd, dtraj[e, k])
    # entries past 2n are never read by n steps
    tp = traj.copy()
    tp[2 * n:, :] += 0.5
    assert _loss(o, tp, G, n, phi0, pi0) == _loss(o, traj, G, n, phi0, pi0)
    # the loss is affine in amp: a central difference is exact up to rounding
    h = 1e-3
    Lp = _loss(_oracle(oracle_mod, amp=1.0 + h)[0], traj, G, n, phi0, pi0)
    Lm = _loss(_oracle(oracle_mod, amp=1.0 - h)[0], traj, G, n, phi0, pi0)
    assert abs((Lp - Lm) / (2 * h) - damp) <= 1e-9 * abs(damp)


def test_moving_adjoint_of_initial_data_is_the_static_one(oracle_mod):
    n = 12
    o, dt, traj, G, phi0, pi0 = _setup(oracle_mod, n, seed=72)
    sp, sq, _, _ = o.adjoint_run(G, n)
    o.set_trajectory(traj)
    mp, mq, _, _ = o.adjoint_run_moving(G, n)
    assert np.array_equal(mp, sp) and np.array_equal(mq, sq)


def test_fixed_orbit_gradients_chain_to_the_static_ones(oracle_mod):
    # phi_e = Omega(r0) t_e: dL/dr0 = sum_e dL/dr0_e + dL/dphi_e t_e dOmega/dr0
    n = 20
    r0 = 7.0
    o, dt = _oracle(oracle_mod, r0=r0)
    rng = np.random.default_rng(73)
    G = rng.standard_normal((n + 1, NTH)) + 1j * rng.standard_normal((n + 1, NTH))
    _, _, s_r0, s_amp = o.adjoint_run(G, n)
    traj = inputs.inspiral_trajectory(r0, A, 1.0, 0.0, dt, n)
    o.set_trajectory(traj)
    _, _, dtraj, m_amp = o.adjoint_run_moving(G, n)
    t = np.arange(2 * n) * 0.5 * dt
    dOm = -1.5 * np.sqrt(r0) / (r0 ** 1.5 + A) ** 2
    chained = np.sum(dtraj[:, 0]) + np.sum(dtraj[:, 1] * t) * dOm
    assert chained == pytest.approx(s_r0, rel=1e-11)
    assert m_amp == pytest.approx(s_amp, rel=1e-12)


def test_moving_adjoint_refuses_a_short_table(oracle_mod):
    n = 6
    o, dt, traj, G, phi0, pi0 = _setup(oracle_mod, n, seed=74)
    o.set_trajectory(traj[:2 * n - 1])
    with pytest.raises(ValueError):
        o.adjoint_run_moving(G, n)
