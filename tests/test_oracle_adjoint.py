"""Pins for the oracle's hand-written reverse step.

(1) Dot-product identity: with the one-step map K assembled column by column
(real 4N x 4N, Eq. 9's real components) on a tiny grid, the reverse step
must equal K^T y.  (2) The reverse sweep's gradients of a waveform misfit
agree with central finite differences (h = 1e-6) for r0, the source
amplitude and random directions of the initial data.
"""
import numpy as np
import pytest

from paper_0909_4039_amd import inputs


def assemble(o, shape):
    nth, nr = shape
    n = nth * nr
    K = np.zeros((4 * n, 4 * n))
    z = np.zeros(shape, complex)
    col = 0
    for field in range(2):
        for unit in (1.0, 1j):
            for k in range(n):
                e = np.zeros(n, complex)
                e[k] = unit
                e = e.reshape(shape)
                p, q = o.step(e, z, 0.0) if field == 0 else o.step(z, e, 0.0)
                K[:, col] = np.concatenate([p.real.ravel(), p.imag.ravel(), q.real.ravel(), q.imag.ravel()])
                col += 1
    return K


def real_view(p, q):
    return np.concatenate([p.real.ravel(), p.imag.ravel(), q.real.ravel(), q.imag.ravel()])


@pytest.mark.parametrize("m,s,a", [(2, -2, 0.9), (1, -2, 0.6), (-3, -2, 0.3), (2, 2, 0.5), (0, -1, 0.7)])
def test_dot_product_identity(oracle_mod, m, s, a):
    nr, nth = 10, 6
    o = oracle_mod.Oracle(nr, nth, -20.0, 30.0, a, 1.0, m, s, 0.05)
    K = assemble(o, (nth, nr))
    lp, lq = inputs.random_state(nr, nth, 11)
    mp, mq, _, _ = o.adjoint_step(lp, lq)
    want = K.T @ real_view(lp, lq)
    got = real_view(mp, mq)
    assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))


def _setup(oracle_mod, r0=10.0, amp=1.0):
    return oracle_mod.Oracle(36, 8, -20.0, 40.0, 0.6, 1.0, 2, -2, 0.03, r0=r0, amp=amp,
                             sigma_r_cells=2.0, sigma_th_cells=2.0, rstar_obs=12.3)


N_STEPS = 120


def _loss(oracle_mod, phi, pi, r0, amp, target):
    o = _setup(oracle_mod, r0, amp)
    _, _, w = o.run(phi, pi, N_STEPS)
    return float(np.sum(np.abs(w - target) ** 2)), w


def test_gradients_match_central_differences(oracle_mod):
    phi, pi = inputs.pulse(36, 8, -20.0, 40.0, 2, 5.0, 3.0, 1.0)
    # target from perturbed parameters and initial data
    _, target = _loss(oracle_mod, 1.02 * phi, 1.02 * pi, 10.15, 0.97, np.zeros((N_STEPS + 1, 8)))
    L0, w = _loss(oracle_mod, phi, pi, 10.0, 1.0, target)
    o = _setup(oracle_mod)
    g = 2.0 * (w - target)
    dphi, dpi, dr0, damp = o.adjoint_run(g, N_STEPS)
    h = 1e-6
    fd_r0 = (_loss(oracle_mod, phi, pi, 10.0 + h, 1.0, target)[0]
             - _loss(oracle_mod, phi, pi, 10.0 - h, 1.0, target)[0]) / (2 * h)
    fd_amp = (_loss(oracle_mod, phi, pi, 10.0, 1.0 + h, target)[0]
              - _loss(oracle_mod, phi, pi, 10.0, 1.0 - h, target)[0]) / (2 * h)
    assert dr0 == pytest.approx(fd_r0, rel=1e-6)
    assert damp == pytest.approx(fd_amp, rel=1e-6)
    rng = np.random.default_rng(7)
    for _ in range(3):
        d = rng.standard_normal(phi.shape) + 1j * rng.standard_normal(phi.shape)
        d /= np.linalg.norm(d)
        fd = (_loss(oracle_mod, phi + h * d, pi, 10.0, 1.0, target)[0]
              - _loss(oracle_mod, phi - h * d, pi, 10.0, 1.0, target)[0]) / (2 * h)
        an = float(np.sum((dphi.conj() * d).real))
        assert an == pytest.approx(fd, rel=1e-6, abs=1e-9 * abs(L0))
        fd = (_loss(oracle_mod, phi, pi + h * d, 10.0, 1.0, target)[0]
              - _loss(oracle_mod, phi, pi - h * d, 10.0, 1.0, target)[0]) / (2 * h)
        an = float(np.sum((dpi.conj() * d).real))
        assert an == pytest.approx(fd, rel=1e-6, abs=1e-9 * abs(L0))
