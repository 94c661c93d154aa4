"""Physics pin: the oracle rings down at the Schwarzschild l=2 quasinormal frequency.

a = 0, s = -2, m = 2 with the discrete l=2 angular eigenvector as profile (the
a = 0 scheme separates in theta exactly), a Gaussian pulse at r* = 20, read at
r* = 40.  A damped sinusoid is fitted (matrix pencil) in the window
t in [100, 180] M, which lies after the scattered burst and before any echo
from the r* boundaries at -100 and 300.  Two resolutions show second-order
convergence towards the classical value in tests/golden.
"""
import json
import os

import numpy as np
import pytest

from paper_0909_4039_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "schwarzschild_qnm_l2.json")))


def pencil(y, dt, order=2):
    n = len(y)
    L = n // 3
    Y = np.array([y[i:i + L + 1] for i in range(n - L)])
    U, s, Vh = np.linalg.svd(Y[:, :-1], full_matrices=False)
    U, s, Vh = U[:, :order], s[:order], Vh[:order]
    Z = np.diag(1 / s) @ U.conj().T @ Y[:, 1:] @ Vh.conj().T
    return 1j * np.log(np.linalg.eigvals(Z)) / dt


def ringdown(oracle_mod, nr, nth=16):
    rmin, rmax = -100.0, 300.0
    A = oracle_mod.angular_matrix(nth, 2, -2)
    ev, V = np.linalg.eig(A)
    k = np.argmin(np.abs(ev + 4.0))
    Y = np.real(V[:, k])
    Y /= Y[np.argmax(np.abs(Y))]
    dt = oracle_mod.stable_dt(nr, nth, rmin, rmax, 0.0, 1.0, 2, -2, 20000)
    n = int(np.ceil(190.0 / dt))
    rs, _ = inputs.grid(nr, nth, rmin, rmax)
    g = np.exp(-(rs - 20.0) ** 2 / 32.0)
    phi = (Y[:, None] * g[None, :]).astype(complex)
    pi = (Y[:, None] * (-(rs - 20.0) / 16.0 * g)[None, :]).astype(complex)
    o = oracle_mod.Oracle(nr, nth, rmin, rmax, 0.0, 1.0, 2, -2, dt, rstar_obs=40.0)
    _, _, w = o.run(phi, pi, n)
    t = np.arange(n + 1) * dt
    sel = (t >= 100.0) & (t <= 180.0)
    stride = max(1, int(0.25 / dt))
    om = pencil(w[sel, nth // 2].real[::stride], dt * stride)
    return om[np.argmax(om.real)]


def test_schwarzschild_l2_qnm(oracle_mod):
    w1 = ringdown(oracle_mod, 513)
    w2 = ringdown(oracle_mod, 1025)
    ref = GOLD["omega_re"] + 1j * GOLD["omega_im"]
    # finest grid within 1% (real part) and 3% (imaginary part)
    assert abs(w2.real - ref.real) < 0.01 * ref.real, w2
    assert abs(w2.imag - ref.imag) < 0.03 * abs(ref.imag), w2
    # second-order convergence: Richardson extrapolation lands closer still
    wx = w2 + (w2 - w1) / 3.0
    assert abs(wx.real - ref.real) < 0.005 * ref.real, wx
    assert abs(wx.imag - ref.imag) < 0.01 * abs(ref.imag), wx
