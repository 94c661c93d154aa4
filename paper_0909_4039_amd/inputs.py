"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module holds no arithmetic of the method: only grid coordinates, seeded
random numbers and analytic initial profiles (a Gaussian pulse in r* times a
spin-weighted angular profile).  Both sides receive the arrays it produces.
"""
from __future__ import annotations

import numpy as np


def grid(nr: int, nth: int, rstar_min: float, rstar_max: float):
    """r* nodes r*_i = r*_min + i dr* and cell-centred theta_j = (j + 1/2) pi / nth."""
    dr = (rstar_max - rstar_min) / (nr - 1)
    rs = rstar_min + np.arange(nr) * dr
    th = (np.arange(nth) + 0.5) * np.pi / nth
    return rs, th


def angular_profile(theta: np.ndarray, m: int) -> np.ndarray:
    """s = -2 profile: sin^{m-2}(th)(1+cos th)^2 for m >= 2, sin(th)(1+cos th) for m = 1.

    Negative m uses the mirror image theta -> pi - theta; m = 0 uses the m = 2 form.
    """
    mm = abs(m)
    th = theta if m >= 0 else np.pi - theta
    if mm == 1:
        return np.sin(th) * (1.0 + np.cos(th))
    k = max(mm, 2) - 2
    return np.sin(th) ** k * (1.0 + np.cos(th)) ** 2


def seeded_amplitude(seed: int) -> float:
    """A = 1 + 0.1 (2U - 1), U ~ U[0,1) from numpy's default_rng(seed)."""
    return 1.0 + 0.1 * (2.0 * np.random.default_rng(seed).random() - 1.0)


def pulse(nr, nth, rstar_min, rstar_max, m, center, width, amplitude):
    """Phi0 = A exp(-(r*-c)^2/(2 w^2)) Y_m(theta);  Pi0 = d Phi0 / d r* (analytic).

    Returns complex128 arrays of shape (nth, nr) (theta rows, r* contiguous).
    """
    rs, th = grid(nr, nth, rstar_min, rstar_max)
    g = amplitude * np.exp(-((rs - center) ** 2) / (2.0 * width ** 2))
    dg = -(rs - center) / width ** 2 * g
    Y = angular_profile(th, m)
    phi = (Y[:, None] * g[None, :]).astype(np.complex128)
    pi = (Y[:, None] * dg[None, :]).astype(np.complex128)
    return phi, pi


def random_state(nr, nth, seed, scale=1.0):
    """Independent N(0,1) real and imaginary parts for Phi and Pi (parity tests)."""
    rng = np.random.default_rng(seed)
    f = lambda: (rng.standard_normal((nth, nr)) + 1j * rng.standard_normal((nth, nr))) * scale
    return f(), f()


def smooth_random_state(nr, nth, rstar_min, rstar_max, seed, n_modes=4):
    """A seeded sum of a few Gaussian pulses with random centres, widths and phases."""
    rng = np.random.default_rng(seed)
    phi = np.zeros((nth, nr), np.complex128)
    pi = np.zeros((nth, nr), np.complex128)
    rs, th = grid(nr, nth, rstar_min, rstar_max)
    span = rstar_max - rstar_min
    for _ in range(n_modes):
        c = rstar_min + span * (0.2 + 0.6 * rng.random())
        w = span * (0.02 + 0.05 * rng.random())
        ph = np.exp(2j * np.pi * rng.random())
        l = rng.integers(0, 4)
        Y = np.cos(l * th) * (1.0 + 0.3 * rng.standard_normal())
        g = np.exp(-((rs - c) ** 2) / (2 * w * w))
        phi += ph * Y[:, None] * g[None, :]
        pi += (rng.standard_normal() + 1j * rng.standard_normal()) * 0.3 * Y[:, None] * g[None, :]
    return phi, pi
