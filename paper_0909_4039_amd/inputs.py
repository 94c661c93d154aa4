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


def isco_radius(a: float, M: float = 1.0) -> float:
    """Prograde innermost stable circular orbit (Bardeen, Press & Teukolsky 1972)."""
    x = a / M
    z1 = 1.0 + (1.0 - x * x) ** (1.0 / 3.0) * ((1.0 + x) ** (1.0 / 3.0) + (1.0 - x) ** (1.0 / 3.0))
    z2 = np.sqrt(3.0 * x * x + z1 * z1)
    return float(M * (3.0 + z2 - np.sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2))))


def inspiral_trajectory(r_start, a, M, q, dt, n_steps, substeps=8):
    """Orbit of a slowly inspiralling particle, sampled at every half step.

    Returns an array (2 n_steps + 1, 2): row k = (r0, phi) at t = k dt / 2.
    r0(t) = (r_start^4 - (256/5) q M^3 t)^(1/4), the quadrupole
    radiation-reaction decay of a circular orbit of mass ratio q (Peters
    1964), held at the prograde ISCO once it gets there; phi(t) is the
    integral of Omega(r0) = sqrt(M) / (r0^(3/2) + a sqrt(M)), by the
    trapezoid rule on `substeps` points per half step.  q = 0 gives a fixed
    orbit with phi = Omega t.
    """
    r_isco = isco_radius(a, M)
    k = 256.0 / 5.0 * q * M ** 3
    n_half = 2 * int(n_steps) + 1
    t = np.arange((n_half - 1) * substeps + 1) * (0.5 * dt / substeps)
    r = np.maximum((r_start ** 4 - k * t) ** 0.25 if k > 0 else np.full_like(t, float(r_start)), r_isco)
    om = np.sqrt(M) / (r ** 1.5 + a * np.sqrt(M))
    h = 0.5 * dt / substeps
    phi = np.concatenate([[0.0], np.cumsum(0.5 * h * (om[1:] + om[:-1]))])
    out = np.empty((n_half, 2))
    out[:, 0] = r[::substeps]
    out[:, 1] = phi[::substeps]
    return out


def projection_weights(shape, seed):
    """Seeded complex weights with independent uniform real and imaginary parts
    in [-1, 1), for random projections <w, u> = sum conj(w) u of a state."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, shape) + 1j * rng.uniform(-1.0, 1.0, shape)
