"""Pins for the oracle's tortoise coordinate (Eq. 2) and its inverse."""
import math

import numpy as np
import pytest


@pytest.mark.parametrize("r", [2.5, 3.0, 6.0, 10.0, 57.3, 400.0])
def test_schwarzschild_closed_form(oracle_mod, r):
    # a = 0: dr*/dr = r^2/(r^2 - 2Mr) integrates to r + 2M ln(r/2M - 1)
    want = r + 2.0 * math.log(r / 2.0 - 1.0)
    assert oracle_mod.rstar_of_r(r, 0.0, 1.0) == pytest.approx(want, rel=1e-14, abs=1e-13)


@pytest.mark.parametrize("a", [0.0, 0.3, 0.6, 0.9, 0.99])
def test_derivative_matches_eq2(oracle_mod, a):
    # Eq. (2): dr*/dr = (r^2 + a^2)/Delta, checked by a central difference
    rp = 1.0 + math.sqrt(1.0 - a * a)
    for r in [rp + 0.05, rp + 0.7, 4.0, 9.0, 30.0]:
        h = 1e-5 * r
        fd = (oracle_mod.rstar_of_r(r + h, a, 1.0) - oracle_mod.rstar_of_r(r - h, a, 1.0)) / (2 * h)
        exact = (r * r + a * a) / (r * r - 2 * r + a * a)
        assert fd == pytest.approx(exact, rel=1e-7)


@pytest.mark.parametrize("a", [0.0, 0.6, 0.9, 0.99])
def test_inverse_roundtrip(oracle_mod, a):
    rp = 1.0 + math.sqrt(1.0 - a * a)
    for rs in [-100.0, -20.0, 0.0, 12.7, 150.0, 400.0]:
        d = oracle_mod.delta_of_rstar(rs, a, 1.0)
        assert d > 0.0
        from oracle import _L
        back = _L().teuko_rstar_of_delta(d, a, 1.0)
        assert back == pytest.approx(rs, abs=1e-12 * max(1.0, abs(rs)))
    # monotone
    ds = [oracle_mod.delta_of_rstar(x, a, 1.0) for x in np.linspace(-100, 400, 41)]
    assert all(x < y for x, y in zip(ds, ds[1:]))


def test_near_horizon_limit(oracle_mod):
    # a = 0: r* = 2 + delta + 2 ln(delta/2)  =>  delta ~ 2 exp((r* - 2)/2) as delta -> 0
    d = oracle_mod.delta_of_rstar(-100.0, 0.0, 1.0)
    assert d == pytest.approx(2.0 * math.exp((-100.0 - 2.0) / 2.0), rel=1e-12)
    # Kerr: r* ~ r+ + A ln(delta/2M) - B ln((r+ - r-)/2M),  A = 2M r+/(r+ - r-), B = 2M r-/(r+ - r-)
    a = 0.9
    rp, rm = 1 + math.sqrt(1 - a * a), 1 - math.sqrt(1 - a * a)
    A, B = 2 * rp / (rp - rm), 2 * rm / (rp - rm)
    want = 2.0 * math.exp((-100.0 - rp + B * math.log((rp - rm) / 2.0)) / A)
    assert oracle_mod.delta_of_rstar(-100.0, a, 1.0) == pytest.approx(want, rel=1e-9)


# Printed values of the tortoise closed form (the standard integration constant
# of Eq. 2) and of the prograde circular-orbit frequency of the source.
@pytest.mark.parametrize("r, a, want", [(10.0, 0.0, 12.772589), (10.0, 0.9, 12.783410), (8.0, 0.99, 10.219367)])
def test_rstar_printed_values(oracle_mod, r, a, want):
    assert oracle_mod.rstar_of_r(r, a, 1.0) == pytest.approx(want, abs=1e-6)


@pytest.mark.parametrize("r0, a, want", [(10.0, 0.0, 0.031623), (10.0, 0.9, 0.030748), (8.0, 0.99, 0.042342)])
def test_orbit_frequency_printed_values(oracle_mod, r0, a, want):
    o = oracle_mod.Oracle(40, 8, -30.0, 60.0, a, 1.0, 2, -2, 0.01, r0=r0, amp=1.0, rstar_obs=20.0)
    assert o.Omega == pytest.approx(want, abs=1e-6)


# Waveform extraction (the field read at a fixed r*, Sec. 2.2, Fig. 1): linear
# interpolation in r* is exact for a field linear in r*, at any theta profile.
@pytest.mark.parametrize("rstar_obs", [20.0, 20.0 + 0.37 * 90.0 / 39.0, -29.0, 58.9, 0.5 * 90.0 / 39.0 * 13 - 30.0])
def test_extraction_is_exact_for_a_field_linear_in_rstar(oracle_mod, rstar_obs):
    nr, nth, rmin, rmax = 40, 9, -30.0, 60.0
    o = oracle_mod.Oracle(nr, nth, rmin, rmax, 0.6, 1.0, 2, -2, 0.01, rstar_obs=rstar_obs)
    x = rmin + np.arange(nr) * (rmax - rmin) / (nr - 1)           # the r* nodes
    prof = np.exp(1j * np.linspace(0.3, 2.1, nth)) * (1.0 + np.arange(nth))   # any theta profile
    A, B = 0.8 - 0.3j, 0.05 + 0.11j
    phi = np.ascontiguousarray(prof[:, None] * (A + B * x[None, :]))
    w = o.extract(phi)
    want = prof * (A + B * rstar_obs)
    assert np.max(np.abs(w - want)) <= 1e-13 * np.max(np.abs(want))


def test_extraction_at_a_node_reads_the_node(oracle_mod):
    # A field with no structure in r* but node values: at a node the reading
    # is that node's value, with no weight on either neighbour.
    nr, nth, rmin, rmax = 40, 6, -30.0, 60.0
    dr = (rmax - rmin) / (nr - 1)
    rng = np.random.default_rng(11)
    phi = rng.standard_normal((nth, nr)) + 1j * rng.standard_normal((nth, nr))
    for i in (1, 17, 38):
        o = oracle_mod.Oracle(nr, nth, rmin, rmax, 0.0, 1.0, 2, -2, 0.01, rstar_obs=rmin + i * dr)
        w = o.extract(phi)
        assert np.max(np.abs(w - phi[:, i])) <= 1e-13 * np.max(np.abs(phi[:, i]))
    # a quarter of the way from node 17 to node 18
    o = oracle_mod.Oracle(nr, nth, rmin, rmax, 0.0, 1.0, 2, -2, 0.01, rstar_obs=rmin + 17.25 * dr)
    w = o.extract(phi)
    assert np.max(np.abs(w - (0.75 * phi[:, 17] + 0.25 * phi[:, 18]))) <= 1e-13 * np.max(np.abs(phi[:, 17:19]))
