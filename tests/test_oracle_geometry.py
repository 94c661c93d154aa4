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
