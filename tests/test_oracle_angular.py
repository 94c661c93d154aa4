"""Pins for the discrete angular operator (centred differences, text after Eq. 14).

The continuous operator Lth f = f'' + cot f' + [s - (m + s cos)^2/sin^2] f has
eigenvalues -(l - s)(l + s + 1), l >= max(|m|, |s|) (spin-weighted spherical
harmonics); a second-order discretisation must reach them at O(dtheta^2).
"""
import numpy as np
import pytest

sp = pytest.importorskip("sympy")


def exact(m, s, k):
    l0 = max(abs(m), abs(s))
    return [(l - s) * (l + s + 1) for l in range(l0, l0 + k)]


def discrete(oracle_mod, nth, m, s, k):
    ev = np.linalg.eigvals(-oracle_mod.angular_matrix(nth, m, s))
    assert np.max(np.abs(ev.imag)) < 1e-6 * np.max(np.abs(ev.real))   # real spectrum
    return np.sort(ev.real)[:k]


@pytest.mark.parametrize("m,s", [(2, -2), (1, -2), (3, -2), (8, -2), (0, -2), (-2, -2),
                                 (2, 2), (1, 0), (0, 0), (2, -1), (1, 1)])
def test_spectrum_second_order(oracle_mod, m, s):
    want = np.array(exact(m, s, 3), dtype=float)
    e1 = np.abs(discrete(oracle_mod, 64, m, s, 3) - want)
    e2 = np.abs(discrete(oracle_mod, 128, m, s, 3) - want)
    assert np.all(e2 < 1e-2 * np.maximum(want, 1.0))
    ratio = e1 / e2
    exact_hit = e1 < 1e-9          # e.g. the constant mode of m = s = 0 is reproduced exactly
    assert np.all((ratio > 3.3) | exact_hit), (e1, e2, ratio)   # at least second order


@pytest.mark.parametrize("m", [1, 2, 3, 5, 8])
def test_profiles_are_eigenfunctions(oracle_mod, m):
    # continuous identity, symbolically: Lth Y_m = -(m+2)(m-1) Y_m for s = -2
    th = sp.symbols("th")
    Y = sp.sin(th) * (1 + sp.cos(th)) if m == 1 else sp.sin(th) ** (m - 2) * (1 + sp.cos(th)) ** 2
    s = -2
    L = sp.diff(Y, th, 2) + sp.cos(th) / sp.sin(th) * sp.diff(Y, th) + (s - (m + s * sp.cos(th)) ** 2 / sp.sin(th) ** 2) * Y
    lam = (max(m, 2) - s) * (max(m, 2) + s + 1)
    for x in (0.3, 1.1, 2.0, 2.9):
        assert float(sp.N((L + lam * Y).subs(th, x))) == pytest.approx(0.0, abs=1e-12)
    # discretely: the Rayleigh quotient of the sampled profile converges to lambda at O(h^2)
    from paper_0909_4039_amd.inputs import angular_profile
    errs = []
    for nth in (64, 128):
        t = (np.arange(nth) + 0.5) * np.pi / nth
        y = angular_profile(t, m).astype(complex)
        Ly = oracle_mod.angular_apply(y, m, s)
        w = np.sin(t)   # the operator is symmetric in the sin(theta)-weighted inner product
        q = -np.sum(w * y.conj() * Ly).real / np.sum(w * np.abs(y) ** 2)
        errs.append(abs(q - lam))
    assert errs[1] < 1e-3 * lam and errs[0] / errs[1] > 3.3


def test_ghost_sign_rule(oracle_mod):
    # the pole ghost mirrors with sign (-1)^|m+s|: a constant column is annihilated by
    # the second difference at row 0 only for the even (Neumann) rule
    nth = 16
    f = np.ones(nth, complex)
    dth = np.pi / nth
    th0 = 0.5 * dth
    for m, s, even in [(2, -2, True), (1, -2, False), (0, 0, True), (1, 1, True)]:
        out = oracle_mod.angular_apply(f, m, s)
        P = s - (m + s * np.cos(th0)) ** 2 / np.sin(th0) ** 2
        sig = 1.0 if even else -1.0
        fp, fm = 1.0, sig
        want = (fp - 2 + fm) / dth ** 2 + np.cos(th0) / np.sin(th0) * (fp - fm) / (2 * dth) + P
        assert out[0].real == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("m,s", [(2, -2), (1, -2), (3, -1), (0, 2)])
def test_a0_evolution_stays_separable(oracle_mod, m, s):
    # a = 0: every coefficient but Lth is independent of theta, so data along a
    # discrete angular eigenvector Y stays Y(theta) R(r*, t) for all time: the
    # ratio Phi / Y must be the same in every row (to rounding).
    nr, nth, rmin, rmax = 90, 20, -30.0, 60.0
    A = oracle_mod.angular_matrix(nth, m, s)
    ev, V = np.linalg.eig(A)
    k = np.argmax(ev.real)                   # the least negative eigenvalue (lowest l)
    Y = np.real(V[:, k])
    Y /= Y[np.argmax(np.abs(Y))]
    rs = rmin + np.arange(nr) * (rmax - rmin) / (nr - 1)
    g = np.exp(-(rs - 10.0) ** 2 / 18.0) * (1.0 + 0.5j)
    phi = (Y[:, None] * g[None, :]).astype(complex)
    pi = (Y[:, None] * (-(rs - 10.0) / 9.0 * g)[None, :]).astype(complex)
    dt = oracle_mod.stable_dt(nr, nth, rmin, rmax, 0.0, 1.0, m, s, 2000)
    o = oracle_mod.Oracle(nr, nth, rmin, rmax, 0.0, 1.0, m, s, dt)
    p, q, _ = o.run(phi, pi, 300, record=False)
    jr = int(np.argmax(np.abs(Y)))             # reference row: largest |Y|
    for f in (p, q):
        # f must equal Y(theta) R(r*), with R read off the reference row
        resid = np.max(np.abs(f - Y[:, None] * (f[jr] / Y[jr])[None, :]))
        assert resid <= 1e-12 * np.max(np.abs(f)), resid
