"""Pins for the first-order system's coefficients (Eqs. 5-12).

The paper defers the matrices M, L, A to its Ref. [9].  Here Eq. (1) is
typed in as printed and the ansatz Eq. (4) with the coordinates of
Eqs. (2)-(3) is substituted symbolically; the normalised equation
  Phi_tt - b^2 Phi_** + c_t Phi_t + c_r Phi_* + V Phi - (Delta/Sigma^2) Lth Phi = ...
is then read off and compared with the oracle's coefficients, where
mu = c_r + b b_* - b c_t follows from Pi = Phi_t + b Phi_* (Eq. 5).
"""
import math
from fractions import Fraction

import pytest

sp = pytest.importorskip("sympy")


def _symbolic_eq1():
    r, a, M, m, s, S, C = sp.symbols("r a M m s S C", real=True)   # S = sin(th), C = cos(th)
    F, Fx, Fxx, Ft, Ftt, Fth, Fthth = sp.symbols("F Fx Fxx Ft Ftt Fth Fthth")
    I = sp.I
    Delta = r ** 2 - 2 * M * r + a ** 2
    w2 = r ** 2 + a ** 2
    xr = w2 / Delta                                      # Eq. (2): dr*/dr

    def Dr(e):      # d/dr at fixed t, theta, phi~ with F = F(r*(r))
        return sp.diff(e, r) + sp.diff(e, F) * xr * Fx + sp.diff(e, Fx) * xr * Fxx

    def Drt(e):     # d/dr at fixed phi acting on e^{i m phi~} e, divided by e^{i m phi~} (Eq. 3)
        return Dr(e) + I * m * a / Delta * e

    psi = r ** 3 * F                                     # Eq. (4)
    E = (-(w2 ** 2 / Delta - a ** 2 * S ** 2) * r ** 3 * Ftt
         - (4 * M * a * r / Delta) * (I * m) * r ** 3 * Ft
         - 2 * s * (r - M * (r ** 2 - a ** 2) / Delta + I * a * C) * r ** 3 * Ft
         + Delta ** (-s) * Drt(Delta ** (s + 1) * Drt(psi))
         + r ** 3 * (Fthth + C / S * Fth)
         + (1 / S ** 2 - a ** 2 / Delta) * (-m ** 2) * psi
         + 2 * s * (a * (r - M) / Delta + I * C / S ** 2) * (I * m) * psi
         - (s ** 2 * C ** 2 / S ** 2 - s) * psi)
    return (r, a, M, m, s, S, C), (F, Fx, Fxx, Ft, Ftt, Fth, Fthth), E


# rational points: (a, r, (S, C)) with S^2 + C^2 = 1 exactly
POINTS = [
    (Fraction(3, 10), Fraction(11, 2), (Fraction(4, 5), Fraction(3, 5)), -3, 0),
    (Fraction(4, 5), Fraction(39, 5), (Fraction(5, 13), Fraction(12, 13)), 3, 1),
    (Fraction(9, 10), Fraction(7, 2), (Fraction(8, 17), Fraction(-15, 17)), 2, -2),
    (Fraction(3, 5), Fraction(27, 2), (Fraction(24, 25), Fraction(-7, 25)), -4, 2),
    (Fraction(99, 100), Fraction(5, 2), (Fraction(20, 29), Fraction(21, 29)), 1, -1),
    (Fraction(0), Fraction(10), (Fraction(3, 5), Fraction(4, 5)), 2, -2),
]


@pytest.mark.parametrize("pt", POINTS)
def test_coefficients_from_eq1(oracle_mod, pt):
    (r, a, M, m, s, S, C), (F, Fx, Fxx, Ft, Ftt, Fth, Fthth), E = _symbolic_eq1()
    av, rv, (Sv, Cv), mv, sv = pt
    vals = {a: sp.Rational(av.numerator, av.denominator), r: sp.Rational(rv.numerator, rv.denominator),
            M: 1, m: mv, s: sv, S: sp.Rational(Sv.numerator, Sv.denominator),
            C: sp.Rational(Cv.numerator, Cv.denominator)}
    D = vals[r] ** 2 - 2 * vals[r] + vals[a] ** 2
    w2 = vals[r] ** 2 + vals[a] ** 2
    Sig2 = w2 ** 2 - vals[a] ** 2 * D * vals[S] ** 2        # Eq. (7)
    norm = sp.expand(E.subs(vals) / (-(Sig2 / D) * vals[r] ** 3))
    co = {k: complex(sp.N(norm.coeff(k), 30)) for k in (Ftt, Fxx, Ft, Fx, Fthth, Fth, F)}
    assert co[Ftt] == pytest.approx(1.0, abs=1e-15)
    th = math.atan2(float(Sv), float(Cv))
    rp = 1.0 + math.sqrt(1.0 - float(av) ** 2)
    got = oracle_mod.coeffs(float(rv) - rp, th, float(av), 1.0, mv, sv)
    b2 = -co[Fxx].real
    assert got["b"] ** 2 == pytest.approx(b2, rel=1e-12)
    assert got["ct"] == pytest.approx(co[Ft], rel=1e-12, abs=1e-14)
    assert got["cr"] == pytest.approx(co[Fx], rel=1e-12, abs=1e-14)
    assert got["DoS2"] == pytest.approx(-co[Fthth].real, rel=1e-12)
    # Fth coefficient is -(Delta/Sigma^2) cot(th): the cot term of Lth
    assert -got["DoS2"] * float(Cv) / float(Sv) == pytest.approx(co[Fth].real, rel=1e-12, abs=1e-15)
    # F coefficient = V - (Delta/Sigma^2)[s - (m + s cos)^2 / sin^2]
    P = sv - (mv + sv * float(Cv)) ** 2 / float(Sv) ** 2
    assert got["V"] - got["DoS2"] * P == pytest.approx(co[F], rel=1e-11, abs=1e-14)
    # b_* = d b / d r* = (Delta/w2) d b/dr, differentiated symbolically
    rr, aa, SS = sp.symbols("rr aa SS", positive=True)
    Dl = rr ** 2 - 2 * rr + aa ** 2
    bexpr = (rr ** 2 + aa ** 2) / sp.sqrt((rr ** 2 + aa ** 2) ** 2 - aa ** 2 * Dl * SS ** 2)
    bst = (Dl / (rr ** 2 + aa ** 2) * sp.diff(bexpr, rr)).subs({rr: vals[r], aa: vals[a], SS: vals[S]})
    assert got["bstar"] == pytest.approx(float(sp.N(bst, 30)), rel=1e-11, abs=1e-15)
    # mu from Pi = Phi_t + b Phi_*  (Eq. 5)
    assert got["mu"] == pytest.approx(got["cr"] + got["b"] * got["bstar"] - got["b"] * got["ct"],
                                      rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("r", [2.5, 3.0, 7.0, 25.0])
def test_schwarzschild_s_minus2_closed_forms(oracle_mod, r):
    # a = 0, s = -2: b = 1, mu = 0, c_t = c_r = -4(r-3M)/r^2, V = 6 M Delta / r^5
    c = oracle_mod.coeffs(r - 2.0, 0.7, 0.0, 1.0, 2, -2)
    D = r * r - 2 * r
    assert c["b"] == 1.0 and c["bstar"] == 0.0
    assert abs(c["mu"]) < 1e-15
    assert c["ct"] == pytest.approx(-4 * (r - 3) / r ** 2, rel=1e-13, abs=1e-16)
    assert c["cr"] == pytest.approx(-4 * (r - 3) / r ** 2, rel=1e-13, abs=1e-16)
    assert c["V"] == pytest.approx(6 * D / r ** 5, rel=1e-13)
    # general s, a = 0: mu = -4 (s + 2) Delta / r^3
    for s in (-1, 0, 1, 2):
        c = oracle_mod.coeffs(r - 2.0, 1.1, 0.0, 1.0, 3, s)
        assert c["mu"] == pytest.approx(-4 * (s + 2) * D / r ** 3, rel=1e-12, abs=1e-15)
