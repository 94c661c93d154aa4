"""The poorly resolved r* mode of long runs, characterised on the CPU.

At a = 0 the angular operator commutes with the step, so data along a
discrete angular eigenvector Y (here l = 2, s = -2) stay along it and the
scheme reduces to a 1+1 problem in r*.  The one-step map of that problem is
assembled here as a matrix -- from the oracle's own step, projected on Y,
and from a plain 1+1 transcription of the two-stage Lax-Wendroff step
(Eqs. 13-14) that the first test ties to the oracle -- and its eigenvalues
are computed at the r* spacing of the 8192 x 256 Kerr source workload
(dr* = 500/8191 M).

Findings pinned here:
  - At small Courant numbers dt/dr* the leading eigenvector is a poorly
    resolved wave (k dr* about 1) sitting next to the potential peak.  It
    grows at 0.11 / M at dt/dr* = 0.006 (the time step of 256 theta rows
    over 1.2 million steps), faster at smaller dt/dr* and slower at larger.
    Its rate stays below max(-c_t / 2) = 1/6 / M, the anti-damping that the
    c_t term of the Pi equation (Eq. 12) gives outside r = 3M for s = -2;
    Lax-Wendroff's own damping of such waves scales with dt/dr* and loses
    to it when dt/dr* is small.  The workload's own time step (dt/dr* =
    0.0134 over 50,000 steps, 41 M) leaves it slower than the growth below.
  - The other reading of S at half points and half times (the average of S
    at the two neighbouring locations, each with centred differences)
    grows at the same rate: it is not the cure.
  - At larger dt/dr* the leading mode is smooth (frequency 0.3 / M, outside
    the peak); its rate does not change with dr* or dt, so it belongs to the
    continuum problem, and it falls as the Dirichlet outer wall moves out:
    the outgoing s = -2 wave, amplified between the peak and the wall, comes
    back from the wall.  It is not a property of the scheme.
"""
import numpy as np
import pytest

A0, M, MM, S = 0.0, 1.0, 2, -2
DR_WORKLOAD = 500.0 / 8191.0


def angular_l2(oracle_mod, nth):
    w, V = np.linalg.eig(oracle_mod.angular_matrix(nth, MM, S))
    k = int(np.argmax(w.real))          # the least negative eigenvalue: l = 2
    Y = V[:, k].real
    return float(w[k].real), Y / np.linalg.norm(Y)


def tables(oracle_mod, nr, rmin, rmax):
    dr = (rmax - rmin) / (nr - 1)
    x = rmin + np.arange(nr) * dr

    def at(xs):
        cs = [oracle_mod.coeffs(oracle_mod.delta_of_rstar(r, A0, M), np.pi / 2, A0, M, MM, S) for r in xs]
        t = {k: np.array([c[k] for c in cs]) for k in ("b", "mu", "V", "ct", "DoS2")}
        assert all(np.all(np.imag(v) == 0.0) for v in t.values())   # every coefficient is real at a = 0
        return {k: np.real(v) for k, v in t.items()}
    return dr, at(x), at(x[:-1] + 0.5 * dr)


def step_matrix(nr, dr, ci, ch, lam, dt, reading="B"):
    """The 1+1 two-stage Lax-Wendroff step on (Phi, Pi) along Y, as a matrix.
    Reading B: S at a half point from the mean and the compact difference of
    its two neighbours (the oracle's).  Reading A: the mean of S at the two
    neighbouring locations, each with a centred difference."""
    n = 2 * nr
    U = np.eye(n)
    P, Q = U[:nr], U[nr:]

    def s_pi(f, g, df, c):    # Pi row of S, Eq. (12), with Lth -> lam on Y
        return (-c["mu"][:, None] * df + (c["DoS2"] * lam)[:, None] * f - c["V"][:, None] * f
                - c["ct"][:, None] * g)

    def cdiff(f):             # centred difference, zero beyond the ends
        z = np.zeros((1, f.shape[1]))
        fz = np.vstack([z, f, z])
        return (fz[2:] - fz[:-2]) / (2 * dr)

    bh = ch["b"][:, None]
    ci_in = {k: v[1:-1] for k, v in ci.items()}
    bi = ci_in["b"][:, None]
    df, dg = (P[1:] - P[:-1]) / dr, (Q[1:] - Q[:-1]) / dr
    f, g = 0.5 * (P[1:] + P[:-1]), 0.5 * (Q[1:] + Q[:-1])
    if reading == "B":
        sp, sq = g, s_pi(f, g, df, ch)
    else:
        sn = s_pi(P, Q, cdiff(P), ci)
        sp, sq = 0.5 * (Q[1:] + Q[:-1]), 0.5 * (sn[1:] + sn[:-1])
    hP = f - 0.5 * dt * (bh * df - sp)
    hQ = g + 0.5 * dt * (bh * dg + sq)
    dF, dG = (hP[1:] - hP[:-1]) / dr, (hQ[1:] - hQ[:-1]) / dr
    F, G = 0.5 * (hP[1:] + hP[:-1]), 0.5 * (hQ[1:] + hQ[:-1])
    if reading == "B":
        sp, sq = G, s_pi(F, G, dF, ci_in)
    else:
        sh = s_pi(hP, hQ, cdiff(hP), ch)
        sp, sq = G, 0.5 * (sh[1:] + sh[:-1])
    K = np.zeros((n, n))
    K[1:nr - 1] = P[1:-1] - dt * (bi * dF - sp)
    K[nr + 1:n - 1] = Q[1:-1] + dt * (bi * dG + sq)
    return K


def modes(K, nr, rmin, dr, dt):
    """(growth rate /M, |frequency| /M, r* of the eigenvector's peak) of every
    eigenvalue, largest growth first."""
    ev, V = np.linalg.eig(K)
    out = []
    for i in np.argsort(-np.abs(ev)):
        if ev[i] == 0.0:          # the Dirichlet rows
            continue
        v = V[:nr, i]
        out.append((float(np.log(abs(ev[i])) / dt), float(abs(np.angle(ev[i])) / dt),
                    float(rmin + np.argmax(np.abs(v)) * dr)))
    return out


def test_one_dimensional_model_is_the_oracle_step(oracle_mod):
    nr, nth, rmin, rmax = 60, 8, -10.0, 20.0
    lam, Y = angular_l2(oracle_mod, nth)
    dr, ci, ch = tables(oracle_mod, nr, rmin, rmax)
    dt = 0.3 * dr
    o = oracle_mod.Oracle(nr, nth, rmin, rmax, A0, M, MM, S, dt)
    Ko = np.zeros((2 * nr, 2 * nr))
    for j in range(2 * nr):
        e = np.zeros(nr)
        e[j % nr] = 1.0
        u = [np.zeros((nth, nr), complex), np.zeros((nth, nr), complex)]
        u[j // nr][:] = Y[:, None] * e[None, :]
        p1, q1 = o.step(u[0], u[1], 0.0)
        # the step keeps the data along Y
        assert np.max(np.abs(p1 - Y[:, None] * (Y @ p1)[None, :])) < 1e-12 * max(1.0, np.max(np.abs(p1)))
        Ko[:nr, j], Ko[nr:, j] = (Y @ p1).real, (Y @ q1).real
    Km = step_matrix(nr, dr, ci, ch, lam, dt, "B")
    assert np.max(np.abs(Km - Ko)) < 1e-12 * np.max(np.abs(Ko))


@pytest.fixture(scope="module")
def window(oracle_mod):
    rmin, rmax = -10.0, 20.0
    nr = int(round((rmax - rmin) / DR_WORKLOAD)) + 1
    lam, _ = angular_l2(oracle_mod, 8)
    dr, ci, ch = tables(oracle_mod, nr, rmin, rmax)
    return nr, rmin, dr, ci, ch, lam


def grid_scale(window, ratio, reading="B"):
    nr, rmin, dr, ci, ch, lam = window
    dt = ratio * dr
    ms = modes(step_matrix(nr, dr, ci, ch, lam, dt, reading), nr, rmin, dr, dt)
    return [mo for mo in ms if mo[1] > 5.0][0]   # the fastest-growing poorly resolved wave


def test_poorly_resolved_mode_at_small_courant_numbers(oracle_mod, window):
    g6, w6, x6 = grid_scale(window, 0.006)
    assert 0.09 < g6 < 0.13, g6
    assert 12.0 < w6 < 20.0 and 0.7 < w6 * window[2] < 1.3, w6     # k dr* ~ 1
    assert 4.0 < x6 < 8.0, x6                                      # next to the potential peak
    g3 = grid_scale(window, 0.003)[0]
    g12 = grid_scale(window, 0.012)[0]
    g134 = grid_scale(window, 0.0134)[0]
    assert g3 > g6 > g12 > g134 > 0.0, (g3, g6, g12, g134)
    # the c_t anti-damping bound: -c_t/2 = 2 (r - 3M)/r^2 <= 1/6 at a = 0, s = -2
    ct = [oracle_mod.coeffs(oracle_mod.delta_of_rstar(x, A0, M), np.pi / 2, A0, M, MM, S)["ct"].real
          for x in np.linspace(-10.0, 20.0, 301)]
    bound = max(-c / 2 for c in ct)
    assert bound == pytest.approx(1.0 / 6.0, rel=1e-3)
    assert g3 < bound
    # the other reading of S at half points grows alike
    gA = grid_scale(window, 0.006, "A")[0]
    assert abs(gA - g6) < 0.02 * g6, (gA, g6)


def test_smooth_mode_belongs_to_the_walls(oracle_mod):
    lam, _ = angular_l2(oracle_mod, 8)
    out = {}
    for key, (rmin, rmax, dr0, ratio) in {"base": (-10.0, 20.0, 2 * DR_WORKLOAD, 0.1),
                                          "fine": (-10.0, 20.0, DR_WORKLOAD, 0.1),
                                          "half_dt": (-10.0, 20.0, 2 * DR_WORKLOAD, 0.05),
                                          "far_wall": (-10.0, 40.0, 2 * DR_WORKLOAD, 0.1)}.items():
        nr = int(round((rmax - rmin) / dr0)) + 1
        dr, ci, ch = tables(oracle_mod, nr, rmin, rmax)
        dt = ratio * dr
        out[key] = modes(step_matrix(nr, dr, ci, ch, lam, dt), nr, rmin, dr, dt)[0]
    g, w, x = out["base"]
    assert g > 0.0 and w < 1.0, out["base"]                       # smooth, and growing
    assert abs(out["fine"][0] - g) < 2e-3 * g and abs(out["half_dt"][0] - g) < 2e-3 * g, out
    assert out["far_wall"][0] < 0.9 * g, out
