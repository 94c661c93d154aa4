/*
 * Plain FP64 CPU oracle for the m-mode 2+1 Teukolsky time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the
 * benchmark's CPU-baseline leg can check the GPU library against a slow,
 * obviously correct implementation written straight from the paper
 * (Khanna & McKennon, "An exploration of CUDA and CBEA for a gravitational
 * wave source-modelling application").  It shares no code, header or table
 * with the HIP library.
 *
 * What is computed, and where it comes from:
 *   - Eq. (2): tortoise coordinate dr* / dr = (r^2+a^2) / Delta.  The paper gives
 *     no integration constant; the reading used here is the standard closed
 *     form r* = r + 2M r+/(r+ - r-) ln((r - r+)/2M) - 2M r-/(r+ - r-) ln((r - r-)/2M).
 *     The inverse r(r*) is found by bisection on ln(r - r+), and Delta is
 *     formed as delta*(delta + r+ - r-) so that it keeps full relative
 *     precision next to the horizon.
 *   - Eqs. (4)-(12): the first-order system.  The paper defers the matrices
 *     M, L, A to its Ref. [9]; they are re-derived here by substituting the
 *     ansatz Psi = e^{i m phi~} r^3 Phi(t,r*,theta) into Eq. (1) and dividing
 *     by -(Sigma^2/Delta) r^3 e^{i m phi~}.  With Pi = d_t Phi + b d_* Phi:
 *        d_t Phi + b d_* Phi = Pi
 *        d_t Pi  - b d_* Pi  = T - mu d_* Phi + (Delta/Sigma^2) Lth Phi - V Phi - c_t Pi
 *     so D = diag(b, b, -b, -b) (Eq. 11) and S_Phi = Pi,
 *     S_Pi = T - mu d_*Phi + (Delta/Sigma^2) Lth Phi - V Phi - c_t Pi (Eq. 12).
 *        Lth f = f'' + cot(th) f' + [s - (m + s cos th)^2 / sin^2 th] f
 *        c_t = [2s(r Delta - M(r^2-a^2)) + i(4 M a m r + 2 s a Delta cos th)] / Sigma^2
 *        c_r = -[6 w2 Delta/r + 2 r Delta + 2 s (r-M) w2 + 2 i m a w2] / Sigma^2
 *        V   = -[Delta(6 Delta/r^2 + 6(1+s)(r-M)/r + 6 i m a/r) + 4 i s m a (r-M)] / Sigma^2
 *        b_* = d b/d r* = a^2 Delta sin^2 th [(r-M) w2 - 2 r Delta] / (w2 Sigma^3)
 *        mu  = c_r + b b_* - b c_t,     w2 = r^2 + a^2,  b = w2/Sigma  (Eqs. 6-7)
 *   - Eqs. (13)-(14): two-step Lax-Wendroff.  Where the paper is silent about
 *     S at half points the reading is: S^n_{i+1/2} is evaluated on the mean
 *     (u_i + u_{i+1})/2 with the compact difference (u_{i+1}-u_i)/dr* and the
 *     coefficients at r*_{i+1/2}; S^{n+1/2}_i on the mean of the two
 *     neighbouring half-point values with their compact difference and the
 *     coefficients at r*_i.  The source enters at t^n (predictor) and
 *     t^n + dt/2 (corrector).
 *   - Angular derivatives: second-order centred differences (text after
 *     Eq. 14) on a cell-centred grid theta_j = (j + 1/2) pi / N_theta.
 *   - Boundary conditions (text after Eq. 14): Phi = Pi = 0 on the first and
 *     last r* node; at the poles the ghost cell mirrors the first cell with
 *     sign (-1)^|m| (Neumann for even |m|, Dirichlet for odd |m|), for Phi,
 *     Pi and the half-step values.  The paper states the rule for even s
 *     (s = +-2); the sign used is (-1)^|m+s|, which equals (-1)^|m| for even
 *     s and follows the pole behaviour theta^|m+s| of the spin-weighted
 *     harmonics for odd s.
 *   - Source: the paper does not print its T (it points to Ref. [14]); the
 *     stand-in is a unit-peak Gaussian in (r*, theta) centred on r*(r0) and
 *     theta = pi/2, times e^{-i m Omega t}, with Omega = sqrt(M)/(r0^{3/2} + a sqrt(M)),
 *     added to the Pi row of S.
 *   - Moving source (an inspiral, as in the paper's Fig. 1): the orbit is
 *     given as input, a table of (r0, phi) at every half step; the source
 *     is the same Gaussian centred on r*(r0(t)) with phase e^{-i m phi(t)},
 *     evaluated at t^n (predictor) and t^n + dt/2 (corrector).  With
 *     phi = Omega t and r0 fixed it is the static source.
 *   - Waveform: linear interpolation of Phi in r* at r*_obs, for every theta.
 *   - Adjoint: the exact transpose of one step in the real 4-component view
 *     (Eq. 9), written out by hand in reverse order, and the source-parameter
 *     gradients it induces: dL/dr0 and dL/damp for the static source, and
 *     dL/dr0_e, dL/dphi_e for every entry e of a moving source's orbit table.
 *
 * The grid may be held as a window (rows j0..j0+nj-1, columns i0..i0+ni-1 of
 * the full grid).  A neighbour that lies inside the full grid but outside the
 * window reads as NaN, so every value that depends on missing data becomes
 * NaN and only the exact domain of dependence survives.
 *
 * Parity status: the coefficient forms, the angular operator, the tortoise
 * map (and its printed values), the waveform extraction (exact for a field
 * linear in r*, node values at nodes), the scheme's order of accuracy, the Schwarzschild l=2 ringdown, the
 * Kerr a = 0.5 l = m = 2 ringdown (which depends on every a-dependent
 * coefficient), the m -> -m mirror symmetry, the adjoint and the
 * moving-source gradients (central differences of the forward run) are
 * pinned by tests.  Kerr pointwise values have no printed reference; they are pinned
 * through the Kerr ringdown and the invariants above.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct {
    int64_t nr, nth;            /* full grid: r* nodes, theta cells              */
    double rstar_min, rstar_max;
    int64_t i0, ni, j0, nj;     /* window held in memory                         */
    double a, M;
    int32_t m, s;
    double dt;
    double r0, amp, sigma_r_cells, sigma_th_cells;   /* source (amp = 0: none)   */
    double rstar_obs;
} teuko_params;

/* ---------------------------------------------------------------- Eq. (2) */

static void horizons(double a, double M, double* rp, double* rm) {
    double q = sqrt(M * M - a * a);
    *rp = M + q;
    *rm = M - q;
}

/* r* as a function of delta = r - r+ (keeps precision next to the horizon). */
double teuko_rstar_of_delta(double delta, double a, double M) {
    double rp, rm;
    horizons(a, M, &rp, &rm);
    double r = rp + delta;
    double A = 2.0 * M * rp / (rp - rm);
    double B = 2.0 * M * rm / (rp - rm);
    double out = r + A * log(delta / (2.0 * M));
    if (B != 0.0) out -= B * log((delta + (rp - rm)) / (2.0 * M));
    return out;
}

double teuko_rstar_of_r(double r, double a, double M) {
    double rp, rm;
    horizons(a, M, &rp, &rm);
    return teuko_rstar_of_delta(r - rp, a, M);
}

/* Inverse of Eq. (2): delta = r - r+ for given r*, by bisection on ln(delta). */
double teuko_delta_of_rstar(double rstar, double a, double M) {
    double lo = -50.0, hi = 10.0;
    while (lo > -740.0 && teuko_rstar_of_delta(exp(lo), a, M) > rstar) lo -= 50.0;
    while (teuko_rstar_of_delta(exp(hi), a, M) < rstar) hi += 10.0;
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (teuko_rstar_of_delta(exp(mid), a, M) < rstar) lo = mid; else hi = mid;
    }
    double dlo = exp(lo), dhi = exp(hi);
    double flo = fabs(teuko_rstar_of_delta(dlo, a, M) - rstar);
    double fhi = fabs(teuko_rstar_of_delta(dhi, a, M) - rstar);
    return flo <= fhi ? dlo : dhi;
}

/* ------------------------------------------------------- Eqs. (5)-(12) */

typedef struct {
    double b;        /* Eq. (6) */
    double bstar;    /* d b / d r* */
    cplx ct, cr, V, mu;
    double DoS2;     /* Delta / Sigma^2 */
} coeffs;

static coeffs coeffs_at(double r, double Delta, double th, double a, double M, int m, int s) {
    coeffs c;
    double w2 = r * r + a * a;
    double sn = sin(th), cs = cos(th);
    double S2 = w2 * w2 - a * a * Delta * sn * sn;     /* Eq. (7) */
    double Sig = sqrt(S2);
    c.b = w2 / Sig;
    c.ct = (2.0 * s * (r * Delta - M * (r * r - a * a))
            + I * (4.0 * M * a * m * r + 2.0 * s * a * Delta * cs)) / S2;
    c.cr = -(6.0 * w2 * Delta / r + 2.0 * r * Delta + 2.0 * s * (r - M) * w2
             + 2.0 * I * m * a * w2) / S2;
    c.V = -(Delta * (6.0 * Delta / (r * r) + 6.0 * (1.0 + s) * (r - M) / r + 6.0 * I * m * a / r)
            + 4.0 * I * s * m * a * (r - M)) / S2;
    c.bstar = a * a * Delta * sn * sn * ((r - M) * w2 - 2.0 * r * Delta) / (w2 * S2 * Sig);
    c.mu = c.cr + c.b * c.bstar - c.b * c.ct;
    c.DoS2 = Delta / S2;
    return c;
}

/* Exported for the coefficient tests: out = b, b_*, Re/Im c_t, Re/Im c_r,
   Re/Im V, Re/Im mu, Delta/Sigma^2.  delta = r - r+. */
void teuko_coeffs(double delta, double th, double a, double M, int m, int s, double* out) {
    double rp, rm;
    horizons(a, M, &rp, &rm);
    double r = rp + delta;
    double Delta = delta * (delta + (rp - rm));
    coeffs c = coeffs_at(r, Delta, th, a, M, m, s);
    out[0] = c.b; out[1] = c.bstar;
    out[2] = creal(c.ct); out[3] = cimag(c.ct);
    out[4] = creal(c.cr); out[5] = cimag(c.cr);
    out[6] = creal(c.V); out[7] = cimag(c.V);
    out[8] = creal(c.mu); out[9] = cimag(c.mu);
    out[10] = c.DoS2;
}

/* ------------------------------------------------------------- context */

typedef struct {
    teuko_params p;
    double dr, dth;
    double sigma;              /* ghost sign (-1)^|m| */
    double rstar0, Omega;      /* source centre and orbital frequency */
    double* th;                /* [nj]   theta of held rows                     */
    coeffs* ci;                /* [nj*ni] coefficients at integer points        */
    coeffs* ch;                /* [nj*ni] coefficients at half points i+1/2     */
    double* gi;                /* [nj*ni] source spatial factor, integer points */
    double* gh;                /* [nj*ni] source spatial factor, half points    */
    double* xi;                /* [ni]  r*_i - r*0   (for d/dr0)                */
    double* xh;                /* [ni]  r*_{i+1/2} - r*0                        */
    /* work */
    cplx *Pb, *Qb, *dP, *dQ, *LP, *hP, *hQ;
    int64_t iobs; double alpha; /* observer: column (full grid) and weight     */
    /* moving source: (r0, phi) at t = traj_t0 + k dt/2, k < traj_n (NULL: static) */
    double* traj;
    int64_t traj_n;
    double traj_t0;
} teuko_ctx;

static double theta_of(const teuko_ctx* c, int64_t J) { return (J + 0.5) * c->dth; }

void teuko_destroy(teuko_ctx* c) {
    if (!c) return;
    free(c->th); free(c->ci); free(c->ch); free(c->gi); free(c->gh); free(c->xi); free(c->xh);
    free(c->traj);
    free(c->Pb); free(c->Qb); free(c->dP); free(c->dQ); free(c->LP); free(c->hP); free(c->hQ);
    free(c);
}

teuko_ctx* teuko_create(const teuko_params* p) {
    if (p->nr < 4 || p->nth < 4 || p->ni < 1 || p->nj < 1) return NULL;
    if (p->i0 < 0 || p->j0 < 0 || p->i0 + p->ni > p->nr || p->j0 + p->nj > p->nth) return NULL;
    if (!(p->a >= 0.0 && p->a < p->M)) return NULL;
    teuko_ctx* c = (teuko_ctx*)calloc(1, sizeof(teuko_ctx));
    c->p = *p;
    int64_t ni = p->ni, nj = p->nj, n = ni * nj;
    c->dr = (p->rstar_max - p->rstar_min) / (double)(p->nr - 1);
    c->dth = M_PI / (double)p->nth;
    c->sigma = (abs(p->m + p->s) % 2 == 0) ? 1.0 : -1.0;
    c->th = (double*)malloc(sizeof(double) * nj);
    c->ci = (coeffs*)malloc(sizeof(coeffs) * n);
    c->ch = (coeffs*)malloc(sizeof(coeffs) * n);
    c->gi = (double*)calloc(n, sizeof(double));
    c->gh = (double*)calloc(n, sizeof(double));
    c->xi = (double*)calloc(ni, sizeof(double));
    c->xh = (double*)calloc(ni, sizeof(double));
    c->Pb = (cplx*)malloc(sizeof(cplx) * n); c->Qb = (cplx*)malloc(sizeof(cplx) * n);
    c->dP = (cplx*)malloc(sizeof(cplx) * n); c->dQ = (cplx*)malloc(sizeof(cplx) * n);
    c->LP = (cplx*)malloc(sizeof(cplx) * n);
    c->hP = (cplx*)malloc(sizeof(cplx) * n); c->hQ = (cplx*)malloc(sizeof(cplx) * n);

    double rp, rm;
    horizons(p->a, p->M, &rp, &rm);
    for (int64_t jj = 0; jj < nj; ++jj) c->th[jj] = theta_of(c, p->j0 + jj);

    /* the source geometry is set up whenever r0 lies outside the horizon, so
       that d/d(amp) is available also at amp = 0 */
    int has_src = p->r0 > rp;
    c->rstar0 = 0.0; c->Omega = 0.0;
    if (has_src) {
        c->rstar0 = teuko_rstar_of_r(p->r0, p->a, p->M);
        c->Omega = sqrt(p->M) / (pow(p->r0, 1.5) + p->a * sqrt(p->M));
    }
    double sr = p->sigma_r_cells * c->dr, st = p->sigma_th_cells * c->dth;

    for (int64_t ii = 0; ii < ni; ++ii) {
        int64_t Ig = p->i0 + ii;
        double xs_i = p->rstar_min + Ig * c->dr;
        double xs_h = p->rstar_min + (Ig + 0.5) * c->dr;
        double d_i = teuko_delta_of_rstar(xs_i, p->a, p->M);
        double d_h = teuko_delta_of_rstar(xs_h, p->a, p->M);
        double r_i = rp + d_i, D_i = d_i * (d_i + (rp - rm));
        double r_h = rp + d_h, D_h = d_h * (d_h + (rp - rm));
        c->xi[ii] = xs_i - c->rstar0;
        c->xh[ii] = xs_h - c->rstar0;
        for (int64_t jj = 0; jj < nj; ++jj) {
            double th = c->th[jj];
            c->ci[jj * ni + ii] = coeffs_at(r_i, D_i, th, p->a, p->M, p->m, p->s);
            c->ch[jj * ni + ii] = coeffs_at(r_h, D_h, th, p->a, p->M, p->m, p->s);
            if (has_src) {
                double gth = exp(-(th - 0.5 * M_PI) * (th - 0.5 * M_PI) / (2.0 * st * st));
                c->gi[jj * ni + ii] = exp(-(xs_i - c->rstar0) * (xs_i - c->rstar0) / (2.0 * sr * sr)) * gth;
                c->gh[jj * ni + ii] = exp(-(xs_h - c->rstar0) * (xs_h - c->rstar0) / (2.0 * sr * sr)) * gth;
            }
        }
    }
    /* observer: r*_obs = r*_{iobs} + alpha dr*, linear interpolation in r* */
    c->iobs = (int64_t)floor((p->rstar_obs - p->rstar_min) / c->dr);
    if (c->iobs < 0) c->iobs = 0;
    if (c->iobs > p->nr - 2) c->iobs = p->nr - 2;
    c->alpha = (p->rstar_obs - (p->rstar_min + c->iobs * c->dr)) / c->dr;
    return c;
}

/* -------------------------------------------------- angular operator Lth */

/* f_{J+dj} for a column held with row stride `stride`; ghost rule at the
   poles (cell-centred mirror with sign (-1)^|m|), NaN outside the window. */
static cplx row_nb(const teuko_ctx* c, const cplx* col, int64_t stride, int64_t jj, int dj) {
    int64_t J = c->p.j0 + jj + dj;
    if (J < 0) return c->sigma * col[(0 - c->p.j0) * stride];          /* row 0 held */
    if (J >= c->p.nth) return c->sigma * col[(c->p.nth - 1 - c->p.j0) * stride];
    int64_t k = jj + dj;
    if (k < 0 || k >= c->p.nj) return NAN;
    return col[k * stride];
}

/* Lth f at held row jj: f'' + cot(th) f' + [s - (m + s cos th)^2/sin^2 th] f,
   second-order centred differences. */
static cplx angular_at(const teuko_ctx* c, const cplx* col, int64_t stride, int64_t jj) {
    double th = c->th[jj], h = c->dth;
    double sn = sin(th), cs = cos(th);
    cplx fp = row_nb(c, col, stride, jj, +1);
    cplx f0 = col[jj * stride];
    cplx fm = row_nb(c, col, stride, jj, -1);
    double P = c->p.s - (c->p.m + c->p.s * cs) * (c->p.m + c->p.s * cs) / (sn * sn);
    return (fp - 2.0 * f0 + fm) / (h * h) + (cs / sn) * (fp - fm) / (2.0 * h) + P * f0;
}

/* Exported for the spectrum tests: apply Lth to one full column f[nth]. */
void teuko_angular_apply(int64_t nth, int32_t m, int32_t s, const double* f_ri, double* out_ri) {
    teuko_params p;
    memset(&p, 0, sizeof(p));
    p.nr = 4; p.nth = nth; p.rstar_min = 0; p.rstar_max = 1;
    p.i0 = 0; p.ni = 1; p.j0 = 0; p.nj = nth; p.a = 0; p.M = 1; p.m = m; p.s = s;
    teuko_ctx c;
    memset(&c, 0, sizeof(c));
    c.p = p;
    c.dth = M_PI / (double)nth;
    c.sigma = (abs(m + s) % 2 == 0) ? 1.0 : -1.0;
    c.th = (double*)malloc(sizeof(double) * nth);
    for (int64_t j = 0; j < nth; ++j) c.th[j] = theta_of(&c, j);
    const cplx* f = (const cplx*)f_ri;
    cplx* o = (cplx*)out_ri;
    for (int64_t j = 0; j < nth; ++j) o[j] = angular_at(&c, f, 1, j);
    free(c.th);
}

/* -------------------------------------------------------------- source */

static cplx phase(const teuko_ctx* c, double t) {
    return cexp(-I * (double)c->p.m * c->Omega * t);
}

/* --------------------------------------------------- Eqs. (13)-(14) */

/* u(i) at column ii+di of held row: NaN outside the window. */
static cplx col_nb(const teuko_ctx* c, const cplx* f, int64_t jj, int64_t ii, int di) {
    int64_t k = ii + di;
    if (k < 0 || k >= c->p.ni) return NAN;
    return f[jj * c->p.ni + k];
}

/* Moving source: set the orbit table (copied).  Entry k holds (r0, phi) at
   t = t0 + k dt/2.  NULL clears it.  Returns -1 for an invalid table. */
int teuko_set_trajectory(teuko_ctx* c, const double* r0_phi, int64_t n_half, double t0) {
    free(c->traj);
    c->traj = NULL;
    c->traj_n = 0;
    if (!r0_phi) return 0;
    double rp, rm;
    horizons(c->p.a, c->p.M, &rp, &rm);
    if (n_half < 2) return -1;
    for (int64_t k = 0; k < n_half; ++k)
        if (!(r0_phi[2 * k] > rp) || !isfinite(r0_phi[2 * k + 1])) return -1;
    c->traj = (double*)malloc(sizeof(double) * 2 * n_half);
    memcpy(c->traj, r0_phi, sizeof(double) * 2 * n_half);
    c->traj_n = n_half;
    c->traj_t0 = t0;
    return 0;
}

/* Unit-amplitude source at row jj of a point at r* = xs for an orbit at
   (r0, phi): exp(-(r* - r*(r0))^2 / (2 sr^2)) exp(-(th - pi/2)^2 / (2 sth^2)) e^{-i m phi}. */
static cplx moving_unit(const teuko_ctx* c, double xs, int64_t jj, double r0, double phi) {
    const teuko_params* p = &c->p;
    double sr = p->sigma_r_cells * c->dr, st = p->sigma_th_cells * c->dth;
    double x = xs - teuko_rstar_of_r(r0, p->a, p->M);
    double th = c->th[jj];
    double gth = exp(-(th - 0.5 * M_PI) * (th - 0.5 * M_PI) / (2.0 * st * st));
    return (exp(-x * x / (2.0 * sr * sr)) * gth) * cexp(-I * (double)p->m * phi);
}

/* T = amp times the unit source. */
static cplx moving_T(const teuko_ctx* c, double xs, int64_t jj, double r0, double phi) {
    return c->p.amp * moving_unit(c, xs, jj, r0, phi);
}

int teuko_step(teuko_ctx* c, const double* phi_ri, const double* pi_ri,
               double* phi_out_ri, double* pi_out_ri, double t) {
    const teuko_params* p = &c->p;
    const cplx* Phi = (const cplx*)phi_ri;
    const cplx* Pi = (const cplx*)pi_ri;
    cplx* Phi1 = (cplx*)phi_out_ri;
    cplx* Pi1 = (cplx*)pi_out_ri;
    int64_t ni = p->ni, nj = p->nj;
    double dt = p->dt, dr = c->dr;
    cplx ph0 = phase(c, t), ph1 = phase(c, t + 0.5 * dt);
    /* moving source: table entries at t (predictor) and t + dt/2 (corrector) */
    const double* oa = NULL;
    const double* ob = NULL;
    if (c->traj) {
        int64_t k = llround((t - c->traj_t0) / (0.5 * dt));
        if (k < 0 || k + 1 >= c->traj_n) return -1;
        oa = c->traj + 2 * k;
        ob = c->traj + 2 * (k + 1);
    }

    /* predictor, Eq. (13): half points ii+1/2 (index ii), time n+1/2 */
    #pragma omp parallel for schedule(static)
    for (int64_t jj = 0; jj < nj; ++jj)
        for (int64_t ii = 0; ii < ni; ++ii) {
            int64_t k = jj * ni + ii;
            cplx P0 = Phi[k], P1 = col_nb(c, Phi, jj, ii, +1);
            cplx Q0 = Pi[k], Q1 = col_nb(c, Pi, jj, ii, +1);
            c->Pb[k] = 0.5 * (P0 + P1);
            c->Qb[k] = 0.5 * (Q0 + Q1);
            c->dP[k] = (P1 - P0) / dr;
            c->dQ[k] = (Q1 - Q0) / dr;
        }
    #pragma omp parallel for schedule(static)
    for (int64_t jj = 0; jj < nj; ++jj)
        for (int64_t ii = 0; ii < ni; ++ii) {
            int64_t k = jj * ni + ii;
            const coeffs* q = &c->ch[k];
            cplx L = angular_at(c, c->Pb + ii, ni, jj);
            cplx T = oa ? moving_T(c, p->rstar_min + (p->i0 + ii + 0.5) * dr, jj, oa[0], oa[1])
                        : p->amp * c->gh[k] * ph0;
            cplx SPhi = c->Qb[k];
            cplx SPi = T - q->mu * c->dP[k] + q->DoS2 * L - q->V * c->Pb[k] - q->ct * c->Qb[k];
            c->hP[k] = c->Pb[k] - 0.5 * dt * (q->b * c->dP[k] - SPhi);
            c->hQ[k] = c->Qb[k] - 0.5 * dt * (-q->b * c->dQ[k] - SPi);
        }
    /* corrector, Eq. (14): integer points, time n+1.  Half point ii-1/2 has index ii-1. */
    #pragma omp parallel for schedule(static)
    for (int64_t jj = 0; jj < nj; ++jj)
        for (int64_t ii = 0; ii < ni; ++ii) {
            int64_t k = jj * ni + ii;
            cplx hPm = col_nb(c, c->hP, jj, ii, -1), hQm = col_nb(c, c->hQ, jj, ii, -1);
            c->Pb[k] = 0.5 * (c->hP[k] + hPm);
            c->Qb[k] = 0.5 * (c->hQ[k] + hQm);
            c->dP[k] = (c->hP[k] - hPm) / dr;
            c->dQ[k] = (c->hQ[k] - hQm) / dr;
        }
    #pragma omp parallel for schedule(static)
    for (int64_t jj = 0; jj < nj; ++jj)
        for (int64_t ii = 0; ii < ni; ++ii) {
            int64_t k = jj * ni + ii;
            int64_t Ig = p->i0 + ii;
            if (Ig == 0 || Ig == p->nr - 1) { Phi1[k] = 0.0; Pi1[k] = 0.0; continue; }
            const coeffs* q = &c->ci[k];
            cplx L = angular_at(c, c->Pb + ii, ni, jj);
            cplx T = ob ? moving_T(c, p->rstar_min + (p->i0 + ii) * dr, jj, ob[0], ob[1])
                        : p->amp * c->gi[k] * ph1;
            cplx SPhi = c->Qb[k];
            cplx SPi = T - q->mu * c->dP[k] + q->DoS2 * L - q->V * c->Pb[k] - q->ct * c->Qb[k];
            Phi1[k] = Phi[k] - dt * (q->b * c->dP[k] - SPhi);
            Pi1[k] = Pi[k] - dt * (-q->b * c->dQ[k] - SPi);
        }
    return 0;
}

/* ---------------------------------------------------------- waveform */

/* w_j = (1-alpha) Phi_{iobs,j} + alpha Phi_{iobs+1,j}; needs both columns held. */
int teuko_extract(const teuko_ctx* c, const double* phi_ri, double* out_ri) {
    const cplx* Phi = (const cplx*)phi_ri;
    cplx* o = (cplx*)out_ri;
    int64_t k0 = c->iobs - c->p.i0;
    if (k0 < 0 || k0 + 1 >= c->p.ni) return -1;
    for (int64_t jj = 0; jj < c->p.nj; ++jj)
        o[jj] = (1.0 - c->alpha) * Phi[jj * c->p.ni + k0] + c->alpha * Phi[jj * c->p.ni + k0 + 1];
    return 0;
}

/* Run n steps from time t0 = t_start (t^k = t_start + k dt).  phi/pi are
   updated in place.  wave (may be NULL) receives w^0 .. w^n: (n+1) x nj. */
int teuko_run(teuko_ctx* c, double* phi_ri, double* pi_ri, int64_t n, double t_start, double* wave_ri) {
    int64_t N = c->p.ni * c->p.nj;
    double* a1 = (double*)malloc(sizeof(cplx) * N);
    double* b1 = (double*)malloc(sizeof(cplx) * N);
    if (wave_ri && teuko_extract(c, phi_ri, wave_ri) != 0) { free(a1); free(b1); return -1; }
    for (int64_t k = 0; k < n; ++k) {
        if (teuko_step(c, phi_ri, pi_ri, a1, b1, t_start + (double)k * c->p.dt) != 0) {
            free(a1); free(b1);
            return -1;
        }
        memcpy(phi_ri, a1, sizeof(cplx) * N);
        memcpy(pi_ri, b1, sizeof(cplx) * N);
        if (wave_ri) teuko_extract(c, phi_ri, wave_ri + 2 * (k + 1) * c->p.nj);
    }
    free(a1); free(b1);
    return 0;
}

/* ------------------------------------------------------------- adjoint */

/* Transpose (in the real 4-component view) of Lth applied over rows, added
   into out: out[j'] += A_{j j'} y[j] for every row j.  The angular
   coefficients are real, so the transpose needs no conjugation. */
static void angular_transpose_add(const teuko_ctx* c, const cplx* y, int64_t ni, int64_t ii, cplx* out) {
    int64_t nj = c->p.nj;
    double h = c->dth;
    for (int64_t jj = 0; jj < nj; ++jj) {
        cplx v = y[jj * ni + ii];
        if (v == 0.0) continue;
        double th = c->th[jj], sn = sin(th), cs = cos(th);
        double P = c->p.s - (c->p.m + c->p.s * cs) * (c->p.m + c->p.s * cs) / (sn * sn);
        double wp = 1.0 / (h * h) + (cs / sn) / (2.0 * h);   /* weight of f_{j+1} */
        double wm = 1.0 / (h * h) - (cs / sn) / (2.0 * h);   /* weight of f_{j-1} */
        double w0 = -2.0 / (h * h) + P;                       /* weight of f_j     */
        int64_t J = c->p.j0 + jj;
        out[jj * ni + ii] += w0 * v;
        /* neighbour j+1 */
        if (J + 1 >= c->p.nth) out[(c->p.nth - 1 - c->p.j0) * ni + ii] += c->sigma * wp * v;
        else if (jj + 1 < nj) out[(jj + 1) * ni + ii] += wp * v;
        /* neighbour j-1 */
        if (J - 1 < 0) out[(0 - c->p.j0) * ni + ii] += c->sigma * wm * v;
        else if (jj - 1 >= 0) out[(jj - 1) * ni + ii] += wm * v;
    }
}

/* One reverse step: given lam1 = adjoint of u^{n+1} (Phi, Pi), produce
   lam0 = K^H lam1 (adjoint of u^n) and the adjoint of the source values
   aTh (half points, time t^n) and aTi (integer points, time t^n + dt/2).
   Complex-linear forward maps y = c x transpose to x' += conj(c) y'. */
int teuko_adjoint_step(teuko_ctx* c, const double* lP1_ri, const double* lQ1_ri,
                       double* lP0_ri, double* lQ0_ri, double* aTh_ri, double* aTi_ri) {
    const teuko_params* p = &c->p;
    int64_t ni = p->ni, nj = p->nj, N = ni * nj;
    double dt = p->dt, dr = c->dr;
    const cplx* lP1 = (const cplx*)lP1_ri;
    const cplx* lQ1 = (const cplx*)lQ1_ri;
    cplx* lP0 = (cplx*)lP0_ri;
    cplx* lQ0 = (cplx*)lQ0_ri;
    cplx* aTh = (cplx*)aTh_ri;
    cplx* aTi = (cplx*)aTi_ri;
    cplx* aPc = (cplx*)calloc(N, sizeof(cplx));   /* adjoint of corrector means  */
    cplx* aQc = (cplx*)calloc(N, sizeof(cplx));
    cplx* adP = (cplx*)calloc(N, sizeof(cplx));   /* adjoint of corrector diffs  */
    cplx* adQ = (cplx*)calloc(N, sizeof(cplx));
    cplx* aL = (cplx*)calloc(N, sizeof(cplx));    /* adjoint of Lth output       */
    cplx* ahP = (cplx*)calloc(N, sizeof(cplx));   /* adjoint of half-point values */
    cplx* ahQ = (cplx*)calloc(N, sizeof(cplx));
    for (int64_t k = 0; k < N; ++k) { lP0[k] = 0; lQ0[k] = 0; aTh[k] = 0; aTi[k] = 0; }

    /* corrector, reversed */
    for (int64_t jj = 0; jj < nj; ++jj)
        for (int64_t ii = 0; ii < ni; ++ii) {
            int64_t k = jj * ni + ii;
            int64_t Ig = p->i0 + ii;
            if (Ig == 0 || Ig == p->nr - 1) continue;   /* boundary outputs are constants */
            const coeffs* q = &c->ci[k];
            cplx yP = lP1[k], yQ = lQ1[k];
            /* Phi1 = Phi - dt b dP + dt Qc */
            lP0[k] += yP;
            adP[k] += -dt * q->b * yP;
            aQc[k] += dt * yP;
            /* Pi1 = Pi + dt b dQ + dt (T - mu dP + DoS2 L - V Pc - ct Qc) */
            lQ0[k] += yQ;
            adQ[k] += dt * q->b * yQ;
            aTi[k] += dt * yQ;
            adP[k] += -dt * conj(q->mu) * yQ;
            aL[k] += dt * q->DoS2 * yQ;
            aPc[k] += -dt * conj(q->V) * yQ;
            aQc[k] += -dt * conj(q->ct) * yQ;
        }
    for (int64_t ii = 0; ii < ni; ++ii) angular_transpose_add(c, aL, ni, ii, aPc);
    /* Pc = (h_k + h_{k-1})/2, dP = (h_k - h_{k-1})/dr  (h_{k-1} = half point ii-1/2) */
    for (int64_t jj = 0; jj < nj; ++jj)
        for (int64_t ii = 0; ii < ni; ++ii) {
            int64_t k = jj * ni + ii;
            ahP[k] += 0.5 * aPc[k] + adP[k] / dr;
            ahQ[k] += 0.5 * aQc[k] + adQ[k] / dr;
            if (ii - 1 >= 0) {
                ahP[k - 1] += 0.5 * aPc[k] - adP[k] / dr;
                ahQ[k - 1] += 0.5 * aQc[k] - adQ[k] / dr;
            }
        }
    /* predictor, reversed.  Reuse aPc/aQc/adP/adQ/aL for the predictor's means,
       differences and Lth output. */
    memset(aPc, 0, sizeof(cplx) * N); memset(aQc, 0, sizeof(cplx) * N);
    memset(adP, 0, sizeof(cplx) * N); memset(adQ, 0, sizeof(cplx) * N);
    memset(aL, 0, sizeof(cplx) * N);
    for (int64_t jj = 0; jj < nj; ++jj)
        for (int64_t ii = 0; ii < ni; ++ii) {
            int64_t k = jj * ni + ii;
            const coeffs* q = &c->ch[k];
            cplx yP = ahP[k], yQ = ahQ[k];
            /* hP = Pb - (dt/2) b dP + (dt/2) Qb */
            aPc[k] += yP;
            adP[k] += -0.5 * dt * q->b * yP;
            aQc[k] += 0.5 * dt * yP;
            /* hQ = Qb + (dt/2) b dQ + (dt/2)(T - mu dP + DoS2 L - V Pb - ct Qb) */
            aQc[k] += yQ;
            adQ[k] += 0.5 * dt * q->b * yQ;
            aTh[k] += 0.5 * dt * yQ;
            adP[k] += -0.5 * dt * conj(q->mu) * yQ;
            aL[k] += 0.5 * dt * q->DoS2 * yQ;
            aPc[k] += -0.5 * dt * conj(q->V) * yQ;
            aQc[k] += -0.5 * dt * conj(q->ct) * yQ;
        }
    for (int64_t ii = 0; ii < ni; ++ii) angular_transpose_add(c, aL, ni, ii, aPc);
    /* Pb = (u_k + u_{k+1})/2, dP = (u_{k+1} - u_k)/dr */
    for (int64_t jj = 0; jj < nj; ++jj)
        for (int64_t ii = 0; ii < ni; ++ii) {
            int64_t k = jj * ni + ii;
            lP0[k] += 0.5 * aPc[k] - adP[k] / dr;
            lQ0[k] += 0.5 * aQc[k] - adQ[k] / dr;
            if (ii + 1 < ni) {
                lP0[k + 1] += 0.5 * aPc[k] + adP[k] / dr;
                lQ0[k + 1] += 0.5 * aQc[k] + adQ[k] / dr;
            }
        }
    free(aPc); free(aQc); free(adP); free(adQ); free(aL); free(ahP); free(ahQ);
    return 0;
}

/* Source derivatives at time t: dT/damp and dT/dr0 per point, contracted
   with the adjoint a as Re sum conj(a) dT/dp.  `half` selects half points. */
static void source_grad_add(const teuko_ctx* c, const cplx* a, int half, double t,
                            double* g_r0, double* g_amp) {
    const teuko_params* p = &c->p;
    int64_t ni = p->ni, nj = p->nj;
    double sr = p->sigma_r_cells * c->dr;
    double r0 = p->r0, a_ = p->a, M = p->M;
    double drs0_dr0 = (r0 * r0 + a_ * a_) / (r0 * r0 - 2.0 * M * r0 + a_ * a_);
    double den = pow(r0, 1.5) + a_ * sqrt(M);
    double dOm_dr0 = -1.5 * sqrt(M) * sqrt(r0) / (den * den);
    cplx ph = phase(c, t);
    double sa = 0.0, sr0 = 0.0;
    for (int64_t jj = 0; jj < nj; ++jj)
        for (int64_t ii = 0; ii < ni; ++ii) {
            int64_t k = jj * ni + ii;
            double G = half ? c->gh[k] : c->gi[k];
            double x = half ? c->xh[ii] : c->xi[ii];
            cplx dT_damp = G * ph;
            cplx dT_dr0 = p->amp * G * ph * (x / (sr * sr) * drs0_dr0 + (-I * (double)p->m * t) * dOm_dr0);
            sa += creal(conj(a[k]) * dT_damp);
            sr0 += creal(conj(a[k]) * dT_dr0);
        }
    *g_amp += sa;
    *g_r0 += sr0;
}

/* Reverse sweep for L(w^0..w^n) with g[k] = dL/dw^k (real view as complex:
   dL/dRe + i dL/dIm).  Returns dL/dPhi0, dL/dPi0 and the source gradients.
   The step is affine in u with state-independent coefficients, so the sweep
   needs no forward states. */
int teuko_adjoint_run(teuko_ctx* c, const double* g_ri, int64_t n, double t_start,
                      double* dphi0_ri, double* dpi0_ri, double* dL_dr0, double* dL_damp) {
    /* the source-parameter gradients are those of the static source */
    if (c->traj) return -1;
    const teuko_params* p = &c->p;
    int64_t ni = p->ni, nj = p->nj, N = ni * nj;
    const cplx* g = (const cplx*)g_ri;
    int64_t k0 = c->iobs - p->i0;
    if (k0 < 0 || k0 + 1 >= ni) return -1;
    cplx* lP = (cplx*)calloc(N, sizeof(cplx));
    cplx* lQ = (cplx*)calloc(N, sizeof(cplx));
    cplx* nP = (cplx*)calloc(N, sizeof(cplx));
    cplx* nQ = (cplx*)calloc(N, sizeof(cplx));
    cplx* aTh = (cplx*)calloc(N, sizeof(cplx));
    cplx* aTi = (cplx*)calloc(N, sizeof(cplx));
    double gr0 = 0.0, gam = 0.0;
    /* lam^n = E^H g^n */
    for (int64_t jj = 0; jj < nj; ++jj) {
        lP[jj * ni + k0] += (1.0 - c->alpha) * g[n * nj + jj];
        lP[jj * ni + k0 + 1] += c->alpha * g[n * nj + jj];
    }
    for (int64_t k = n - 1; k >= 0; --k) {
        teuko_adjoint_step(c, (double*)lP, (double*)lQ, (double*)nP, (double*)nQ, (double*)aTh, (double*)aTi);
        double t = t_start + (double)k * p->dt;
        source_grad_add(c, aTh, 1, t, &gr0, &gam);
        source_grad_add(c, aTi, 0, t + 0.5 * p->dt, &gr0, &gam);
        for (int64_t jj = 0; jj < nj; ++jj) {
            nP[jj * ni + k0] += (1.0 - c->alpha) * g[k * nj + jj];
            nP[jj * ni + k0 + 1] += c->alpha * g[k * nj + jj];
        }
        cplx* t1 = lP; lP = nP; nP = t1;
        cplx* t2 = lQ; lQ = nQ; nQ = t2;
    }
    memcpy(dphi0_ri, lP, sizeof(cplx) * N);
    memcpy(dpi0_ri, lQ, sizeof(cplx) * N);
    *dL_dr0 = gr0;
    *dL_damp = gam;
    free(lP); free(lQ); free(nP); free(nQ); free(aTh); free(aTi);
    return 0;
}

/* Moving-source gradients of one stage: table entry (r0, phi) with the
   source adjoint a at half (half = 1) or integer points.  With
   T = amp rho(r*) gth(th) e^{-i m phi}, rho = exp(-x^2 / (2 sr^2)),
   x = r* - r*(r0), and U = T / amp the unit-amplitude source:
     dT/damp = U,
     dT/dr0  = T (x / sr^2) (d r* / d r)(r0),  with d r* / d r = (r^2 + a^2) / Delta (Eq. 2),
     dT/dphi = -i m T,
   each contracted as Re sum conj(a) dT/dp. */
static void moving_grad(const teuko_ctx* c, const cplx* a, int half, const double* entry,
                        double* g_r0, double* g_phi, double* g_amp) {
    const teuko_params* p = &c->p;
    int64_t ni = p->ni, nj = p->nj;
    double sr = p->sigma_r_cells * c->dr;
    double r0 = entry[0], phi = entry[1];
    double drs0_dr0 = (r0 * r0 + p->a * p->a) / (r0 * r0 - 2.0 * p->M * r0 + p->a * p->a);
    double sa = 0.0, sr0 = 0.0, sph = 0.0;
    for (int64_t jj = 0; jj < nj; ++jj)
        for (int64_t ii = 0; ii < ni; ++ii) {
            double xs = p->rstar_min + (p->i0 + ii + (half ? 0.5 : 0.0)) * c->dr;
            double x = xs - teuko_rstar_of_r(r0, p->a, p->M);
            cplx U = moving_unit(c, xs, jj, r0, phi);
            cplx ca = conj(a[jj * ni + ii]);
            sa += creal(ca * U);
            sr0 += creal(ca * (p->amp * U) * ((x / (sr * sr)) * drs0_dr0));
            sph += creal(ca * (-I * (double)p->m) * (p->amp * U));
        }
    *g_r0 += sr0;
    *g_phi += sph;
    *g_amp += sa;
}

/* Reverse sweep for a moving source: as teuko_adjoint_run, for a forward
   run of n steps from the first entry of the orbit table (step k used
   entries 2k and 2k+1).  Returns dL/dPhi0, dL/dPi0, dL/damp and, for every
   entry e < 2n, dL/dr0_e and dL/dphi_e in dL_dtraj[2e], dL_dtraj[2e+1]. */
int teuko_adjoint_run_moving(teuko_ctx* c, const double* g_ri, int64_t n, double* dphi0_ri, double* dpi0_ri,
                             double* dL_dtraj, double* dL_damp) {
    if (!c->traj || 2 * n > c->traj_n) return -1;
    const teuko_params* p = &c->p;
    int64_t ni = p->ni, nj = p->nj, N = ni * nj;
    const cplx* g = (const cplx*)g_ri;
    int64_t k0 = c->iobs - p->i0;
    if (k0 < 0 || k0 + 1 >= ni) return -1;
    cplx* lP = (cplx*)calloc(N, sizeof(cplx));
    cplx* lQ = (cplx*)calloc(N, sizeof(cplx));
    cplx* nP = (cplx*)calloc(N, sizeof(cplx));
    cplx* nQ = (cplx*)calloc(N, sizeof(cplx));
    cplx* aTh = (cplx*)calloc(N, sizeof(cplx));
    cplx* aTi = (cplx*)calloc(N, sizeof(cplx));
    double gam = 0.0;
    for (int64_t e = 0; e < 2 * n; ++e) { dL_dtraj[2 * e] = 0.0; dL_dtraj[2 * e + 1] = 0.0; }
    for (int64_t jj = 0; jj < nj; ++jj) {
        lP[jj * ni + k0] += (1.0 - c->alpha) * g[n * nj + jj];
        lP[jj * ni + k0 + 1] += c->alpha * g[n * nj + jj];
    }
    for (int64_t k = n - 1; k >= 0; --k) {
        teuko_adjoint_step(c, (double*)lP, (double*)lQ, (double*)nP, (double*)nQ, (double*)aTh, (double*)aTi);
        /* predictor: entry 2k on half points; corrector: entry 2k+1 on integer points */
        moving_grad(c, aTh, 1, c->traj + 2 * (2 * k), &dL_dtraj[2 * (2 * k)], &dL_dtraj[2 * (2 * k) + 1], &gam);
        moving_grad(c, aTi, 0, c->traj + 2 * (2 * k + 1), &dL_dtraj[2 * (2 * k + 1)],
                    &dL_dtraj[2 * (2 * k + 1) + 1], &gam);
        for (int64_t jj = 0; jj < nj; ++jj) {
            nP[jj * ni + k0] += (1.0 - c->alpha) * g[k * nj + jj];
            nP[jj * ni + k0 + 1] += c->alpha * g[k * nj + jj];
        }
        cplx* t1 = lP; lP = nP; nP = t1;
        cplx* t2 = lQ; lQ = nQ; nQ = t2;
    }
    memcpy(dphi0_ri, lP, sizeof(cplx) * N);
    memcpy(dpi0_ri, lQ, sizeof(cplx) * N);
    *dL_damp = gam;
    free(lP); free(lQ); free(nP); free(nQ); free(aTh); free(aTi);
    return 0;
}

/* Small accessors for the Python side. */
double teuko_dr(const teuko_ctx* c) { return c->dr; }
double teuko_dth(const teuko_ctx* c) { return c->dth; }
double teuko_rstar0(const teuko_ctx* c) { return c->rstar0; }
double teuko_Omega(const teuko_ctx* c) { return c->Omega; }
int64_t teuko_iobs(const teuko_ctx* c) { return c->iobs; }
double teuko_alpha(const teuko_ctx* c) { return c->alpha; }
/* max over held points of Delta/Sigma^2 (integer and half points) */
double teuko_max_DoS2(const teuko_ctx* c) {
    double mx = 0.0;
    int64_t N = c->p.ni * c->p.nj;
    for (int64_t k = 0; k < N; ++k) {
        if (c->ci[k].DoS2 > mx) mx = c->ci[k].DoS2;
        if (c->ch[k].DoS2 > mx) mx = c->ch[k].DoS2;
    }
    return mx;
}

/* Number of OpenMP threads the step loops use. */
#ifdef _OPENMP
#include <omp.h>
int teuko_threads(void) { return omp_get_max_threads(); }
#else
int teuko_threads(void) { return 1; }
#endif
