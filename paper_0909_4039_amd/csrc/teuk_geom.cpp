// Host-side geometry of libteuk: the tortoise map (paper Eq. 2), the radial
// coefficient numerators of the first-order system (Eqs. 5-12) and the
// angular difference weights (centred second differences on a cell-centred
// theta grid, with the pole rule stated after Eq. 14).  FP64, built once
// per context and uploaded.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <thread>

#include "teuk_internal.h"

namespace teuk {

static void horizons(double a, double M, double& rp, double& rm) {
    double q = std::sqrt(M * M - a * a);
    rp = M + q;
    rm = M - q;
}

// Eq. (2) integrated: r* = r + 2M r+/(r+-r-) ln((r-r+)/2M) - 2M r-/(r+-r-) ln((r-r-)/2M),
// written in delta = r - r+ so that the horizon limit keeps its precision.
double rstar_of_delta(double delta, double a, double M) {
    double rp, rm;
    horizons(a, M, rp, rm);
    double k = rp - rm;
    double v = rp + delta + (2.0 * M * rp / k) * std::log(delta / (2.0 * M));
    if (rm > 0.0) v -= (2.0 * M * rm / k) * std::log((delta + k) / (2.0 * M));
    return v;
}

// Solve r*(delta) = rstar for x = ln delta by safeguarded Newton:
// d r*/dx = delta (r^2 + a^2)/Delta = (r^2 + a^2)/(r - r-) > 0.
double delta_of_rstar(double rstar, double a, double M) {
    double rp, rm;
    horizons(a, M, rp, rm);
    auto f = [&](double x) { return rstar_of_delta(std::exp(x), a, M) - rstar; };
    auto fp = [&](double x) {
        double d = std::exp(x), r = rp + d;
        return (r * r + a * a) / (r - rm);
    };
    double lo = -60.0, hi = 12.0;
    while (lo > -740.0 && f(lo) > 0.0) lo -= 60.0;
    while (f(hi) < 0.0) hi += 12.0;
    double x = (rstar > rp + 1.0) ? std::log(std::max(rstar - rp, 1e-300)) : 0.5 * (lo + hi);
    x = std::min(std::max(x, lo), hi);
    for (int it = 0; it < 200; ++it) {
        double fx = f(x);
        if (fx == 0.0) break;
        if (fx < 0.0) lo = x; else hi = x;
        double xn = x - fx / fp(x);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (std::fabs(xn - x) <= 1e-16 * std::max(1.0, std::fabs(x))) { x = xn; break; }
        x = xn;
    }
    return std::exp(x);
}

static void radial_entry(const Geometry& g, double rstar, std::vector<double>& tab, int64_t i) {
    const double a = g.a, M = g.M;
    const double s = g.s, m = g.m;
    double d = delta_of_rstar(rstar, a, M);
    double r = g.rp + d;
    double D = d * (d + (g.rp - g.rm));
    double w2 = r * r + a * a;
    auto put = [&](int f, double v) { tab[(int64_t)f * g.stride + i] = v; };
    put(R_W2, w2);
    put(R_DEL, D);
    put(R_WBN, a * a * D * ((r - M) * w2 - 2.0 * r * D));
    put(R_CTR, 2.0 * s * (r * D - M * (r * r - a * a)));
    put(R_CTI0, 4.0 * M * a * m * r);
    put(R_CRR, -(6.0 * w2 * D / r + 2.0 * r * D + 2.0 * s * (r - M) * w2));
    put(R_VR, -D * (6.0 * D / (r * r) + 6.0 * (1.0 + s) * (r - M) / r));
    put(R_VI, -(6.0 * m * a * D / r + 4.0 * s * m * a * (r - M)));
    put(R_GR, 0.0);
    put(R_XR, 0.0);
}

void build_geometry(Geometry& g) {
    horizons(g.a, g.M, g.rp, g.rm);
    g.dr = (g.rmax - g.rmin) / double(g.nr - 1);
    g.dth = M_PI / double(g.nth);
    g.stride = (g.nr + 63) / 64 * 64;
    g.rad_i.assign((size_t)R_NFIELDS * g.stride, 0.0);
    g.rad_h.assign((size_t)R_NFIELDS * g.stride, 0.0);
    // Each column inverts Eq. (2) on its own (a few microseconds): large
    // grids split the columns over host threads (OMP_NUM_THREADS if set,
    // else the hardware's count, at most 64).  Every entry is computed the
    // same way whatever the split.
    auto fill = [&g](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            radial_entry(g, g.rmin + double(i) * g.dr, g.rad_i, i);
            radial_entry(g, g.rmin + (double(i) + 0.5) * g.dr, g.rad_h, i);
        }
    };
    int64_t nt = 1;
    if (g.nr >= 65536) {
        const char* env = std::getenv("OMP_NUM_THREADS");
        nt = env ? std::atoi(env) : (int64_t)std::thread::hardware_concurrency();
        nt = std::min<int64_t>(std::max<int64_t>(nt, 1), 64);
    }
    if (nt == 1) {
        fill(0, g.nr);
    } else {
        std::vector<std::thread> pool;
        for (int64_t t = 0; t < nt; ++t) pool.emplace_back(fill, g.nr * t / nt, g.nr * (t + 1) / nt);
        for (std::thread& th : pool) th.join();
    }
    // padding columns repeat the last node so that clamped reads stay finite
    for (int f = 0; f < R_NFIELDS; ++f)
        for (int64_t i = g.nr; i < g.stride; ++i) {
            g.rad_i[(size_t)f * g.stride + i] = g.rad_i[(size_t)f * g.stride + g.nr - 1];
            g.rad_h[(size_t)f * g.stride + i] = g.rad_h[(size_t)f * g.stride + g.nr - 1];
        }
    g.ang.assign((size_t)g.nth * A_STRIDE, 0.0);
    const double h = g.dth;
    const double sig = ((std::abs(g.m + g.s) % 2) == 0) ? 1.0 : -1.0;
    for (int64_t j = 0; j < g.nth; ++j) {
        double th = (double(j) + 0.5) * h;
        double sn = std::sin(th), cs = std::cos(th);
        double cot = cs / sn;
        double q = g.m + g.s * cs;
        double* A = &g.ang[(size_t)j * A_STRIDE];
        A[A_SIN2] = sn * sn;
        A[A_A2S2] = g.a * g.a * sn * sn;
        A[A_CS] = 2.0 * g.s * g.a * cs;
        double wp = 1.0 / (h * h) + cot / (2.0 * h);
        double wm = 1.0 / (h * h) - cot / (2.0 * h);
        double w0 = -2.0 / (h * h) + (g.s - q * q / (sn * sn));
        // pole ghosts: f_{-1} = sig f_0, f_{nth} = sig f_{nth-1}
        if (j == 0) { w0 += sig * wm; wm = 0.0; }
        if (j == g.nth - 1) { w0 += sig * wp; wp = 0.0; }
        A[A_P] = wp;
        A[A_M] = wm;
        A[A_0] = w0;
        A[A_GTH] = 0.0;
        A[A_AGTH] = 0.0;
    }
}

void build_source(Geometry& g, double rstar0, double sr, double sth, double amp) {
    for (int64_t i = 0; i < g.stride; ++i) {
        int64_t k = std::min(i, g.nr - 1);
        double xi = g.rmin + double(k) * g.dr - rstar0;
        double xh = g.rmin + (double(k) + 0.5) * g.dr - rstar0;
        g.rad_i[(size_t)R_GR * g.stride + i] = std::exp(-xi * xi / (2.0 * sr * sr));
        g.rad_h[(size_t)R_GR * g.stride + i] = std::exp(-xh * xh / (2.0 * sr * sr));
        g.rad_i[(size_t)R_XR * g.stride + i] = xi / (sr * sr);
        g.rad_h[(size_t)R_XR * g.stride + i] = xh / (sr * sr);
    }
    for (int64_t j = 0; j < g.nth; ++j) {
        double th = (double(j) + 0.5) * g.dth;
        double d = th - 0.5 * M_PI;
        double gth = std::exp(-d * d / (2.0 * sth * sth));
        g.ang[(size_t)j * A_STRIDE + A_GTH] = gth;
        g.ang[(size_t)j * A_STRIDE + A_AGTH] = amp * gth;
    }
}

double angular_bound(const Geometry& g) {
    // Gershgorin: every eigenvalue of the tridiagonal angular matrix lies in
    // a disc around a diagonal entry (pole ghosts are already folded in).
    double best = 0.0;
    for (int64_t j = 0; j < g.nth; ++j) {
        const double* A = &g.ang[(size_t)j * A_STRIDE];
        best = std::max(best, std::fabs(A[A_0]) + std::fabs(A[A_P]) + std::fabs(A[A_M]));
    }
    return best;
}

double max_delta_over_sigma2(const Geometry& g) {
    double smax = 0.0;
    for (int64_t j = 0; j < g.nth; ++j) smax = std::max(smax, g.ang[(size_t)j * A_STRIDE + A_SIN2]);
    double best = 0.0;
    for (const std::vector<double>* t : {&g.rad_i, &g.rad_h})
        for (int64_t i = 0; i < g.nr; ++i) {
            double D = (*t)[(size_t)R_DEL * g.stride + i];
            double w2 = (*t)[(size_t)R_W2 * g.stride + i];
            best = std::max(best, D / (w2 * w2 - g.a * g.a * D * smax));
        }
    return best;
}


// ----------------------------------------------------- shared host checks

int default_rows(int nth, int kblock, int prec) {
    // Measured on 32768 x 1024: single steps prefer short chunks (16 rows:
    // many wavefronts, small tail); two fused steps need 4 halo rows per
    // side and prefer 64 (FP32) to 96 (FP64) rows.
    int rows = (kblock >= 2) ? (prec == TEUK_FP32 ? 64 : 96) : 16;   // FP32 storage with FP64 arithmetic: as FP64
    return std::min(rows, std::max(nth, 1));
}

bool observer_index(const Geometry& g, double rstar_obs, int& i0, double& alpha) {
    if (!(rstar_obs > g.rmin && rstar_obs < g.rmax)) return false;
    int64_t i = (int64_t)std::floor((rstar_obs - g.rmin) / g.dr);
    i = std::min<int64_t>(std::max<int64_t>(i, 0), g.nr - 2);
    i0 = (int)i;
    alpha = (rstar_obs - (g.rmin + double(i) * g.dr)) / g.dr;
    return true;
}

int validate_phys(const teuk_grid* g, double a, double M, int32_t s) {
    if (!g) return TEUK_EINVAL;
    if (g->n_rstar < 4 || g->n_theta < 4) return TEUK_EINVAL;
    if (g->n_rstar > (int64_t)1 << 26 || g->n_theta > (int64_t)1 << 20) return TEUK_EINVAL;
    if ((int64_t)g->n_rstar * g->n_theta > ((int64_t)1 << 40)) return TEUK_EINVAL;
    if (!(g->rstar_min < g->rstar_max) || !std::isfinite(g->rstar_min) || !std::isfinite(g->rstar_max))
        return TEUK_EINVAL;
    if (!(M > 0.0) || !(a >= 0.0) || !(a < M) || !std::isfinite(M)) return TEUK_EINVAL;
    if (s < -2 || s > 2) return TEUK_EINVAL;
    return TEUK_OK;
}

// Angular frequency of the circular equatorial orbit at r0.
double orbit_omega(double r0, double a, double M) { return std::sqrt(M) / (std::pow(r0, 1.5) + a * std::sqrt(M)); }

}  // namespace teuk
