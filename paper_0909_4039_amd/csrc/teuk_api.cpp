// C ABI of libteuk: context, argument checks, table upload and the step
// loop.  See include/teuk.h for the contract of every entry point.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>

#include "teuk_internal.h"

using namespace teuk;

struct teuk_ctx {
    Geometry geo;
    double dt = 0;
    int prec = 64;
    hipStream_t stream = nullptr;
    int device = 0;
    // device tables (element type follows prec)
    void* d_rad_i = nullptr;
    void* d_rad_h = nullptr;
    void* d_ang = nullptr;
    unsigned int* d_flag = nullptr;
    // bound state
    void* buf[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [pair][phi/pi]
    int cur = 0;
    bool bound = false;
    // source
    bool has_src = false;
    double r0 = 0, amp = 0, sig_r = 2, sig_th = 2, rstar0 = 0, Omega = 0;
    // observer
    void* wave = nullptr;
    int64_t wave_cap = 0, obs_step0 = 0;
    int iobs = 0;
    double alpha = 0;
    // time: t = t0 + (step - step0) dt
    double t0 = 0;
    int64_t step0 = 0, step = 0;
    // tiling
    int rows = 0;
    int order = 0;
    int kblock = 2;   // steps fused per launch
    bool rows_default = true;   // rows follow kblock until set explicitly
    // errors
    int status = TEUK_OK;
    char err[512] = {0};
};

namespace {

int fail(teuk_ctx* c, int code, const char* fmt, ...) {
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(c->err, sizeof(c->err), fmt, ap);
        va_end(ap);
        if (code == TEUK_EDEVICE || code == TEUK_EUNSTABLE) c->status = code;
    }
    return code;
}

#define HIP_TRY(c, expr)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) return fail((c), TEUK_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t elem_size(int prec) { return prec == 64 ? sizeof(double) : sizeof(float); }

int default_rows(int nth, int kblock, int prec) {
    // Measured on 32768 x 1024: single steps prefer short chunks (16 rows:
    // many wavefronts, small tail); two fused steps need 4 halo rows per
    // side and prefer 64 (FP32) to 96 (FP64) rows.
    int rows = (kblock >= 2) ? (prec == 64 ? 96 : 64) : 16;
    return std::min(rows, std::max(nth, 1));
}

int upload_tables(teuk_ctx* c) {
    const Geometry& g = c->geo;
    size_t nrad = g.rad_i.size(), nang = g.ang.size();
    if (c->prec == 64) {
        HIP_TRY(c, hipMemcpyAsync(c->d_rad_i, g.rad_i.data(), nrad * 8, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->d_rad_h, g.rad_h.data(), nrad * 8, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->d_ang, g.ang.data(), nang * 8, hipMemcpyHostToDevice, c->stream));
    } else {
        std::vector<float> a(g.rad_i.begin(), g.rad_i.end()), b(g.rad_h.begin(), g.rad_h.end()),
            d(g.ang.begin(), g.ang.end());
        HIP_TRY(c, hipMemcpyAsync(c->d_rad_i, a.data(), nrad * 4, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->d_rad_h, b.data(), nrad * 4, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->d_ang, d.data(), nang * 4, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));  // host vectors go out of scope
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TEUK_OK;
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

template <typename R>
int launch_steps(teuk_ctx* c, int64_t n) {
    const Geometry& g = c->geo;
    StepArgs<R> a{};
    a.rad_i = (const R*)c->d_rad_i;
    a.rad_h = (const R*)c->d_rad_h;
    a.ang = (const R*)c->d_ang;
    a.stride = g.stride;
    a.nr = (int)g.nr;
    a.nth = (int)g.nth;
    a.rows = c->rows;
    a.n_chunks = (int)((g.nth + c->rows - 1) / c->rows);
    a.order = c->order;
    a.dt = (R)c->dt;
    a.hdt = (R)(0.5 * c->dt);
    a.inv_dr = (R)(1.0 / g.dr);
    a.m2ma = (R)(-2.0 * g.m * g.a);
    a.wave = (R*)c->wave;
    a.iobs = c->iobs;
    a.alpha = (R)c->alpha;
    for (int64_t done = 0; done < n;) {
        const int kb = (c->kblock >= 2 && n - done >= 2) ? 2 : 1;
        const int so = WAVE - 2 * kb;   // valid output columns per strip
        a.kb = kb;
        a.n_strips = (int)((g.nr + so - 1) / so);
        a.n_tiles = a.n_strips * a.n_chunks;
        for (int q = 0; q < KB_MAX; ++q) {
            double t = c->t0 + double(c->step + q - c->step0) * c->dt;
            double w0 = g.m * c->Omega * t, w1 = g.m * c->Omega * (t + 0.5 * c->dt);
            a.ph[2 * q][0] = (R)std::cos(w0);
            a.ph[2 * q][1] = (R)(-std::sin(w0));
            a.ph[2 * q + 1][0] = (R)std::cos(w1);
            a.ph[2 * q + 1][1] = (R)(-std::sin(w1));
            int64_t row = c->step + q - c->obs_step0;
            a.wave_row[q] = (q < kb && c->wave && row >= 0 && row < c->wave_cap) ? row : -1;
        }
        a.phi = (const R*)c->buf[c->cur][0];
        a.pi = (const R*)c->buf[c->cur][1];
        a.phi_out = (R*)c->buf[1 - c->cur][0];
        a.pi_out = (R*)c->buf[1 - c->cur][1];
        if constexpr (std::is_same<R, double>::value) launch_step_fp64(a, c->stream);
        else launch_step_fp32(a, c->stream);
        HIP_TRY(c, hipGetLastError());
        c->cur = 1 - c->cur;
        c->step += kb;
        done += kb;
    }
    // the last state's waveform row
    int64_t row = c->step - c->obs_step0;
    if (c->wave && row >= 0 && row < c->wave_cap) {
        if (c->prec == 64)
            launch_extract_fp64((const double*)c->buf[c->cur][0], (double*)c->wave + 2 * row * g.nth, (int)g.nr,
                                (int)g.nth, c->iobs, c->alpha, c->stream);
        else
            launch_extract_fp32((const float*)c->buf[c->cur][0], (float*)c->wave + 2 * row * g.nth, (int)g.nr,
                                (int)g.nth, c->iobs, (float)c->alpha, c->stream);
        HIP_TRY(c, hipGetLastError());
    }
    return TEUK_OK;
}

}  // namespace

extern "C" {

int teuk_create(const teuk_grid* g, double a, double M, int32_t m, int32_t s, double dt, int32_t prec,
                void* hip_stream, teuk_ctx** out) {
    if (!out) return TEUK_EINVAL;
    *out = nullptr;
    if (validate_phys(g, a, M, s) != TEUK_OK) return TEUK_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return TEUK_EINVAL;
    if (prec != TEUK_FP64 && prec != TEUK_FP32) return TEUK_EINVAL;
    if (m < -1000 || m > 1000) return TEUK_EINVAL;
    teuk_ctx* c = new (std::nothrow) teuk_ctx();
    if (!c) return TEUK_EDEVICE;
    c->prec = prec;
    c->dt = dt;
    c->stream = (hipStream_t)hip_stream;
    Geometry& geo = c->geo;
    geo.nr = g->n_rstar;
    geo.nth = g->n_theta;
    geo.rmin = g->rstar_min;
    geo.rmax = g->rstar_max;
    geo.a = a;
    geo.M = M;
    geo.m = m;
    geo.s = s;
    build_geometry(geo);
    c->rows = default_rows((int)geo.nth, c->kblock, prec);
    size_t es = elem_size(prec);
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipMalloc(&c->d_rad_i, geo.rad_i.size() * es) != hipSuccess ||
        hipMalloc(&c->d_rad_h, geo.rad_h.size() * es) != hipSuccess ||
        hipMalloc(&c->d_ang, geo.ang.size() * es) != hipSuccess ||
        hipMalloc((void**)&c->d_flag, sizeof(unsigned int)) != hipSuccess) {
        teuk_destroy(c);
        return TEUK_EDEVICE;
    }
    if (upload_tables(c) != TEUK_OK) {
        teuk_destroy(c);
        return TEUK_EDEVICE;
    }
    *out = c;
    return TEUK_OK;
}

int teuk_destroy(teuk_ctx* c) {
    if (!c) return TEUK_EINVAL;
    if (c->d_rad_i || c->d_rad_h || c->d_ang || c->d_flag) (void)hipStreamSynchronize(c->stream);
    if (c->d_rad_i) (void)hipFree(c->d_rad_i);
    if (c->d_rad_h) (void)hipFree(c->d_rad_h);
    if (c->d_ang) (void)hipFree(c->d_ang);
    if (c->d_flag) (void)hipFree(c->d_flag);
    delete c;
    return TEUK_OK;
}

int teuk_bind_state(teuk_ctx* c, void* phi, void* pi, void* phi_next, void* pi_next) {
    if (!c) return TEUK_EINVAL;
    void* p[4] = {phi, pi, phi_next, pi_next};
    for (int i = 0; i < 4; ++i) {
        if (!p[i]) return fail(c, TEUK_EINVAL, "state pointer %d is NULL", i);
        if ((uintptr_t)p[i] % 16 != 0) return fail(c, TEUK_EINVAL, "state pointer %d is not 16-byte aligned", i);
        for (int k = 0; k < i; ++k)
            if (p[k] == p[i]) return fail(c, TEUK_EINVAL, "state pointers %d and %d alias", k, i);
    }
    c->buf[0][0] = phi;
    c->buf[0][1] = pi;
    c->buf[1][0] = phi_next;
    c->buf[1][1] = pi_next;
    c->cur = 0;
    c->bound = true;
    return TEUK_OK;
}

int teuk_set_source(teuk_ctx* c, double r0, double amp, double sigma_r_cells, double sigma_th_cells) {
    if (!c) return TEUK_EINVAL;
    Geometry& g = c->geo;
    if (!std::isfinite(amp) || !std::isfinite(r0)) return fail(c, TEUK_EINVAL, "non-finite source parameter");
    if (!(r0 > g.rp)) return fail(c, TEUK_EINVAL, "r0 = %g must exceed r+ = %g", r0, g.rp);
    if (!(sigma_r_cells > 0.0) || !(sigma_th_cells > 0.0)) return fail(c, TEUK_EINVAL, "source widths must be > 0");
    c->r0 = r0;
    c->amp = amp;
    c->sig_r = sigma_r_cells;
    c->sig_th = sigma_th_cells;
    c->rstar0 = rstar_of_delta(r0 - g.rp, g.a, g.M);
    c->Omega = std::sqrt(g.M) / (std::pow(r0, 1.5) + g.a * std::sqrt(g.M));
    c->has_src = true;
    build_source(g, c->rstar0, sigma_r_cells * g.dr, sigma_th_cells * g.dth, amp);
    return upload_tables(c);
}

int teuk_set_observer(teuk_ctx* c, double rstar_obs, void* wave, int64_t capacity_rows) {
    if (!c) return TEUK_EINVAL;
    if (!wave) {
        c->wave = nullptr;
        c->wave_cap = 0;
        return TEUK_OK;
    }
    int i0;
    double al;
    if (!observer_index(c->geo, rstar_obs, i0, al))
        return fail(c, TEUK_EINVAL, "rstar_obs = %g outside the open grid interval", rstar_obs);
    if (capacity_rows < 0) return fail(c, TEUK_EINVAL, "negative capacity");
    if ((uintptr_t)wave % 16 != 0) return fail(c, TEUK_EINVAL, "wave buffer not 16-byte aligned");
    c->wave = wave;
    c->wave_cap = capacity_rows;
    c->iobs = i0;
    c->alpha = al;
    c->obs_step0 = c->step;
    return TEUK_OK;
}

int teuk_step(teuk_ctx* c, int64_t n) {
    if (!c) return TEUK_EINVAL;
    if (c->status != TEUK_OK) return c->status;
    if (n < 0) return fail(c, TEUK_EINVAL, "negative step count");
    if (!c->bound) return fail(c, TEUK_ESTATE, "no state bound");
    if (n == 0 && !c->wave) return TEUK_OK;
    if (c->prec == 64) return launch_steps<double>(c, n);
    return launch_steps<float>(c, n);
}

int teuk_extract(teuk_ctx* c, double rstar_obs, void* out) {
    if (!c || !out) return TEUK_EINVAL;
    if (!c->bound) return fail(c, TEUK_ESTATE, "no state bound");
    int i0;
    double al;
    if (!observer_index(c->geo, rstar_obs, i0, al))
        return fail(c, TEUK_EINVAL, "rstar_obs = %g outside the open grid interval", rstar_obs);
    if (c->prec == 64)
        launch_extract_fp64((const double*)c->buf[c->cur][0], (double*)out, (int)c->geo.nr, (int)c->geo.nth, i0, al,
                            c->stream);
    else
        launch_extract_fp32((const float*)c->buf[c->cur][0], (float*)out, (int)c->geo.nr, (int)c->geo.nth, i0,
                            (float)al, c->stream);
    HIP_TRY(c, hipGetLastError());
    return TEUK_OK;
}

int teuk_get_time(teuk_ctx* c, double* t, int64_t* step) {
    if (!c) return TEUK_EINVAL;
    if (t) *t = c->t0 + double(c->step - c->step0) * c->dt;
    if (step) *step = c->step;
    return TEUK_OK;
}

int teuk_set_time(teuk_ctx* c, double t, int64_t step) {
    if (!c || !std::isfinite(t)) return TEUK_EINVAL;
    c->t0 = t;
    c->step0 = step;
    c->obs_step0 += step - c->step;
    c->step = step;
    return TEUK_OK;
}

int teuk_current(teuk_ctx* c) {
    if (!c) return TEUK_EINVAL;
    return c->cur;
}

int teuk_set_tiling(teuk_ctx* c, int32_t rows_per_wave, int32_t order) {
    if (!c) return TEUK_EINVAL;
    if (order < 0 || order > 1) return fail(c, TEUK_EINVAL, "order must be 0 or 1");
    if (rows_per_wave == 0) {
        c->rows = default_rows((int)c->geo.nth, c->kblock, c->prec);
        c->order = 0;
        c->rows_default = true;
        return TEUK_OK;
    }
    if (rows_per_wave < 1 || rows_per_wave > 4096) return fail(c, TEUK_EINVAL, "rows_per_wave out of range");
    c->rows = rows_per_wave;
    c->rows_default = false;
    c->order = order;
    return TEUK_OK;
}

int teuk_set_blocking(teuk_ctx* c, int32_t steps_per_launch) {
    if (!c) return TEUK_EINVAL;
    if (steps_per_launch < 1 || steps_per_launch > KB_MAX)
        return fail(c, TEUK_EINVAL, "steps_per_launch must be 1..%d", KB_MAX);
    c->kblock = steps_per_launch;
    if (c->rows_default) c->rows = default_rows((int)c->geo.nth, c->kblock, c->prec);
    return TEUK_OK;
}

int teuk_get_blocking(teuk_ctx* c) { return c ? c->kblock : TEUK_EINVAL; }

int teuk_get_tiling(teuk_ctx* c, int32_t* rows_per_wave, int32_t* order) {
    if (!c) return TEUK_EINVAL;
    if (rows_per_wave) *rows_per_wave = c->rows;
    if (order) *order = c->order;
    return TEUK_OK;
}

int teuk_check_finite(teuk_ctx* c) {
    if (!c) return TEUK_EINVAL;
    if (c->status != TEUK_OK) return c->status;
    if (!c->bound) return fail(c, TEUK_ESTATE, "no state bound");
    unsigned int zero = 0, flag = 0;
    HIP_TRY(c, hipMemcpyAsync(c->d_flag, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream));
    int64_t n = 2 * c->geo.nr * c->geo.nth;
    for (int f = 0; f < 2; ++f) {
        if (c->prec == 64) launch_count_nonfinite_fp64((const double*)c->buf[c->cur][f], n, c->d_flag, c->stream);
        else launch_count_nonfinite_fp32((const float*)c->buf[c->cur][f], n, c->d_flag, c->stream);
        HIP_TRY(c, hipGetLastError());
    }
    HIP_TRY(c, hipMemcpyAsync(&flag, c->d_flag, sizeof(flag), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (flag) return fail(c, TEUK_EUNSTABLE, "non-finite value in the state at step %lld", (long long)c->step);
    return TEUK_OK;
}

int teuk_status(teuk_ctx* c) { return c ? c->status : TEUK_EINVAL; }

const char* teuk_last_error(teuk_ctx* c) { return c ? c->err : "null context"; }

const char* teuk_strerror(int code) {
    switch (code) {
        case TEUK_OK: return "TEUK_OK";
        case TEUK_EINVAL: return "TEUK_EINVAL: invalid argument";
        case TEUK_ESTATE: return "TEUK_ESTATE: call out of order";
        case TEUK_EDEVICE: return "TEUK_EDEVICE: HIP runtime error";
        case TEUK_EUNSTABLE: return "TEUK_EUNSTABLE: non-finite values in the state";
        case TEUK_ENOTSUP: return "TEUK_ENOTSUP: not supported";
        default: return "unknown teuk error";
    }
}

int teuk_suggest_dt(const teuk_grid* g, double a, double M, int32_t m, int32_t s, int64_t n_steps, double* dt_out) {
    if (!dt_out || n_steps < 1) return TEUK_EINVAL;
    if (validate_phys(g, a, M, s) != TEUK_OK) return TEUK_EINVAL;
    Geometry geo;
    geo.nr = g->n_rstar;
    geo.nth = g->n_theta;
    geo.rmin = g->rstar_min;
    geo.rmax = g->rstar_max;
    geo.a = a;
    geo.M = M;
    geo.m = m;
    geo.s = s;
    build_geometry(geo);
    double wmax = std::sqrt(angular_bound(geo) * max_delta_over_sigma2(geo));
    double dt = 0.5 * geo.dr;
    if (wmax > 0.0) dt = std::min(dt, std::pow(8.0 / double(n_steps), 0.25) / wmax);
    *dt_out = dt;
    return TEUK_OK;
}

double teuk_rstar_of_r(double r, double a, double M) {
    double rp = M + std::sqrt(M * M - a * a);
    return rstar_of_delta(r - rp, a, M);
}

double teuk_delta_of_rstar(double rstar, double a, double M) { return delta_of_rstar(rstar, a, M); }

}  // extern "C"
