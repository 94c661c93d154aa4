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
    // moving source: (r0, phi) at t(traj_step0) + k dt/2, k < traj_n
    std::vector<double> traj;
    int64_t traj_n = 0, traj_step0 = 0;
    // tiling
    int rows = 0;
    int order = 0;
    int kblock = 2;   // steps fused per launch
    bool rows_default = true;   // rows follow kblock until set explicitly
    // tiling of the reverse sweep: adj_rows 0 follows the forward's rows
    int adj_rows = 0;
    int adj_kb = 1;
    // watchdog: scan the state every watch_every steps (0: off); d_watch
    // holds step + 1 of the first scan that found a value at or above
    // watch_lim, and each teuk_step ends with a copy of it into the pinned
    // host word h_watch, read without waiting by later calls
    int64_t watch_every = 0;
    double watch_lim = 0;
    unsigned long long* d_watch = nullptr;
    volatile unsigned long long* h_watch = nullptr;
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

// Element size of the coefficient tables: FP64 for FP64 arithmetic (TEUK_FP64
// and TEUK_FP32S), FP32 for TEUK_FP32.
size_t elem_size(int prec) { return prec == TEUK_FP32 ? sizeof(float) : sizeof(double); }

// Element size of the state and the waveform: FP32 for TEUK_FP32 and
// TEUK_FP32S, FP64 for TEUK_FP64.
size_t storage_size(int prec) { return prec == TEUK_FP64 ? sizeof(double) : sizeof(float); }

// The device's last-level cache (MI355X Infinity Cache, 256 MiB): a state
// pair larger than this does not stay resident from one launch to the next.
constexpr double kLastLevelCacheBytes = 256.0 * 1024 * 1024;

// Turn a watchdog finding that has reached the host into the sticky
// TEUK_EUNSTABLE (no wait: a scan still in flight is seen by a later call).
int watch_poll(teuk_ctx* c) {
    if (c->status == TEUK_OK && c->h_watch && *c->h_watch != 0ull)
        return fail(c, TEUK_EUNSTABLE, "watchdog: a value not below %g in magnitude (or not finite) at step %lld",
                    c->watch_lim, (long long)(*c->h_watch - 1));
    return c->status;
}

int upload_tables(teuk_ctx* c) {
    const Geometry& g = c->geo;
    size_t nrad = g.rad_i.size(), nang = g.ang.size();
    if (c->prec != TEUK_FP32) {
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

template <typename R>
StepArgs<R> step_args(const teuk_ctx* c) {
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
    a.order = c->order == 2 ? 0 : c->order;
    a.split = c->order == 2 ? 1 : 0;   // two fused steps on a pair of wavefronts
    // Output rows of a streamed state are not read again within the launch:
    // non-temporal stores measured 2-5 % faster on 32768 x 1024 FP64 and up
    // to 3 % slower on 8192 x 256, whose state pair stays cache-resident.
    const double state_bytes = 2.0 * double(g.nr) * double(g.nth) * 2.0 * double(storage_size(c->prec));
    a.stream_out = state_bytes > kLastLevelCacheBytes ? 1 : 0;
    a.dt = (R)c->dt;
    a.hdt = (R)(0.5 * c->dt);
    a.inv_dr = (R)(1.0 / g.dr);
    a.m2ma = (R)(-2.0 * g.m * g.a);
    a.wave = (R*)c->wave;
    a.iobs = c->iobs;
    a.alpha = (R)c->alpha;
    a.moving = c->traj_n > 0 ? 1 : 0;
    const double sr = c->sig_r * g.dr;
    a.two_sr2 = (R)(2.0 * sr * sr);
    a.rmin = (R)g.rmin;
    a.dr = (R)g.dr;
    return a;
}

// One launch of kb steps from the state at step `step` in pair `src` into
// pair 1 - src; the recorder writes the entering states' rows if `record`.
template <typename R>
int launch_one(teuk_ctx* c, StepArgs<R>& a, int kb, int src, int64_t step, bool record) {
    const Geometry& g = c->geo;
    const int so = WAVE - 2 * kb;   // valid output columns per strip
    a.kb = kb;
    a.n_strips = (int)((g.nr + so - 1) / so);
    a.n_tiles = a.n_strips * a.n_chunks;
    for (int q = 0; q < KB_MAX; ++q) {
        double t = c->t0 + double(step + q - c->step0) * c->dt;
        double w0 = g.m * c->Omega * t, w1 = g.m * c->Omega * (t + 0.5 * c->dt);
        if (c->traj_n > 0) {
            // moving source: orbit entries at t (predictor) and t + dt/2 (corrector)
            int64_t k = 2 * (step + q - c->traj_step0);
            k = std::min<int64_t>(std::max<int64_t>(k, 0), c->traj_n - 2);   // q >= kb: unused
            const double* e = &c->traj[2 * k];
            a.rs0[2 * q] = (R)rstar_of_delta(e[0] - g.rp, g.a, g.M);
            a.rs0[2 * q + 1] = (R)rstar_of_delta(e[2] - g.rp, g.a, g.M);
            w0 = g.m * e[1];
            w1 = g.m * e[3];
        }
        a.ph[2 * q][0] = (R)std::cos(w0);
        a.ph[2 * q][1] = (R)(-std::sin(w0));
        a.ph[2 * q + 1][0] = (R)std::cos(w1);
        a.ph[2 * q + 1][1] = (R)(-std::sin(w1));
        int64_t row = step + q - c->obs_step0;
        a.wave_row[q] = (record && q < kb && c->wave && row >= 0 && row < c->wave_cap) ? row : -1;
    }
    a.phi = (const R*)c->buf[src][0];
    a.pi = (const R*)c->buf[src][1];
    a.phi_out = (R*)c->buf[1 - src][0];
    a.pi_out = (R*)c->buf[1 - src][1];
    if constexpr (std::is_same<R, double>::value) {
        if (c->prec == TEUK_FP32S) launch_step_fp32s(a, c->stream);   // float state, FP64 arithmetic
        else launch_step_fp64(a, c->stream);
    } else {
        launch_step_fp32(a, c->stream);
    }
    HIP_TRY(c, hipGetLastError());
    return TEUK_OK;
}

// Watchdog scan of the current state (both fields), tagged with the step.
int launch_watch(teuk_ctx* c) {
    const int64_t n = 2 * c->geo.nr * c->geo.nth;
    for (int f = 0; f < 2; ++f) {
        if (c->prec == TEUK_FP64)
            launch_watch_fp64((const double*)c->buf[c->cur][f], n, c->watch_lim, c->step, c->d_watch, c->stream);
        else
            launch_watch_fp32((const float*)c->buf[c->cur][f], n, (float)c->watch_lim, c->step, c->d_watch,
                              c->stream);
        HIP_TRY(c, hipGetLastError());
    }
    return TEUK_OK;
}

template <typename R>
int launch_steps(teuk_ctx* c, int64_t n) {
    const Geometry& g = c->geo;
    StepArgs<R> a = step_args<R>(c);
    for (int64_t done = 0; done < n;) {
        // with the watchdog on, a launch never crosses a multiple of watch_every
        int kb = (c->kblock >= 2 && n - done >= 2) ? 2 : 1;
        if (c->watch_every > 0 && kb == 2 && (c->step + 1) % c->watch_every == 0) kb = 1;
        int rc = launch_one<R>(c, a, kb, c->cur, c->step, true);
        if (rc != TEUK_OK) return rc;
        c->cur = 1 - c->cur;
        c->step += kb;
        done += kb;
        if (c->watch_every > 0 && c->step % c->watch_every == 0) {
            rc = launch_watch(c);
            if (rc != TEUK_OK) return rc;
        }
    }
    if (c->watch_every > 0 && n > 0)
        HIP_TRY(c, hipMemcpyAsync((void*)c->h_watch, c->d_watch, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                  c->stream));
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

// Seconds per step of `launches` trial launches at the context's current
// tiling and blocking.  Every trial launch reads the current pair and writes
// the other one, so the state, the step count and the waveform are left as
// they were (the other pair is scratch between steps).
template <typename R>
int time_trial(teuk_ctx* c, int launches, double* sec_per_step) {
    StepArgs<R> a = step_args<R>(c);
    const int kb = c->kblock;
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(c, TEUK_EDEVICE, "hipEventCreate failed");
    }
    int rc = launch_one<R>(c, a, kb, c->cur, c->step, false);   // warm-up
    if (rc == TEUK_OK && hipEventRecord(e0, c->stream) != hipSuccess) rc = fail(c, TEUK_EDEVICE, "event record");
    for (int k = 0; rc == TEUK_OK && k < launches; ++k) rc = launch_one<R>(c, a, kb, c->cur, c->step, false);
    if (rc == TEUK_OK && hipEventRecord(e1, c->stream) != hipSuccess) rc = fail(c, TEUK_EDEVICE, "event record");
    float ms = 0.0f;
    if (rc == TEUK_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = fail(c, TEUK_EDEVICE, "event timing");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == TEUK_OK) *sec_per_step = 1e-3 * ms / double(launches * kb);
    return rc;
}

int adjoint_rows(const teuk_ctx* c) { return c->adj_rows > 0 ? c->adj_rows : c->rows; }

// Blocks of the reverse sweep's launch grid at `rows` θ rows per wave and
// kb steps per launch.
int64_t adjoint_blocks(const Geometry& g, int rows, int kb) {
    const int64_t nchunks = (g.nth + rows - 1) / rows;
    const int64_t so = WAVE - 2 * kb;
    const int64_t strips = (g.nr + so - 1) / so;
    return (strips + WG_WAVES - 1) / WG_WAVES * nchunks;
}

// Gradient slots: one per wave of the launch grid.  The workspace holds
// enough for any tiling (one row per wave, two steps per launch has the most
// blocks), so its size does not change when the tiling does.
int64_t adjoint_slots_max(const Geometry& g) {
    int64_t best = 0;
    for (int kb = 1; kb <= KB_MAX; ++kb) best = std::max(best, adjoint_blocks(g, 1, kb));
    return best * WG_WAVES;
}
int64_t adjoint_slots_used(const teuk_ctx* c) {
    return adjoint_blocks(c->geo, adjoint_rows(c), c->adj_kb) * WG_WAVES;
}

int64_t round256(int64_t b) { return (b + 255) / 256 * 256; }

// Workspace layout: [lambda Phi][lambda Pi] (complex128 [nth][nr] each),
// then the per-wave gradient slots (3 sums per wave for the static source;
// for a moving one, two buffers of 3 per table entry of a launch, used by
// alternate launches), then 4 doubles of result, then, with an orbit table
// of n entries, the moving source's per-entry sums [n][3].
struct AdjLayout {
    int64_t lam, slots, result, mout, total, n_slots;
};
AdjLayout adjoint_layout(const teuk_ctx* c) {
    AdjLayout L;
    const int64_t n = c->geo.nr * c->geo.nth;
    L.n_slots = adjoint_slots_max(c->geo);
    L.lam = 0;
    L.slots = round256(2 * n * 16);
    L.result = L.slots + 2 * round256(L.n_slots * 6 * KB_MAX * 8);
    L.mout = L.result + 256;
    L.total = L.mout + round256(c->traj_n * 3 * 8);
    return L;
}

// Launch arguments of the reverse sweep that do not change from launch to
// launch, at the context's reverse-sweep tiling.
AdjArgs adjoint_args(const teuk_ctx* c, const double* g, int iobs, double alpha, double* slots) {
    const Geometry& geo = c->geo;
    const int rows = adjoint_rows(c);
    AdjArgs a{};
    a.rad_i = (const double*)c->d_rad_i;
    a.rad_h = (const double*)c->d_rad_h;
    a.ang = (const double*)c->d_ang;
    a.stride = geo.stride;
    a.nr = (int)geo.nr;
    a.nth = (int)geo.nth;
    a.rows = rows;
    a.n_chunks = (int)((geo.nth + rows - 1) / rows);
    a.dt = c->dt;
    a.hdt = 0.5 * c->dt;
    a.inv_dr = 1.0 / geo.dr;
    a.m2ma = -2.0 * geo.m * geo.a;
    a.g = g;
    a.iobs = iobs;
    a.alpha = alpha;
    a.slots = slots;
    return a;
}

// The per-launch part: kb reverse steps reading lambda^top, stage times and
// source phases of the forward steps top-1 .. top-kb; the dL/dw rows are
// injected when `inject` is set.  With a.moving the source follows the
// orbit table from its first entry (forward step k used entries 2k and
// 2k + 1): r*0 and the phase come from the table, as in the forward step.
void adjoint_launch_args(const teuk_ctx* c, AdjArgs& a, int kb, int64_t top, double t_start, bool inject) {
    const Geometry& geo = c->geo;
    a.kb = kb;
    a.n_strips = (int)((geo.nr + (WAVE - 2 * kb) - 1) / (WAVE - 2 * kb));
    for (int k = 0; k < KB_MAX; ++k) {
        const int64_t step = top - 1 - k;   // forward step reversed by stage k
        const double t0 = t_start + double(step) * c->dt, t1 = t0 + 0.5 * c->dt;
        double w0 = geo.m * c->Omega * t0, w1 = geo.m * c->Omega * t1;
        if (a.moving) {
            const int64_t e = std::min<int64_t>(std::max<int64_t>(2 * step, 0), c->traj_n - 2);   // k >= kb: unused
            const double* ent = &c->traj[2 * e];
            a.rs0[2 * k] = rstar_of_delta(ent[0] - geo.rp, geo.a, geo.M);
            a.rs0[2 * k + 1] = rstar_of_delta(ent[2] - geo.rp, geo.a, geo.M);
            w0 = geo.m * ent[1];
            w1 = geo.m * ent[3];
        }
        a.t[2 * k] = t0;
        a.t[2 * k + 1] = t1;
        a.ph[2 * k][0] = std::cos(w0);
        a.ph[2 * k][1] = -std::sin(w0);
        a.ph[2 * k + 1][0] = std::cos(w1);
        a.ph[2 * k + 1][1] = -std::sin(w1);
        a.g_row[k] = (inject && k < kb) ? step : -1;
    }
}

// The reverse sweep.  Static source: res_host gets the three sums
// (sum Re c, sum Re c x, sum t Im c).  Moving source (moving_host != NULL):
// moving_host gets [2n][3], the sums (Re c, Re c x, Im c) of every table
// entry the n forward steps used.
int adjoint_sweep(teuk_ctx* c, int iobs, double alpha, const double* g, int64_t n, double t_start, char* ws,
                  double* dphi0, double* dpi0, double* res_host, double* moving_host = nullptr) {
    const bool moving = moving_host != nullptr;
    const Geometry& geo = c->geo;
    const AdjLayout lay = adjoint_layout(c);
    const int64_t npts = geo.nr * geo.nth;
    const int64_t n_slots = adjoint_slots_used(c);
    double* wl[2] = {(double*)(ws + lay.lam), (double*)(ws + lay.lam) + 2 * npts};
    double* slots = (double*)(ws + lay.slots);
    double* result = (double*)(ws + lay.result);
    double* mout = (double*)(ws + lay.mout);
    // launches from the top: kb steps each, the odd remainder last
    std::vector<int> plan;
    for (int64_t r = n; r > 0;) {
        const int kb = (c->adj_kb >= 2 && r >= 2) ? 2 : 1;
        plan.push_back(kb);
        r -= kb;
    }
    // start in the pair that makes the last launch write (dphi0, dpi0)
    double* pair[2][2] = {{dphi0, dpi0}, {wl[0], wl[1]}};
    int cur = (plan.size() % 2 == 1) ? 1 : 0;
    launch_adjoint_init(pair[cur][0], pair[cur][1], g + 2 * n * geo.nth, npts, (int)geo.nr, iobs, alpha, c->stream);
    HIP_TRY(c, hipGetLastError());
    if (!moving) {
        launch_fill_zero(slots, n_slots * 3, c->stream);
        HIP_TRY(c, hipGetLastError());
    }
    AdjArgs a = adjoint_args(c, g, iobs, alpha, slots);
    double* mbuf[2] = {slots, slots + lay.n_slots * 6 * KB_MAX};   // alternate launches
    int64_t launch = 0;
    if (moving) {
        const double sr = c->sig_r * geo.dr;
        a.moving = 1;
        a.mout = mout;
        a.inv_sr2 = 1.0 / (sr * sr);
        a.two_sr2 = 2.0 * sr * sr;
        a.rmin = geo.rmin;
        a.dr = geo.dr;
    }
    int64_t top = n;   // this launch reads lambda^top
    for (int kb : plan) {
        if (moving) {
            // the previous launch's slots are reduced by block 0 of this one
            a.prev_mslots = launch > 0 ? a.mslots : nullptr;
            a.prev_n_slots = (int64_t)((a.n_strips + WG_WAVES - 1) / WG_WAVES) * a.n_chunks * WG_WAVES;
            a.prev_kb = a.kb;
            a.prev_top = top + a.kb;
            a.mslots = mbuf[launch & 1];
        }
        adjoint_launch_args(c, a, kb, top, t_start, true);
        a.lp = pair[cur][0];
        a.lq = pair[cur][1];
        a.lp_out = pair[1 - cur][0];
        a.lq_out = pair[1 - cur][1];
        launch_adjoint_step(a, c->stream);
        HIP_TRY(c, hipGetLastError());
        ++launch;
        cur = 1 - cur;
        top -= kb;
    }
    if (moving) {
        if (launch > 0) {
            // the last launch's slots, over its own grid (a one-step
            // remainder has fewer blocks); it reversed steps top .. top+kb-1
            const int64_t last_slots = (int64_t)((a.n_strips + WG_WAVES - 1) / WG_WAVES) * a.n_chunks * WG_WAVES;
            launch_moving_slot_sum(a.mslots, last_slots, a.kb, top + a.kb, mout, c->stream);
            HIP_TRY(c, hipGetLastError());
        }
        HIP_TRY(c, hipMemcpyAsync(moving_host, mout, (size_t)(2 * n * 3) * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        return TEUK_OK;
    }
    launch_slot_sum(slots, n_slots, result, c->stream);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipMemcpyAsync(res_host, result, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TEUK_OK;
}

// Seconds per reverse step of `launches` trial launches at the context's
// reverse-sweep tiling.  The trial reads the bound state's current pair as
// lambda and writes the other pair, which is scratch between forward steps,
// so the state, the step count and the waveform are left as they were; the
// gradient slots go to `slots` (room for adjoint_slots_max entries).
int adjoint_time_trial(teuk_ctx* c, int launches, double* slots, double* sec_per_step) {
    const int kb = c->adj_kb;
    launch_fill_zero(slots, adjoint_slots_used(c) * 3, c->stream);
    HIP_TRY(c, hipGetLastError());
    AdjArgs a = adjoint_args(c, nullptr, 0, 0.0, slots);
    adjoint_launch_args(c, a, kb, kb, 0.0, false);
    a.lp = (const double*)c->buf[c->cur][0];
    a.lq = (const double*)c->buf[c->cur][1];
    a.lp_out = (double*)c->buf[1 - c->cur][0];
    a.lq_out = (double*)c->buf[1 - c->cur][1];
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(c, TEUK_EDEVICE, "hipEventCreate failed");
    }
    int rc = TEUK_OK;
    launch_adjoint_step(a, c->stream);   // warm-up
    if (hipGetLastError() != hipSuccess) rc = fail(c, TEUK_EDEVICE, "reverse-step launch failed");
    if (rc == TEUK_OK && hipEventRecord(e0, c->stream) != hipSuccess) rc = fail(c, TEUK_EDEVICE, "event record");
    for (int k = 0; rc == TEUK_OK && k < launches; ++k) {
        launch_adjoint_step(a, c->stream);
        if (hipGetLastError() != hipSuccess) rc = fail(c, TEUK_EDEVICE, "reverse-step launch failed");
    }
    if (rc == TEUK_OK && hipEventRecord(e1, c->stream) != hipSuccess) rc = fail(c, TEUK_EDEVICE, "event record");
    float ms = 0.0f;
    if (rc == TEUK_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = fail(c, TEUK_EDEVICE, "event timing");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == TEUK_OK) *sec_per_step = 1e-3 * ms / double(launches * kb);
    return rc;
}

}  // namespace

// Context accessors for the library's other translation units.
namespace teuk {
int ctx_device(const teuk_ctx* c) { return c->device; }
int ctx_fail(teuk_ctx* c, int code, const char* msg) { return fail(c, code, "%s", msg); }
}  // namespace teuk

extern "C" {

static int init_ctx(teuk_ctx* c, const teuk_grid* g, double a, double M, int32_t m, int32_t s, double dt,
                    int32_t prec, void* hip_stream) {
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
        hipMalloc((void**)&c->d_flag, sizeof(unsigned int)) != hipSuccess)
        return TEUK_EDEVICE;
    if (upload_tables(c) != TEUK_OK) return TEUK_EDEVICE;
    return TEUK_OK;
}

int teuk_create(const teuk_grid* g, double a, double M, int32_t m, int32_t s, double dt, int32_t prec,
                void* hip_stream, teuk_ctx** out) {
    if (!out) return TEUK_EINVAL;
    *out = nullptr;
    if (validate_phys(g, a, M, s) != TEUK_OK) return TEUK_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return TEUK_EINVAL;
    if (prec != TEUK_FP64 && prec != TEUK_FP32 && prec != TEUK_FP32S) return TEUK_EINVAL;
    if (m < -1000 || m > 1000) return TEUK_EINVAL;
    teuk_ctx* c = new (std::nothrow) teuk_ctx();
    if (!c) return TEUK_EDEVICE;
    int rc;
    try {
        rc = init_ctx(c, g, a, M, m, s, dt, prec, hip_stream);
    } catch (...) {  // host allocation or thread start failed; no C++ exception crosses the ABI
        rc = TEUK_EDEVICE;
    }
    if (rc != TEUK_OK) {
        teuk_destroy(c);
        return rc;
    }
    *out = c;
    return TEUK_OK;
}

int teuk_destroy(teuk_ctx* c) {
    if (!c) return TEUK_EINVAL;
    if (c->d_rad_i || c->d_rad_h || c->d_ang || c->d_flag || c->d_watch) (void)hipStreamSynchronize(c->stream);
    if (c->d_rad_i) (void)hipFree(c->d_rad_i);
    if (c->d_rad_h) (void)hipFree(c->d_rad_h);
    if (c->d_ang) (void)hipFree(c->d_ang);
    if (c->d_flag) (void)hipFree(c->d_flag);
    if (c->d_watch) (void)hipFree(c->d_watch);
    if (c->h_watch) (void)hipHostFree((void*)c->h_watch);
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

static int teuk_set_source_impl(teuk_ctx* c, double r0, double amp, double sigma_r_cells, double sigma_th_cells) {
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
    c->Omega = orbit_omega(r0, g.a, g.M);
    c->has_src = true;
    build_source(g, c->rstar0, sigma_r_cells * g.dr, sigma_th_cells * g.dth, amp);
    return upload_tables(c);
}

int teuk_set_source(teuk_ctx* c, double r0, double amp, double sigma_r_cells, double sigma_th_cells) {
    try {
        return teuk_set_source_impl(c, r0, amp, sigma_r_cells, sigma_th_cells);
    } catch (...) {  // no C++ exception crosses the ABI
        return fail(c, TEUK_EDEVICE, "host allocation or thread start failed");
    }
}

static int teuk_set_trajectory_impl(teuk_ctx* c, const double* r0_phase, int64_t n_half) {
    if (!c) return TEUK_EINVAL;
    if (!r0_phase) {
        c->traj.clear();
        c->traj_n = 0;
        return TEUK_OK;
    }
    if (!c->has_src) return fail(c, TEUK_ESTATE, "teuk_set_source must come first (amplitude and widths)");
    if (n_half < 2 || n_half > ((int64_t)1 << 34)) return fail(c, TEUK_EINVAL, "n_half must be 2..2^34");
    for (int64_t k = 0; k < n_half; ++k)
        if (!(r0_phase[2 * k] > c->geo.rp) || !std::isfinite(r0_phase[2 * k]) || !std::isfinite(r0_phase[2 * k + 1]))
            return fail(c, TEUK_EINVAL, "orbit entry %lld: r0 must exceed r+ and both values be finite", (long long)k);
    c->traj.assign(r0_phase, r0_phase + 2 * n_half);
    c->traj_n = n_half;
    c->traj_step0 = c->step;
    return TEUK_OK;
}

int teuk_set_trajectory(teuk_ctx* c, const double* r0_phase, int64_t n_half) {
    try {
        return teuk_set_trajectory_impl(c, r0_phase, n_half);
    } catch (...) {  // no C++ exception crosses the ABI
        return fail(c, TEUK_EDEVICE, "host allocation or thread start failed");
    }
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

static int teuk_step_impl(teuk_ctx* c, int64_t n) {
    if (!c) return TEUK_EINVAL;
    if (watch_poll(c) != TEUK_OK) return c->status;
    if (n < 0) return fail(c, TEUK_EINVAL, "negative step count");
    if (!c->bound) return fail(c, TEUK_ESTATE, "no state bound");
    if (n == 0 && !c->wave) return TEUK_OK;
    if (c->traj_n > 0) {
        const int64_t s0 = c->step - c->traj_step0;
        // step s (counted from the call) reads entries 2s and 2s + 1
        if (s0 < 0 || (n > 0 && 2 * (s0 + n) > c->traj_n))
            return fail(c, TEUK_EINVAL, "steps %lld..%lld since the trajectory was set need %lld orbit entries, "
                        "it has %lld", (long long)s0, (long long)(s0 + n - 1), (long long)(2 * (s0 + n)),
                        (long long)c->traj_n);
    }
    if (c->prec != TEUK_FP32) return launch_steps<double>(c, n);
    return launch_steps<float>(c, n);
}

int teuk_step(teuk_ctx* c, int64_t n) {
    try {
        return teuk_step_impl(c, n);
    } catch (...) {  // no C++ exception crosses the ABI
        return fail(c, TEUK_EDEVICE, "host allocation or thread start failed");
    }
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

int teuk_set_time(teuk_ctx* c, double t, int64_t step) { return teuk_set_clock(c, t, step, step); }

int teuk_get_clock(teuk_ctx* c, double* t0, int64_t* step0, int64_t* step) {
    if (!c) return TEUK_EINVAL;
    if (t0) *t0 = c->t0;
    if (step0) *step0 = c->step0;
    if (step) *step = c->step;
    return TEUK_OK;
}

int teuk_set_clock(teuk_ctx* c, double t0, int64_t step0, int64_t step) {
    if (!c || !std::isfinite(t0)) return TEUK_EINVAL;
    c->t0 = t0;
    c->step0 = step0;
    // the observer rows and the orbit table stay attached to the same steps
    c->obs_step0 += step - c->step;
    c->traj_step0 += step - c->step;
    c->step = step;
    return TEUK_OK;
}

int teuk_current(teuk_ctx* c) {
    if (!c) return TEUK_EINVAL;
    return c->cur;
}

int teuk_set_tiling(teuk_ctx* c, int32_t rows_per_wave, int32_t order) {
    if (!c) return TEUK_EINVAL;
    if (order < 0 || order > 2) return fail(c, TEUK_EINVAL, "order must be 0, 1 or 2");
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

static int teuk_autotune_impl(teuk_ctx* c, int32_t launches_per_trial, int32_t* rows_out, int32_t* kb_out) {
    if (!c) return TEUK_EINVAL;
    if (c->status != TEUK_OK) return c->status;
    if (!c->bound) return fail(c, TEUK_ESTATE, "no state bound");
    if (launches_per_trial < 1 || launches_per_trial > 10000)
        return fail(c, TEUK_EINVAL, "launches_per_trial must be 1..10000");
    // 80 and 112: on 32768 x 1024 FP32 at 80 rows ran 1-3 % faster than at
    // any other height, and FP64 at 112 as fast as at 96
    static const int kRows[] = {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 80, 96, 112, 128, 192, 256};
    const int nth = (int)c->geo.nth;
    const int keep_rows = c->rows, keep_kb = c->kblock, keep_order = c->order;
    const bool keep_default = c->rows_default;
    // launch forms: one step per launch; two fused steps on one wavefront
    // (block order 0 chunk-major, 1 group-major) or on a pair of wavefronts
    // (order 2).  Every candidate is timed twice, the second pass in the
    // reverse order, and keeps its faster trial, so that neither a drift
    // over the trials nor one slow trial decides (see the reverse sweep's
    // tuner below).
    static const int kForms[][2] = {{1, 0}, {2, 0}, {2, 1}, {2, 2}};
    struct Cand {
        int rows, kb, order;
        double sec;
    };
    std::vector<Cand> cand;
    for (const auto& form : kForms) {
        int prev = 0;
        for (int r : kRows) {
            const int rows = std::min(r, nth);
            if (rows == prev) continue;   // candidates clipped to n_theta repeat
            prev = rows;
            cand.push_back({rows, form[0], form[1], 0.0});
        }
    }
    const int nc = (int)cand.size();
    for (int pass = 0; pass < 2; ++pass) {
        for (int j = 0; j < nc; ++j) {
            Cand& x = cand[pass == 0 ? j : nc - 1 - j];
            c->rows = x.rows;
            c->kblock = x.kb;
            c->order = x.order;
            double sec = 0.0;
            int rc = (c->prec != TEUK_FP32) ? time_trial<double>(c, launches_per_trial, &sec)
                                     : time_trial<float>(c, launches_per_trial, &sec);
            if (rc != TEUK_OK) {
                c->rows = keep_rows;
                c->kblock = keep_kb;
                c->order = keep_order;
                c->rows_default = keep_default;
                return rc;
            }
            if (pass == 0 || sec < x.sec) x.sec = sec;
        }
    }
    double best = 0.0;
    int best_rows = keep_rows, best_kb = keep_kb, best_order = 0;
    for (const Cand& x : cand) {
        if (best == 0.0 || x.sec < best) {
            best = x.sec;
            best_rows = x.rows;
            best_kb = x.kb;
            best_order = x.order;
        }
    }
    c->rows = best_rows;
    c->kblock = best_kb;
    c->order = best_order;
    c->rows_default = false;
    if (rows_out) *rows_out = best_rows;
    if (kb_out) *kb_out = best_kb;
    return TEUK_OK;
}

int teuk_autotune(teuk_ctx* c, int32_t launches_per_trial, int32_t* rows_out, int32_t* kb_out) {
    try {
        return teuk_autotune_impl(c, launches_per_trial, rows_out, kb_out);
    } catch (...) {  // no C++ exception crosses the ABI
        return fail(c, TEUK_EDEVICE, "host allocation or thread start failed");
    }
}

int teuk_get_tiling(teuk_ctx* c, int32_t* rows_per_wave, int32_t* order) {
    if (!c) return TEUK_EINVAL;
    if (rows_per_wave) *rows_per_wave = c->rows;
    if (order) *order = c->order;
    return TEUK_OK;
}

int teuk_set_adjoint_tiling(teuk_ctx* c, int32_t rows_per_wave, int32_t steps_per_launch) {
    if (!c) return TEUK_EINVAL;
    if (rows_per_wave < 0 || rows_per_wave > 4096) return fail(c, TEUK_EINVAL, "rows_per_wave out of range");
    if (steps_per_launch < 1 || steps_per_launch > KB_MAX)
        return fail(c, TEUK_EINVAL, "steps_per_launch must be 1..%d", KB_MAX);
    c->adj_rows = rows_per_wave;
    c->adj_kb = steps_per_launch;
    return TEUK_OK;
}

int teuk_get_adjoint_tiling(teuk_ctx* c, int32_t* rows_per_wave, int32_t* steps_per_launch) {
    if (!c) return TEUK_EINVAL;
    if (rows_per_wave) *rows_per_wave = adjoint_rows(c);
    if (steps_per_launch) *steps_per_launch = c->adj_kb;
    return TEUK_OK;
}

// The candidates are timed twice, the second pass in the reverse order, and
// each keeps its faster trial: a single pass in a fixed order (every
// one-step candidate first) picked two-step launches on 4096 x 256 with 40
// launches per trial although one step per launch ran the whole sweep 7 %
// faster.
static int adjoint_autotune_trials(teuk_ctx* c, int32_t launches_per_trial, double* slots, int* best_rows,
                                   int* best_kb) {
    static const int kRows[] = {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256};
    const int nth = (int)c->geo.nth;
    struct Cand {
        int rows, kb;
        double sec;
    };
    std::vector<Cand> cand;
    for (int kb = 1; kb <= KB_MAX; ++kb) {
        int prev = 0;
        for (int r : kRows) {
            const int rows = std::min(r, nth);
            if (rows == prev) continue;   // candidates clipped to n_theta repeat
            prev = rows;
            cand.push_back({rows, kb, 0.0});
        }
    }
    const int nc = (int)cand.size();
    for (int pass = 0; pass < 2; ++pass) {
        for (int j = 0; j < nc; ++j) {
            Cand& x = cand[pass == 0 ? j : nc - 1 - j];
            c->adj_rows = x.rows;
            c->adj_kb = x.kb;
            double sec = 0.0;
            const int rc = adjoint_time_trial(c, launches_per_trial, slots, &sec);
            if (rc != TEUK_OK) return rc;
            if (pass == 0 || sec < x.sec) x.sec = sec;
        }
    }
    double best = 0.0;
    for (const Cand& x : cand) {
        if (best == 0.0 || x.sec < best) {
            best = x.sec;
            *best_rows = x.rows;
            *best_kb = x.kb;
        }
    }
    return TEUK_OK;
}

int teuk_adjoint_autotune(teuk_ctx* c, int32_t launches_per_trial, int32_t* rows_out, int32_t* kb_out) {
    if (!c) return TEUK_EINVAL;
    if (c->status != TEUK_OK) return c->status;
    if (c->prec != TEUK_FP64) return fail(c, TEUK_ENOTSUP, "the reverse sweep is FP64 only");
    if (!c->bound) return fail(c, TEUK_ESTATE, "no state bound");
    if (launches_per_trial < 1 || launches_per_trial > 10000)
        return fail(c, TEUK_EINVAL, "launches_per_trial must be 1..10000");
    double* slots = nullptr;
    HIP_TRY(c, hipMalloc((void**)&slots, adjoint_slots_max(c->geo) * 3 * sizeof(double)));
    const int keep_rows = c->adj_rows, keep_kb = c->adj_kb;
    int best_rows = adjoint_rows(c), best_kb = keep_kb;
    const int rc = adjoint_autotune_trials(c, launches_per_trial, slots, &best_rows, &best_kb);
    (void)hipStreamSynchronize(c->stream);   // the trials are done with the slots
    (void)hipFree(slots);
    if (rc != TEUK_OK) {
        c->adj_rows = keep_rows;
        c->adj_kb = keep_kb;
        return rc;
    }
    c->adj_rows = best_rows;
    c->adj_kb = best_kb;
    if (rows_out) *rows_out = best_rows;
    if (kb_out) *kb_out = best_kb;
    return TEUK_OK;
}

int64_t teuk_adjoint_workspace_bytes(teuk_ctx* c) {
    if (!c) return TEUK_EINVAL;
    if (c->prec != TEUK_FP64) return TEUK_ENOTSUP;
    return adjoint_layout(c).total;
}

// Checks shared by both reverse-sweep entry points; finds the observer.
static int adjoint_check(teuk_ctx* c, double rstar_obs, const void* dL_dwave, int64_t n_steps, void* workspace,
                         int64_t workspace_bytes, void* dL_dphi0, void* dL_dpi0, int* iobs, double* alpha) {
    if (c->status != TEUK_OK) return c->status;
    if (c->prec != TEUK_FP64) return fail(c, TEUK_ENOTSUP, "the reverse sweep is FP64 only");
    if (n_steps < 0) return fail(c, TEUK_EINVAL, "negative step count");
    if (!dL_dwave || !workspace || !dL_dphi0 || !dL_dpi0) return fail(c, TEUK_EINVAL, "NULL buffer");
    if ((uintptr_t)workspace % 256 != 0) return fail(c, TEUK_EINVAL, "workspace not 256-byte aligned");
    if ((uintptr_t)dL_dwave % 16 != 0 || (uintptr_t)dL_dphi0 % 16 != 0 || (uintptr_t)dL_dpi0 % 16 != 0)
        return fail(c, TEUK_EINVAL, "dL_dwave, dL_dphi0 and dL_dpi0 must be 16-byte aligned");
    if (dL_dphi0 == dL_dpi0) return fail(c, TEUK_EINVAL, "dL_dphi0 and dL_dpi0 alias");
    const AdjLayout lay = adjoint_layout(c);
    if (workspace_bytes < lay.total)
        return fail(c, TEUK_EINVAL, "workspace of %lld B is smaller than the %lld B needed", (long long)workspace_bytes,
                    (long long)lay.total);
    const Geometry& g = c->geo;
    const int64_t nb = 2 * g.nr * g.nth * 16;
    auto overlap = [](const void* a, int64_t na, const void* b, int64_t nbb) {
        return (const char*)a < (const char*)b + nbb && (const char*)b < (const char*)a + na;
    };
    if (overlap(workspace, lay.total, dL_dphi0, nb / 2) || overlap(workspace, lay.total, dL_dpi0, nb / 2) ||
        overlap(dL_dphi0, nb / 2, dL_dpi0, nb / 2))
        return fail(c, TEUK_EINVAL, "workspace and output buffers overlap");
    if (!observer_index(g, rstar_obs, *iobs, *alpha))
        return fail(c, TEUK_EINVAL, "rstar_obs = %g outside the open grid interval", rstar_obs);
    return TEUK_OK;
}

static int teuk_adjoint_impl(teuk_ctx* c, double rstar_obs, const void* dL_dwave, int64_t n_steps, double t_start,
                 void* workspace, int64_t workspace_bytes, void* dL_dphi0, void* dL_dpi0, double* dL_dr0,
                 double* dL_damp) {
    if (!c) return TEUK_EINVAL;
    if (c->traj_n > 0) return fail(c, TEUK_ENOTSUP, "a moving source's reverse sweep is teuk_adjoint_moving");
    if (!std::isfinite(t_start)) return fail(c, TEUK_EINVAL, "non-finite t_start");
    int iobs;
    double alpha;
    int rc = adjoint_check(c, rstar_obs, dL_dwave, n_steps, workspace, workspace_bytes, dL_dphi0, dL_dpi0, &iobs,
                           &alpha);
    if (rc != TEUK_OK) return rc;
    const Geometry& g = c->geo;
    double res[3] = {0.0, 0.0, 0.0};
    rc = adjoint_sweep(c, iobs, alpha, (const double*)dL_dwave, n_steps, t_start, (char*)workspace,
                       (double*)dL_dphi0, (double*)dL_dpi0, res);
    if (rc != TEUK_OK) return rc;
    // dT/damp = G e^{-i m Omega t};
    // dT/dr0 = amp G e^{-i m Omega t} [x dr*0/dr0 - i m t dOmega/dr0],
    // x = (r* - r*0)/sr^2, dr*/dr = (r^2 + a^2)/Delta (Eq. 2).
    double damp = 0.0, dr0 = 0.0;
    if (c->has_src) {
        const double r0 = c->r0, a = g.a, M = g.M;
        const double drs0 = (r0 * r0 + a * a) / (r0 * r0 - 2.0 * M * r0 + a * a);
        const double den = std::pow(r0, 1.5) + a * std::sqrt(M);
        const double dOm = -1.5 * std::sqrt(M) * std::sqrt(r0) / (den * den);
        damp = res[0];
        dr0 = c->amp * (drs0 * res[1] + double(g.m) * dOm * res[2]);
    }
    if (dL_damp) *dL_damp = damp;
    if (dL_dr0) *dL_dr0 = dr0;
    return TEUK_OK;
}

static int teuk_adjoint_moving_impl(teuk_ctx* c, double rstar_obs, const void* dL_dwave, int64_t n_steps,
                                    void* workspace, int64_t workspace_bytes, void* dL_dphi0, void* dL_dpi0,
                                    double* dL_dtraj, double* dL_damp) {
    if (!c) return TEUK_EINVAL;
    if (c->traj_n == 0) return fail(c, TEUK_ESTATE, "no orbit table: teuk_set_trajectory comes first");
    if (n_steps > 0 && !dL_dtraj) return fail(c, TEUK_EINVAL, "NULL dL_dtraj");
    if (2 * n_steps > c->traj_n)
        return fail(c, TEUK_EINVAL, "%lld steps need %lld orbit entries, the table has %lld", (long long)n_steps,
                    (long long)(2 * n_steps), (long long)c->traj_n);
    int iobs;
    double alpha;
    int rc = adjoint_check(c, rstar_obs, dL_dwave, n_steps, workspace, workspace_bytes, dL_dphi0, dL_dpi0, &iobs,
                           &alpha);
    if (rc != TEUK_OK) return rc;
    std::vector<double> sums((size_t)(2 * n_steps * 3) + 3);
    rc = adjoint_sweep(c, iobs, alpha, (const double*)dL_dwave, n_steps, 0.0, (char*)workspace,
                       (double*)dL_dphi0, (double*)dL_dpi0, nullptr, sums.data());
    if (rc != TEUK_OK) return rc;
    // per entry e, with c = conj(a_T) U (U: unit-amplitude source):
    // dL/dr0_e = amp dr*/dr(r0_e) sum Re c x, dL/dphi_e = amp m sum Im c,
    // dL/damp = sum over entries of sum Re c (summed here in entry order)
    const Geometry& g = c->geo;
    double damp = 0.0;
    for (int64_t e = 0; e < 2 * n_steps; ++e) {
        const double r0 = c->traj[2 * e];
        const double drs0 = (r0 * r0 + g.a * g.a) / (r0 * r0 - 2.0 * g.M * r0 + g.a * g.a);
        const double* v = &sums[3 * e];
        damp += v[0];
        dL_dtraj[2 * e] = c->amp * drs0 * v[1];
        dL_dtraj[2 * e + 1] = c->amp * double(g.m) * v[2];
    }
    if (dL_damp) *dL_damp = damp;
    return TEUK_OK;
}

int teuk_adjoint_moving(teuk_ctx* c, double rstar_obs, const void* dL_dwave, int64_t n_steps, void* workspace,
                        int64_t workspace_bytes, void* dL_dphi0, void* dL_dpi0, double* dL_dtraj, double* dL_damp) {
    try {
        return teuk_adjoint_moving_impl(c, rstar_obs, dL_dwave, n_steps, workspace, workspace_bytes, dL_dphi0,
                                        dL_dpi0, dL_dtraj, dL_damp);
    } catch (...) {  // no C++ exception crosses the ABI
        return fail(c, TEUK_EDEVICE, "host allocation failed");
    }
}

int teuk_adjoint(teuk_ctx* c, double rstar_obs, const void* dL_dwave, int64_t n_steps, double t_start,
                 void* workspace, int64_t workspace_bytes, void* dL_dphi0, void* dL_dpi0, double* dL_dr0,
                 double* dL_damp) {
    try {
        return teuk_adjoint_impl(c, rstar_obs, dL_dwave, n_steps, t_start, workspace, workspace_bytes, dL_dphi0, dL_dpi0, dL_dr0, dL_damp);
    } catch (...) {  // no C++ exception crosses the ABI
        return fail(c, TEUK_EDEVICE, "host allocation or thread start failed");
    }
}

// ------------------------------------------------------- parameter gradients

// Launch arguments of one FP64 step of x (its tables, source and tiling; one
// step per launch) from (ip, iq) into (op, oq) at time t, with a
// fixed-orbit source; no waveform is recorded.
static StepArgs<double> step_args_at(teuk_ctx* x, const double* ip, const double* iq, double* op, double* oq,
                                     double t, int rows, int kb = 1) {
    const Geometry& g = x->geo;
    StepArgs<double> a = step_args<double>(x);
    a.kb = kb;
    a.rows = rows;
    a.n_chunks = (int)((g.nth + rows - 1) / rows);
    const int so = WAVE - 2 * kb;
    a.n_strips = (int)((g.nr + so - 1) / so);
    a.n_tiles = a.n_strips * a.n_chunks;
    for (int q = 0; q < KB_MAX; ++q) {
        const double tq = t + double(q) * x->dt;
        const double w0 = g.m * x->Omega * tq, w1 = g.m * x->Omega * (tq + 0.5 * x->dt);
        a.ph[2 * q][0] = std::cos(w0);
        a.ph[2 * q][1] = -std::sin(w0);
        a.ph[2 * q + 1][0] = std::cos(w1);
        a.ph[2 * q + 1][1] = -std::sin(w1);
        a.wave_row[q] = -1;
    }
    a.phi = ip;
    a.pi = iq;
    a.phi_out = op;
    a.pi_out = oq;
    return a;
}

// kb FP64 steps of x (one launch) from (ip, iq) into (op, oq) from time
// t, `rows` theta rows per wave (see step_args_at; kb = 2 in the launch
// form of x's tiling); leaves x's bound state, step count and time alone.
static int step_at(teuk_ctx* x, const double* ip, const double* iq, double* op, double* oq, double t, int rows,
                   int kb = 1) {
    launch_step_fp64(step_args_at(x, ip, iq, op, oq, t, rows, kb), x->stream);
    HIP_TRY(x, hipGetLastError());
    return TEUK_OK;
}

// Theta rows per wave of the parameter sweep's one-step launches (the
// recomputed forward steps and the fused contraction, 4 wavefronts per
// workgroup).  The context's rows are tuned for its own launches, often two
// fused steps on tall chunks, which leave a one-step launch of a mid-size
// grid short of workgroups.  A launch takes ceil(blocks / resident) rounds
// of workgroups, each about as long as its chunk plus 2 halo rows, and the
// contraction does two steps' work per point: the height r from 1 to 16
// (the one-step default) that minimises (2 rounds_pdot + rounds_step)(r + 2)
// is taken, the tallest on a tie.  It depends on the grid and the device
// only, so results repeat bit for bit.  On 4096 x 256 (256 CUs, 2 and 3
// resident workgroups per CU) the model ranks 9 and 10 rows first; 10 rows
// measured 1.80 s for the sweep against 1.88 s at 6, 2.00 s at 8 and
// 2.12 s at 16.
static int sweep_rows(const Geometry& g, int cus, int pdot_per_cu, int step_per_cu) {
    const int64_t groups = ((g.nr + WAVE - 3) / (WAVE - 2) + WG_WAVES - 1) / WG_WAVES;   // strip groups
    const int64_t cap_p = (int64_t)pdot_per_cu * cus, cap_s = (int64_t)step_per_cu * cus;
    const int top = (int)std::min<int64_t>(16, g.nth);
    int best = 1;
    int64_t best_cost = -1;
    for (int r = 1; r <= top; ++r) {
        const int64_t blocks = groups * ((g.nth + r - 1) / r);
        const int64_t cost = (2 * ((blocks + cap_p - 1) / cap_p) + (blocks + cap_s - 1) / cap_s) * (r + 2);
        if (best_cost < 0 || cost <= best_cost) {
            best_cost = cost;
            best = r;
        }
    }
    return best;
}

// sweep_rows for c's grid on c's device; 0 if the device cannot be queried.
static int sweep_rows(const teuk_ctx* c) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || cus < 1)
        return 0;
    int pdot_per_cu = 1, step_per_cu = 1;
    sweep_blocks_per_cu(&pdot_per_cu, &step_per_cu);
    return sweep_rows(c->geo, cus, pdot_per_cu, step_per_cu);
}

// Workspace of a parameter gradient: two adjoint pairs, the reverse step's
// gradient slots, ceil(n / C) checkpoints, C - 1 segment states, the fused
// contraction's per-tile parts for each step of a segment (summed once per
// segment) and one double per step.  A state is Phi and Pi, complex128
// [nth][nr] each.  rows: the sweep's theta rows per wave (sweep_rows).
struct ParamLayout {
    int64_t state, lam, slots, ckpt, seg, parts, n_parts, res, total, n_ckpt;
};
static ParamLayout param_layout(const teuk_ctx* c, int64_t n, int64_t C, int rows) {
    ParamLayout L;
    const int64_t npts = c->geo.nr * c->geo.nth;
    const int64_t strips1 = (c->geo.nr + WAVE - 3) / (WAVE - 2);   // strips of a one-step launch
    L.state = round256(2 * npts * 16);
    L.n_ckpt = n > 0 ? (n + C - 1) / C : 1;
    L.n_parts = strips1 * ((c->geo.nth + rows - 1) / rows);
    L.lam = 0;
    L.slots = L.lam + 2 * L.state;
    L.ckpt = L.slots + round256(adjoint_slots_max(c->geo) * 3 * 8);
    L.seg = L.ckpt + L.n_ckpt * L.state;
    L.parts = L.seg + std::max<int64_t>(C - 1, 0) * L.state;
    L.res = L.parts + round256(std::max<int64_t>(std::min(C, n), 1) * L.n_parts * 8);
    L.total = L.res + round256(std::max<int64_t>(n, 1) * 8);
    return L;
}

static int64_t default_interval(int64_t n) {
    int64_t C = (int64_t)std::ceil(std::sqrt((double)std::max<int64_t>(n, 1)));
    return std::max<int64_t>(C, 1);
}

// The checkpointed sweep: forward from u^0 keeping every C-th state, then
// segment by segment from the last, recompute the segment's states from its
// checkpoint, and for each step k (descending) contract lambda^{k+1} with
// step_{p+h}(u^k) - step_{p-h}(u^k) (one fused launch, lw_pdot_kernel, that
// does not store the two steps) and take the reverse step to lambda^k.
static int param_sweep(teuk_ctx* c, teuk_ctx* xp, teuk_ctx* xm, int iobs, double alpha, const double* g, int64_t n,
                       double t_start, const double* phi0, const double* pi0, int64_t C, int rows, char* ws,
                       std::vector<double>& res, const double** lam0) {
    const Geometry& geo = c->geo;
    const ParamLayout L = param_layout(c, n, C, rows);
    const int64_t npts = geo.nr * geo.nth;
    auto state = [&](int64_t off) { return (double*)(ws + off); };
    auto pi_of = [&](double* phi) { return phi + 2 * npts; };
    double* lam[2] = {state(L.lam), state(L.lam + L.state)};
    double* slots = state(L.slots);
    auto ckpt = [&](int64_t j) { return state(L.ckpt + j * L.state); };
    auto seg = [&](int64_t j, int64_t i) { return i == 0 ? ckpt(j) : state(L.seg + (i - 1) * L.state); };
    double* parts = state(L.parts);
    double* dres = state(L.res);
    const double dt = c->dt;
    // forward pass, keeping u^{jC}
    HIP_TRY(c, hipMemcpyAsync(ckpt(0), phi0, npts * 16, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(pi_of(ckpt(0)), pi0, npts * 16, hipMemcpyDeviceToDevice, c->stream));
    // forward states between checkpoints alternate between the two adjoint
    // pairs, which are not in use yet; u^n itself is not needed.  Only every
    // C-th state is kept, so this pass takes the context's own launches, two
    // fused steps where no checkpoint falls between them (bitwise equal to
    // single steps).
    double* tmp[2] = {lam[0], lam[1]};
    double* cur = ckpt(0);
    for (int64_t k = 0; k + 1 < n;) {
        const int kb = (c->kblock == 2 && k + 2 < n && (k + 1) % C != 0) ? 2 : 1;
        double* next = ((k + kb) % C == 0) ? ckpt((k + kb) / C) : (cur == tmp[0] ? tmp[1] : tmp[0]);
        int rc = kb == 2 ? step_at(c, cur, pi_of(cur), next, pi_of(next), t_start + double(k) * dt, c->rows, 2)
                         : step_at(c, cur, pi_of(cur), next, pi_of(next), t_start + double(k) * dt, rows);
        if (rc != TEUK_OK) return rc;
        cur = next;
        k += kb;
    }
    // lambda^n = E^H g^n
    launch_adjoint_init(lam[0], pi_of(lam[0]), g + 2 * n * geo.nth, npts, (int)geo.nr, iobs, alpha, c->stream);
    HIP_TRY(c, hipGetLastError());
    launch_fill_zero(slots, adjoint_slots_max(geo) * 3, c->stream);
    HIP_TRY(c, hipGetLastError());
    AdjArgs a = adjoint_args(c, g, iobs, alpha, slots);
    if (pdot_parts(step_args_at(xp, nullptr, nullptr, nullptr, nullptr, t_start, rows)) != L.n_parts)
        return fail(c, TEUK_EINVAL, "contraction parts do not match the workspace layout");
    int li = 0;   // lam[li] holds lambda^{k+1}
    for (int64_t j = L.n_ckpt - 1; j >= 0 && n > 0; --j) {
        const int64_t k0 = j * C, k1 = std::min(k0 + C, n);
        for (int64_t i = 1; i < k1 - k0; ++i) {
            double* in = seg(j, i - 1);
            double* out = seg(j, i);
            int rc = step_at(c, in, pi_of(in), out, pi_of(out), t_start + double(k0 + i - 1) * dt, rows);
            if (rc != TEUK_OK) return rc;
        }
        for (int64_t k = k1 - 1; k >= k0; --k) {
            double* u = seg(j, k - k0);
            const double t = t_start + double(k) * dt;
            PdotArgs pd;
            pd.s[0] = step_args_at(xp, u, pi_of(u), nullptr, nullptr, t, rows);
            pd.s[1] = step_args_at(xm, u, pi_of(u), nullptr, nullptr, t, rows);
            pd.lp = lam[li];
            pd.lq = pi_of(lam[li]);
            pd.part = parts + (k - k0) * L.n_parts;
            launch_param_pdot(pd, u, pi_of(u), c->stream);
            HIP_TRY(c, hipGetLastError());
            adjoint_launch_args(c, a, 1, k + 1, t_start, true);
            a.lp = lam[li];
            a.lq = pi_of(lam[li]);
            a.lp_out = lam[1 - li];
            a.lq_out = pi_of(lam[1 - li]);
            launch_adjoint_step(a, c->stream);
            HIP_TRY(c, hipGetLastError());
            li = 1 - li;
        }
        // the segment's contractions, one fixed-order sum per step
        launch_pdot_sums(parts, L.n_parts, k1 - k0, dres + k0, c->stream);
        HIP_TRY(c, hipGetLastError());
    }
    res.assign((size_t)std::max<int64_t>(n, 0), 0.0);
    if (n > 0)
        HIP_TRY(c, hipMemcpyAsync(res.data(), dres, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *lam0 = lam[li];   // lambda^0
    return TEUK_OK;
}

int64_t teuk_param_gradient_workspace_bytes(teuk_ctx* c, int64_t n_steps, int64_t checkpoint_interval) {
    if (!c || n_steps < 0 || checkpoint_interval < 0) return TEUK_EINVAL;
    const int64_t C = checkpoint_interval > 0 ? checkpoint_interval : default_interval(n_steps);
    const int rows = sweep_rows(c);
    if (rows < 1) return TEUK_EDEVICE;
    return param_layout(c, n_steps, C, rows).total;
}

static int teuk_param_gradient_impl(teuk_ctx* c, int32_t param, double h, double rstar_obs, const void* dL_dwave,
                                    int64_t n_steps, double t_start, const void* phi0, const void* pi0,
                                    int64_t checkpoint_interval, void* workspace, int64_t workspace_bytes,
                                    double* dL_dparam, void* dL_dphi0, void* dL_dpi0) {
    if (!c) return TEUK_EINVAL;
    if (c->traj_n > 0) return fail(c, TEUK_ENOTSUP, "parameter gradients need a fixed orbit (no trajectory)");
    if (param < TEUK_PARAM_A || param > TEUK_PARAM_AMP) return fail(c, TEUK_EINVAL, "unknown parameter %d", param);
    if (!(h > 0.0) || !std::isfinite(h)) return fail(c, TEUK_EINVAL, "h must be positive and finite");
    if (!std::isfinite(t_start)) return fail(c, TEUK_EINVAL, "non-finite t_start");
    if (checkpoint_interval < 0) return fail(c, TEUK_EINVAL, "negative checkpoint interval");
    if (!dL_dparam) return fail(c, TEUK_EINVAL, "NULL dL_dparam");
    if (!phi0 || !pi0 || (uintptr_t)phi0 % 16 != 0 || (uintptr_t)pi0 % 16 != 0)
        return fail(c, TEUK_EINVAL, "phi0 and pi0 must be 16-byte aligned device buffers");
    if ((param == TEUK_PARAM_R0 || param == TEUK_PARAM_AMP) && !c->has_src)
        return fail(c, TEUK_ESTATE, "no source: teuk_set_source first");
    const int64_t C = checkpoint_interval > 0 ? checkpoint_interval : default_interval(n_steps);
    const int rows = sweep_rows(c);
    if (rows < 1) return fail(c, TEUK_EDEVICE, "compute unit count unavailable");
    const ParamLayout L = param_layout(c, n_steps, C, rows);
    if (!dL_dwave || !workspace) return fail(c, TEUK_EINVAL, "NULL buffer");
    if ((uintptr_t)workspace % 256 != 0) return fail(c, TEUK_EINVAL, "workspace not 256-byte aligned");
    if ((uintptr_t)dL_dwave % 16 != 0) return fail(c, TEUK_EINVAL, "dL_dwave must be 16-byte aligned");
    if (workspace_bytes < L.total)
        return fail(c, TEUK_EINVAL, "workspace of %lld B is smaller than the %lld B needed", (long long)workspace_bytes,
                    (long long)L.total);
    if ((dL_dphi0 == nullptr) != (dL_dpi0 == nullptr)) return fail(c, TEUK_EINVAL, "give both dL_dphi0 and dL_dpi0 or neither");
    if (c->status != TEUK_OK) return c->status;
    if (c->prec != TEUK_FP64) return fail(c, TEUK_ENOTSUP, "parameter gradients are FP64 only");
    if (n_steps < 0) return fail(c, TEUK_EINVAL, "negative step count");
    const Geometry& geo = c->geo;
    int iobs;
    double alpha;
    if (!observer_index(geo, rstar_obs, iobs, alpha))
        return fail(c, TEUK_EINVAL, "rstar_obs = %g outside the open grid interval", rstar_obs);
    // the two perturbed contexts: same grid, mode, dt, tiling and source, one parameter moved by +-h
    teuk_grid gr{geo.nr, geo.nth, geo.rmin, geo.rmax};
    double pa[2] = {geo.a, geo.a}, pM[2] = {geo.M, geo.M}, pr0[2] = {c->r0, c->r0}, pamp[2] = {c->amp, c->amp};
    double* moved = param == TEUK_PARAM_A ? pa : param == TEUK_PARAM_M ? pM : param == TEUK_PARAM_R0 ? pr0 : pamp;
    moved[0] += h;
    moved[1] -= h;
    struct Owned {   // the perturbed contexts are destroyed on every path
        teuk_ctx* p = nullptr;
        ~Owned() {
            if (p) teuk_destroy(p);
        }
    } own[2];
    teuk_ctx* x[2] = {nullptr, nullptr};
    int rc = TEUK_OK;
    for (int i = 0; i < 2 && rc == TEUK_OK; ++i) {
        if (validate_phys(&gr, pa[i], pM[i], geo.s) != TEUK_OK) {
            rc = fail(c, TEUK_EINVAL, "the parameter moved by %s h leaves the valid range", i == 0 ? "+" : "-");
            break;
        }
        x[i] = own[i].p = new (std::nothrow) teuk_ctx();
        if (!x[i]) {
            rc = fail(c, TEUK_EDEVICE, "host allocation failed");
            break;
        }
        rc = init_ctx(x[i], &gr, pa[i], pM[i], geo.m, geo.s, c->dt, TEUK_FP64, (void*)c->stream);
        if (rc != TEUK_OK) {
            rc = fail(c, TEUK_EDEVICE, "perturbed context: %s", x[i]->err);
            break;
        }
        x[i]->rows = rows;
        if (c->has_src) {
            rc = teuk_set_source_impl(x[i], pr0[i], pamp[i], c->sig_r, c->sig_th);
            if (rc != TEUK_OK) rc = fail(c, rc, "perturbed source: %s", x[i]->err);
        }
    }
    std::vector<double> res;
    const double* lam0 = nullptr;
    if (rc == TEUK_OK)
        rc = param_sweep(c, x[0], x[1], iobs, alpha, (const double*)dL_dwave, n_steps, t_start, (const double*)phi0,
                         (const double*)pi0, C, rows, (char*)workspace, res, &lam0);
    if (rc != TEUK_OK) return rc;
    // sum in step order, then the central difference's 1/(2h)
    double sum = 0.0;
    for (double v : res) sum += v;
    *dL_dparam = sum / (2.0 * h);
    if (dL_dphi0) {
        const int64_t npts = geo.nr * geo.nth;
        HIP_TRY(c, hipMemcpyAsync(dL_dphi0, lam0, npts * 16, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(dL_dpi0, lam0 + 2 * npts, npts * 16, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return TEUK_OK;
}

int teuk_param_gradient(teuk_ctx* c, int32_t param, double h, double rstar_obs, const void* dL_dwave, int64_t n_steps,
                        double t_start, const void* phi0, const void* pi0, int64_t checkpoint_interval,
                        void* workspace, int64_t workspace_bytes, double* dL_dparam, void* dL_dphi0, void* dL_dpi0) {
    try {
        return teuk_param_gradient_impl(c, param, h, rstar_obs, dL_dwave, n_steps, t_start, phi0, pi0,
                                        checkpoint_interval, workspace, workspace_bytes, dL_dparam, dL_dphi0,
                                        dL_dpi0);
    } catch (...) {  // no C++ exception crosses the ABI
        return fail(c, TEUK_EDEVICE, "host allocation failed");
    }
}

int teuk_check_finite(teuk_ctx* c) {
    if (!c) return TEUK_EINVAL;
    if (watch_poll(c) != TEUK_OK) return c->status;
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

int teuk_status(teuk_ctx* c) { return c ? watch_poll(c) : TEUK_EINVAL; }

int teuk_set_watchdog(teuk_ctx* c, int64_t every_steps, double max_abs) {
    if (!c) return TEUK_EINVAL;
    if (every_steps < 0) return fail(c, TEUK_EINVAL, "negative watchdog interval");
    if (std::isnan(max_abs)) return fail(c, TEUK_EINVAL, "watchdog bound is NaN");
    if (c->status != TEUK_OK) return c->status;
    if (every_steps > 0 && !c->d_watch) {
        HIP_TRY(c, hipMalloc((void**)&c->d_watch, sizeof(unsigned long long)));
        void* h = nullptr;
        HIP_TRY(c, hipHostMalloc(&h, sizeof(unsigned long long), hipHostMallocDefault));
        c->h_watch = (volatile unsigned long long*)h;
    }
    if (c->d_watch) {
        // drop earlier findings: no copy into h_watch is in flight after the wait
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        launch_fill_zero((double*)c->d_watch, 1, c->stream);
        HIP_TRY(c, hipGetLastError());
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        *c->h_watch = 0ull;
    }
    c->watch_every = every_steps;
    c->watch_lim = max_abs > 0.0 ? max_abs : HUGE_VAL;
    return TEUK_OK;
}

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

static int teuk_suggest_dt_impl(const teuk_grid* g, double a, double M, int32_t m, int32_t s, int64_t n_steps, double* dt_out) {
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

int teuk_suggest_dt(const teuk_grid* g, double a, double M, int32_t m, int32_t s, int64_t n_steps, double* dt_out) {
    try {
        return teuk_suggest_dt_impl(g, a, M, m, s, n_steps, dt_out);
    } catch (...) {  // no C++ exception crosses the ABI
        return TEUK_EDEVICE;
    }
}

double teuk_rstar_of_r(double r, double a, double M) {
    double rp = M + std::sqrt(M * M - a * a);
    return rstar_of_delta(r - rp, a, M);
}

double teuk_delta_of_rstar(double rstar, double a, double M) { return delta_of_rstar(rstar, a, M); }

}  // extern "C"
