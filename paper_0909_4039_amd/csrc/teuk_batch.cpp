// Batched stepping of many independent m-modes (paper Sec. 2.2: after the
// ansatz of Eq. 4 every azimuthal mode evolves on its own 2+1 grid), one
// persistent launch per step for the whole batch, optionally replayed from a
// captured HIP graph.  See include/teuk.h for the contract of every entry
// point.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "teuk_internal.h"

using namespace teuk;

struct teuk_batch {
    int n = 0;
    hipStream_t stream = nullptr;
    int64_t max_steps = 0;
    std::vector<Geometry> geo;
    std::vector<BatchInst> inst;        // host mirror of the device descriptors
    std::vector<bool> bound;
    std::vector<double> omega;          // fixed-orbit Omega of each instance (0: no source)
    std::vector<bool> has_src;
    std::vector<double*> rs0_mem;       // device r*0 rows of each instance, allocated on first use
    std::vector<void*> allocs;          // device tables and phase rows
    BatchInst* d_inst = nullptr;
    BatchClock* d_clock = nullptr;
    int64_t step = 0, launches = 0;     // host mirror of the device clock
    int rows = 0;                       // 0: per-instance defaults
    int kblock = 2;
    int persistent = 1;                 // launch form (see lw_batch_kernel / lw_batch_grid_kernel)
    int n_tiles[KB_MAX] = {0, 0};
    int cus = 0;
    int per_cu[2 * KB_MAX] = {1, 1, 1, 1};   // [2 (kb - 1) + moving]
    int n_moving = 0;                   // instances with a moving source
    bool dirty = true;                  // descriptors changed since the last upload
    hipGraphExec_t graph = nullptr;
    int graph_launches = 0;             // launches of kblock steps per replay
    // watchdog: every teuk_batch_step ends with a scan of each bound
    // instance; d_watch keeps (instance << 40 | step) + 1 of the first
    // finding and is copied into the pinned word h_watch
    bool watch_on = false;
    double watch_lim = 0;
    unsigned long long* d_watch = nullptr;
    volatile unsigned long long* h_watch = nullptr;
    int status = TEUK_OK;
    char err[512] = {0};
};

namespace {

int bfail(teuk_batch* b, int code, const char* fmt, ...) {
    if (b) {
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(b->err, sizeof(b->err), fmt, ap);
        va_end(ap);
        if (code == TEUK_EDEVICE || code == TEUK_EUNSTABLE) b->status = code;
    }
    return code;
}

#define BHIP(b, expr)                                                                                    \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) return bfail((b), TEUK_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int WATCH_SHIFT = 40;   // steps below 2^40 in a watchdog label

// Turn a watchdog finding that has reached the host into the sticky
// TEUK_EUNSTABLE (no wait).
int watch_poll(teuk_batch* b) {
    if (b->status == TEUK_OK && b->h_watch && *b->h_watch != 0ull) {
        const unsigned long long v = *b->h_watch - 1;
        return bfail(b, TEUK_EUNSTABLE,
                     "watchdog: instance %llu has a value not below %g in magnitude (or not finite) at step %llu",
                     v >> WATCH_SHIFT, b->watch_lim, v & ((1ull << WATCH_SHIFT) - 1));
    }
    return b->status;
}

int dev_copy(teuk_batch* b, void** dst, const void* src, size_t bytes) {
    b->allocs.reserve(b->allocs.size() + 1);  // a failed push_back must not lose the device block
    BHIP(b, hipMalloc(dst, bytes));
    b->allocs.push_back(*dst);
    BHIP(b, hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    return TEUK_OK;
}

// Phase rows of every step the batch may take, with the single-mode step's
// expressions: row k = e^{-i m w(t_k)}, e^{-i m w(t_k + dt/2)}, where w =
// Omega t for a fixed orbit and the table's phi (entries 2k, 2k + 1,
// clamped to the table) for a moving one; rs0 (moving only) gets r*(r0) of
// the same entries.
void fill_phases(const Geometry& g, double omega, double dt, int64_t rows, const double* traj, int64_t n_half,
                 std::vector<double>& ph, std::vector<double>* rs0) {
    ph.assign((size_t)rows * 4, 0.0);
    if (rs0) rs0->assign((size_t)rows * 2, 0.0);
    for (int64_t k = 0; k < rows; ++k) {
        double w0, w1;
        if (traj) {
            const int64_t e = std::min<int64_t>(2 * k, n_half - 2);
            const double* en = &traj[2 * e];
            w0 = g.m * en[1];
            w1 = g.m * en[3];
            (*rs0)[2 * k + 0] = rstar_of_delta(en[0] - g.rp, g.a, g.M);
            (*rs0)[2 * k + 1] = rstar_of_delta(en[2] - g.rp, g.a, g.M);
        } else {
            double t = 0.0 + double(k - 0) * dt;
            w0 = g.m * omega * t;
            w1 = g.m * omega * (t + 0.5 * dt);
        }
        ph[4 * k + 0] = std::cos(w0);
        ph[4 * k + 1] = -std::sin(w0);
        ph[4 * k + 2] = std::cos(w1);
        ph[4 * k + 3] = -std::sin(w1);
    }
}

// Tiles per instance and their prefix for every kb at the current rows.
int layout(teuk_batch* b) {
    for (int kb = 1; kb <= KB_MAX; ++kb) {
        int64_t total = 0;
        for (int i = 0; i < b->n; ++i) {
            const Geometry& g = b->geo[i];
            const int rows = b->inst[i].rows;
            const int64_t so = WAVE - 2 * kb;
            const int64_t ngrp = ((g.nr + so - 1) / so + WG_WAVES - 1) / WG_WAVES;
            const int64_t nchunks = (g.nth + rows - 1) / rows;
            b->inst[i].first_tile[kb - 1] = (int32_t)total;
            total += ngrp * nchunks;
            if (total > INT32_MAX) return bfail(b, TEUK_EINVAL, "batch has more than 2^31 tiles");
        }
        b->n_tiles[kb - 1] = (int)total;
    }
    b->dirty = true;
    return TEUK_OK;
}

void set_rows(teuk_batch* b, int rows) {
    b->rows = rows;
    for (int i = 0; i < b->n; ++i)
        b->inst[i].rows = rows > 0 ? std::min<int>(rows, (int)b->geo[i].nth)
                                   : default_rows((int)b->geo[i].nth, b->kblock, 64);
}

void drop_graph(teuk_batch* b) {
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    b->graph_launches = 0;
}

int upload(teuk_batch* b) {
    if (!b->dirty) return TEUK_OK;
    BHIP(b, hipMemcpyAsync(b->d_inst, b->inst.data(), sizeof(BatchInst) * b->n, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    b->dirty = false;
    return TEUK_OK;
}

int grid_blocks(const teuk_batch* b, int kb) {
    if (!b->persistent) return b->n_tiles[kb - 1];   // one workgroup per tile
    // as many workgroups as stay resident, a multiple of the 8 XCDs
    int resident = std::max(8, (b->cus * b->per_cu[2 * (kb - 1) + (b->n_moving > 0 ? 1 : 0)]) / 8 * 8);
    int need = (b->n_tiles[kb - 1] + 7) / 8 * 8;
    return std::max(8, std::min(resident, need));
}

// One launch of kb steps at (step, launch count) = clock + offsets.
int launch(teuk_batch* b, int kb, bool record, int step_off, int launch_off) {
    BatchArgs a{};
    a.inst = b->d_inst;
    a.clock = b->d_clock;
    a.n_inst = b->n;
    a.n_tiles = b->n_tiles[kb - 1];
    a.kb = kb;
    a.record = record ? 1 : 0;
    a.persistent = b->persistent;
    a.step_off = step_off;
    a.launch_off = launch_off;
    a.moving = b->n_moving > 0 ? 1 : 0;
    launch_batch_step(a, grid_blocks(b, kb), b->stream);
    BHIP(b, hipGetLastError());
    return TEUK_OK;
}

int advance(teuk_batch* b, int steps, int launches) {
    launch_batch_advance(b->d_clock, steps, launches, b->stream);
    BHIP(b, hipGetLastError());
    return TEUK_OK;
}

int ready(teuk_batch* b) {
    if (b->status != TEUK_OK) return b->status;
    for (int i = 0; i < b->n; ++i)
        if (!b->bound[i]) return bfail(b, TEUK_ESTATE, "instance %d has no state bound", i);
    return upload(b);
}

}  // namespace

extern "C" {

static int init_batch(teuk_batch* b, int32_t n, const teuk_desc* d, int64_t max_steps, void* hip_stream) {
    b->n = n;
    b->stream = (hipStream_t)hip_stream;
    b->max_steps = max_steps;
    b->geo.resize(n);
    b->inst.resize(n);
    b->bound.assign(n, false);
    b->omega.assign(n, 0.0);
    b->has_src.assign(n, false);
    b->rs0_mem.assign(n, nullptr);
    int rc = TEUK_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return TEUK_EDEVICE;
    for (int kb = 1; kb <= KB_MAX; ++kb)
        for (int mv = 0; mv < 2; ++mv) b->per_cu[2 * (kb - 1) + mv] = batch_blocks_per_cu(kb, mv != 0);
    for (int i = 0; i < n && rc == TEUK_OK; ++i) {
        const teuk_desc& e = d[i];
        Geometry& g = b->geo[i];
        g.nr = e.grid.n_rstar;
        g.nth = e.grid.n_theta;
        g.rmin = e.grid.rstar_min;
        g.rmax = e.grid.rstar_max;
        g.a = e.a;
        g.M = e.M;
        g.m = e.m;
        g.s = e.s;
        build_geometry(g);
        int iobs;
        double alpha;
        if (!observer_index(g, e.rstar_obs, iobs, alpha)) {
            rc = TEUK_EINVAL;
            break;
        }
        // the source as teuk_set_source builds it
        double omega = 0.0;
        if (e.r0 != 0.0) {
            const double sr = e.sigma_r_cells > 0.0 ? e.sigma_r_cells : 2.0;
            const double sth = e.sigma_th_cells > 0.0 ? e.sigma_th_cells : 2.0;
            if (!(e.r0 > g.rp)) {
                rc = TEUK_EINVAL;
                break;
            }
            omega = orbit_omega(e.r0, g.a, g.M);
            build_source(g, rstar_of_delta(e.r0 - g.rp, g.a, g.M), sr * g.dr, sth * g.dth, e.amp);
        }
        b->omega[i] = omega;
        b->has_src[i] = e.r0 != 0.0;
        std::vector<double> ph;
        fill_phases(g, omega, e.dt, max_steps + KB_MAX, nullptr, 0, ph, nullptr);
        BatchInst& I = b->inst[i];
        std::memset(&I, 0, sizeof(I));
        void *ri = nullptr, *rh = nullptr, *an = nullptr, *pp = nullptr;
        if ((rc = dev_copy(b, &ri, g.rad_i.data(), g.rad_i.size() * 8)) != TEUK_OK) break;
        if ((rc = dev_copy(b, &rh, g.rad_h.data(), g.rad_h.size() * 8)) != TEUK_OK) break;
        if ((rc = dev_copy(b, &an, g.ang.data(), g.ang.size() * 8)) != TEUK_OK) break;
        if ((rc = dev_copy(b, &pp, ph.data(), ph.size() * 8)) != TEUK_OK) break;
        I.rad_i = (const double*)ri;
        I.rad_h = (const double*)rh;
        I.ang = (const double*)an;
        I.phase = (const double*)pp;
        I.stride = g.stride;
        I.nr = (int)g.nr;
        I.nth = (int)g.nth;
        I.iobs = iobs;
        I.alpha = alpha;
        I.dt = e.dt;
        I.hdt = 0.5 * e.dt;
        I.inv_dr = 1.0 / g.dr;
        I.m2ma = -2.0 * g.m * g.a;
        const double sr = (e.sigma_r_cells > 0.0 ? e.sigma_r_cells : 2.0) * g.dr;
        I.rs0tab = nullptr;
        I.two_sr2 = 2.0 * sr * sr;
        I.rmin = g.rmin;
        I.dr = g.dr;
    }
    if (rc == TEUK_OK) {
        set_rows(b, 0);
        rc = layout(b);
    }
    if (rc == TEUK_OK &&
        (hipMalloc((void**)&b->d_inst, sizeof(BatchInst) * n) != hipSuccess ||
         hipMalloc((void**)&b->d_clock, sizeof(BatchClock)) != hipSuccess))
        rc = TEUK_EDEVICE;
    if (rc == TEUK_OK) {
        BatchClock z{0, 0};
        if (hipMemcpy(b->d_clock, &z, sizeof(z), hipMemcpyHostToDevice) != hipSuccess) rc = TEUK_EDEVICE;
    }
    return rc;
}

int teuk_batch_create(int32_t n, const teuk_desc* d, int64_t max_steps, void* hip_stream, teuk_batch** out) {
    if (!out) return TEUK_EINVAL;
    *out = nullptr;
    if (n < 1 || n > 65535 || !d || max_steps < 1 || max_steps > ((int64_t)1 << 40)) return TEUK_EINVAL;
    for (int i = 0; i < n; ++i) {
        const teuk_desc& e = d[i];
        if (validate_phys(&e.grid, e.a, e.M, e.s) != TEUK_OK) return TEUK_EINVAL;
        if (!(e.dt > 0.0) || !std::isfinite(e.dt) || e.m < -1000 || e.m > 1000) return TEUK_EINVAL;
        if (!std::isfinite(e.r0) || !std::isfinite(e.amp) || !std::isfinite(e.rstar_obs)) return TEUK_EINVAL;
    }
    teuk_batch* b = new (std::nothrow) teuk_batch();
    if (!b) return TEUK_EDEVICE;
    int rc;
    try {
        rc = init_batch(b, n, d, max_steps, hip_stream);
    } catch (...) {  // host allocation failed; no C++ exception crosses the ABI
        rc = TEUK_EDEVICE;
    }
    if (rc != TEUK_OK) {
        teuk_batch_destroy(b);
        return rc;
    }
    *out = b;
    return TEUK_OK;
}

int teuk_batch_destroy(teuk_batch* b) {
    if (!b) return TEUK_EINVAL;
    (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    for (void* p : b->allocs) (void)hipFree(p);
    if (b->d_inst) (void)hipFree(b->d_inst);
    if (b->d_clock) (void)hipFree(b->d_clock);
    if (b->d_watch) (void)hipFree(b->d_watch);
    if (b->h_watch) (void)hipHostFree((void*)b->h_watch);
    delete b;
    return TEUK_OK;
}

int teuk_batch_bind(teuk_batch* b, int32_t i, void* phi, void* pi, void* phi_next, void* pi_next, void* wave,
                    int64_t wave_rows) {
    if (!b) return TEUK_EINVAL;
    if (i < 0 || i >= b->n) return bfail(b, TEUK_EINVAL, "instance %d out of range", i);
    void* p[4] = {phi, pi, phi_next, pi_next};
    for (int k = 0; k < 4; ++k) {
        if (!p[k] || (uintptr_t)p[k] % 16 != 0) return bfail(b, TEUK_EINVAL, "state pointer %d NULL or misaligned", k);
        for (int q = 0; q < k; ++q)
            if (p[q] == p[k]) return bfail(b, TEUK_EINVAL, "state pointers %d and %d alias", q, k);
    }
    if (wave && ((uintptr_t)wave % 16 != 0 || wave_rows < 0))
        return bfail(b, TEUK_EINVAL, "wave buffer misaligned or negative capacity");
    // the pair that holds the current state follows the launch parity
    const int cur = (int)(b->launches & 1);
    BatchInst& I = b->inst[i];
    I.buf[cur][0] = (double*)phi;
    I.buf[cur][1] = (double*)pi;
    I.buf[1 - cur][0] = (double*)phi_next;
    I.buf[1 - cur][1] = (double*)pi_next;
    I.wave = (double*)wave;
    I.wave_cap = wave ? wave_rows : 0;
    b->bound[i] = true;
    b->dirty = true;
    return TEUK_OK;
}

int teuk_batch_step(teuk_batch* b, int64_t n) {
    if (!b) return TEUK_EINVAL;
    if (watch_poll(b) != TEUK_OK) return b->status;
    if (n < 0) return bfail(b, TEUK_EINVAL, "negative step count");
    int rc = ready(b);
    if (rc != TEUK_OK) return rc;
    if (b->step + n > b->max_steps)
        return bfail(b, TEUK_EINVAL, "step %lld + %lld exceeds max_steps %lld", (long long)b->step, (long long)n,
                     (long long)b->max_steps);
    int64_t done = 0;
    if (b->graph) {
        const int64_t per = (int64_t)b->graph_launches * b->kblock;
        for (; n - done >= per; done += per) {
            BHIP(b, hipGraphLaunch(b->graph, b->stream));
            b->launches += b->graph_launches;
        }
    }
    // the rest by direct launches at offsets from the clock, then one advance
    // (in chunks, so that the offsets stay small)
    while (done < n) {
        int soff = 0, loff = 0;
        while (done < n && soff < (1 << 20)) {
            const int kb = (b->kblock >= 2 && n - done >= 2) ? 2 : 1;
            if ((rc = launch(b, kb, true, soff, loff)) != TEUK_OK) return rc;
            soff += kb;
            loff += 1;
            done += kb;
        }
        if ((rc = advance(b, soff, loff)) != TEUK_OK) return rc;
        b->launches += loff;
    }
    b->step += n;
    int max_nth = 0;
    for (const Geometry& g : b->geo) max_nth = std::max<int>(max_nth, (int)g.nth);
    launch_batch_extract(b->d_inst, b->n, max_nth, b->d_clock, b->stream);
    BHIP(b, hipGetLastError());
    if (b->watch_on && n > 0) {
        const int cur = (int)(b->launches & 1);
        for (int i = 0; i < b->n; ++i) {
            const int64_t npts = 2 * b->geo[i].nr * b->geo[i].nth;
            const int64_t tag = ((int64_t)i << WATCH_SHIFT) | (b->step & ((1ll << WATCH_SHIFT) - 1));
            for (int f = 0; f < 2; ++f) {
                launch_watch_fp64(b->inst[i].buf[cur][f], npts, b->watch_lim, tag, b->d_watch, b->stream);
                BHIP(b, hipGetLastError());
            }
        }
        BHIP(b, hipMemcpyAsync((void*)b->h_watch, b->d_watch, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                               b->stream));
    }
    return TEUK_OK;
}

int teuk_batch_set_watchdog(teuk_batch* b, int32_t on, double max_abs) {
    if (!b) return TEUK_EINVAL;
    if (std::isnan(max_abs)) return bfail(b, TEUK_EINVAL, "watchdog bound is NaN");
    if (b->status != TEUK_OK) return b->status;
    if (on && !b->d_watch) {
        BHIP(b, hipMalloc((void**)&b->d_watch, sizeof(unsigned long long)));
        void* h = nullptr;
        BHIP(b, hipHostMalloc(&h, sizeof(unsigned long long), hipHostMallocDefault));
        b->h_watch = (volatile unsigned long long*)h;
    }
    if (b->d_watch) {
        BHIP(b, hipStreamSynchronize(b->stream));
        launch_fill_zero((double*)b->d_watch, 1, b->stream);
        BHIP(b, hipGetLastError());
        BHIP(b, hipStreamSynchronize(b->stream));
        *b->h_watch = 0ull;
    }
    b->watch_on = on != 0;
    b->watch_lim = max_abs > 0.0 ? max_abs : HUGE_VAL;
    return TEUK_OK;
}

int teuk_batch_capture_graph(teuk_batch* b, int64_t steps_per_graph) {
    if (!b) return TEUK_EINVAL;
    drop_graph(b);
    if (steps_per_graph == 0) return TEUK_OK;
    if (steps_per_graph < 0 || steps_per_graph % b->kblock != 0 || steps_per_graph / b->kblock > 100000)
        return bfail(b, TEUK_EINVAL, "steps_per_graph must be a positive multiple of %d (at most 100000 launches)",
                     b->kblock);
    if (!b->stream) return bfail(b, TEUK_EINVAL, "graph capture needs a non-null stream");
    int rc = ready(b);
    if (rc != TEUK_OK) return rc;
    const int L = (int)(steps_per_graph / b->kblock);
    BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < L && rc == TEUK_OK; ++k) rc = launch(b, b->kblock, true, k * b->kblock, k);
    if (rc == TEUK_OK) rc = advance(b, L * b->kblock, L);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc != TEUK_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc != TEUK_OK ? rc : bfail(b, TEUK_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->graph = nullptr;
        return bfail(b, TEUK_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    b->graph_launches = L;
    return TEUK_OK;
}

int teuk_batch_set_tiling(teuk_batch* b, int32_t rows_per_wave, int32_t steps_per_launch, int32_t persistent) {
    if (!b) return TEUK_EINVAL;
    if (rows_per_wave < 0 || rows_per_wave > 4096) return bfail(b, TEUK_EINVAL, "rows_per_wave out of range");
    if (steps_per_launch < 1 || steps_per_launch > KB_MAX)
        return bfail(b, TEUK_EINVAL, "steps_per_launch must be 1..%d", KB_MAX);
    if (persistent < 0 || persistent > 1) return bfail(b, TEUK_EINVAL, "persistent must be 0 or 1");
    drop_graph(b);
    b->kblock = steps_per_launch;
    b->persistent = persistent;
    set_rows(b, rows_per_wave);
    return layout(b);
}

int teuk_batch_autotune(teuk_batch* b, int32_t launches_per_trial, int32_t* rows_out, int32_t* kb_out,
                        int32_t* persistent_out) {
    if (!b) return TEUK_EINVAL;
    if (launches_per_trial < 1 || launches_per_trial > 10000)
        return bfail(b, TEUK_EINVAL, "launches_per_trial must be 1..10000");
    int rc = ready(b);
    if (rc != TEUK_OK) return rc;
    static const int kRows[] = {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256};
    hipEvent_t e0, e1;
    BHIP(b, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return bfail(b, TEUK_EDEVICE, "hipEventCreate failed");
    }
    double best = 0.0;
    int best_rows = b->rows, best_kb = b->kblock, best_form = b->persistent;
    for (int cand = 0; cand < 2 * KB_MAX && rc == TEUK_OK; ++cand) {
        const int kb = 1 + cand % KB_MAX, form = cand / KB_MAX;
        for (int r : kRows) {
            drop_graph(b);
            b->kblock = kb;
            b->persistent = form;
            set_rows(b, r);
            if ((rc = layout(b)) != TEUK_OK || (rc = upload(b)) != TEUK_OK) break;
            // trial launches read the current pair and write the other one;
            // the clock does not move and the recorder is off
            if ((rc = launch(b, kb, false, 0, 0)) != TEUK_OK) break;
            if (hipEventRecord(e0, b->stream) != hipSuccess) { rc = bfail(b, TEUK_EDEVICE, "event record"); break; }
            for (int k = 0; k < launches_per_trial && rc == TEUK_OK; ++k) rc = launch(b, kb, false, 0, 0);
            if (rc != TEUK_OK) break;
            float ms = 0.0f;
            if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = bfail(b, TEUK_EDEVICE, "event timing");
                break;
            }
            const double sec = 1e-3 * ms / double(launches_per_trial * kb);
            if (best == 0.0 || sec < best) {
                best = sec;
                best_rows = r;
                best_kb = kb;
                best_form = form;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != TEUK_OK) return rc;
    b->kblock = best_kb;
    b->persistent = best_form;
    set_rows(b, best_rows);
    if ((rc = layout(b)) != TEUK_OK) return rc;
    if (rows_out) *rows_out = best_rows;
    if (kb_out) *kb_out = best_kb;
    if (persistent_out) *persistent_out = best_form;
    return TEUK_OK;
}

static int teuk_batch_set_trajectory_impl(teuk_batch* b, int32_t i, const double* r0_phase, int64_t n_half) {
    if (!b) return TEUK_EINVAL;
    if (b->status != TEUK_OK) return b->status;
    if (i < 0 || i >= b->n) return bfail(b, TEUK_EINVAL, "instance %d out of range", i);
    const Geometry& g = b->geo[i];
    BatchInst& I = b->inst[i];
    const int64_t rows = b->max_steps + KB_MAX;
    if (r0_phase) {
        if (!b->has_src[i]) return bfail(b, TEUK_ESTATE, "instance %d has no source (r0 = 0 in its descriptor)", i);
        if (n_half < 2 * b->max_steps || n_half > ((int64_t)1 << 34))
            return bfail(b, TEUK_EINVAL, "the table needs 2 max_steps = %lld entries, it has %lld",
                         (long long)(2 * b->max_steps), (long long)n_half);
        for (int64_t k = 0; k < n_half; ++k)
            if (!(r0_phase[2 * k] > g.rp) || !std::isfinite(r0_phase[2 * k]) || !std::isfinite(r0_phase[2 * k + 1]))
                return bfail(b, TEUK_EINVAL, "orbit entry %lld: r0 must exceed r+ and both values be finite",
                             (long long)k);
    } else if (!I.rs0tab) {
        return TEUK_OK;   // already a fixed orbit
    }
    std::vector<double> ph, rs0;
    fill_phases(g, b->omega[i], I.dt, rows, r0_phase, n_half, ph, r0_phase ? &rs0 : nullptr);
    const bool was_moving = I.rs0tab != nullptr;
    // no launch may be reading the rows being replaced, and the copies are
    // ordered on the batch's stream (which need not synchronise with the
    // null stream); the stream is synchronised again before the host
    // vectors go away, on the error paths too
    BHIP(b, hipStreamSynchronize(b->stream));
    if (r0_phase && !b->rs0_mem[i]) {
        b->allocs.reserve(b->allocs.size() + 1);   // a failed push_back must not lose the block
        void* p = nullptr;
        BHIP(b, hipMalloc(&p, rs0.size() * sizeof(double)));
        b->allocs.push_back(p);
        b->rs0_mem[i] = (double*)p;
    }
    hipError_t e = hipMemcpyAsync((void*)I.phase, ph.data(), ph.size() * sizeof(double), hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess && r0_phase)
        e = hipMemcpyAsync(b->rs0_mem[i], rs0.data(), rs0.size() * sizeof(double), hipMemcpyHostToDevice,
                           b->stream);
    const hipError_t es = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return bfail(b, TEUK_EDEVICE, "orbit table upload: %s", hipGetErrorString(e));
    I.rs0tab = r0_phase ? b->rs0_mem[i] : nullptr;   // cleared rows stay allocated for a later table
    const int before = b->n_moving;
    b->n_moving += (I.rs0tab != nullptr ? 1 : 0) - (was_moving ? 1 : 0);
    if ((before > 0) != (b->n_moving > 0)) drop_graph(b);   // a captured graph holds the other kernel build
    b->dirty = true;
    return TEUK_OK;
}

int teuk_batch_set_trajectory(teuk_batch* b, int32_t i, const double* r0_phase, int64_t n_half) {
    try {
        return teuk_batch_set_trajectory_impl(b, i, r0_phase, n_half);
    } catch (...) {  // no C++ exception crosses the ABI
        return bfail(b, TEUK_EDEVICE, "host allocation failed");
    }
}

int teuk_batch_current(teuk_batch* b) { return b ? (int)(b->launches & 1) : TEUK_EINVAL; }

int teuk_batch_get_step(teuk_batch* b, int64_t* step) {
    if (!b || !step) return TEUK_EINVAL;
    *step = b->step;
    return TEUK_OK;
}

int teuk_batch_status(teuk_batch* b) { return b ? watch_poll(b) : TEUK_EINVAL; }

const char* teuk_batch_last_error(teuk_batch* b) { return b ? b->err : "null batch"; }

}  // extern "C"
