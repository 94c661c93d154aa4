/*
 * teuk.h -- C ABI of libteuk, an MI355X (gfx950) library that evolves one
 * azimuthal mode of the Teukolsky equation on an (r*, theta) grid with the
 * two-step Lax-Wendroff scheme.
 *
 * Paper: G. Khanna and J. McKennon, "An exploration of CUDA and CBEA for a
 * gravitational wave source-modelling application".  The problem statement
 * is Sec. 2: Eq. (1) (Teukolsky master equation, spin weight s, Kerr
 * parameter a, mass M, source T), the tortoise/azimuthal coordinates of
 * Eqs. (2)-(3), the m-mode ansatz Eq. (4), the first-order system
 * Eqs. (5)-(12) for u = (Phi, Pi), the Lax-Wendroff predictor/corrector
 * Eqs. (13)-(14), centred angular differences and the boundary conditions
 * stated after Eq. (14), and the waveform read at an extraction radius
 * (Sec. 2.2, Fig. 1).
 *
 * Conventions shared by every call:
 *   - Fields are complex and stored as interleaved (re, im) pairs, row-major
 *     [n_theta][n_rstar] with r* contiguous: complex128 for TEUK_FP64,
 *     complex64 for TEUK_FP32 (torch.complex128 / torch.complex64 layout).
 *   - Grid: r*_i = rstar_min + i dr*, dr* = (rstar_max - rstar_min)/(n_rstar - 1);
 *     theta_j = (j + 1/2) pi / n_theta (cell-centred, poles excluded).
 *   - Every pointer named "device" must point to device memory of the GPU
 *     that was current at teuk_create; it stays owned by the caller.  The
 *     library's own device memory is small and lives with the context:
 *     its coefficient tables (about 200 B per r* node and 64 B per theta
 *     row) from teuk_create to teuk_destroy; a batch's tables and phase
 *     rows from teuk_batch_create to teuk_batch_destroy; and, for the
 *     duration of one call, the trial slots of teuk_adjoint_autotune and
 *     the two parameter-moved tables of teuk_param_gradient; and, once a
 *     watchdog is set, 8 B of device and 8 B of pinned host memory per
 *     context or batch.  States, waveforms and workspaces are the caller's.
 *   - Calls are asynchronous on the stream given at create unless noted.
 *   - Return value: TEUK_OK (0) or a negative TEUK_E* code.  No C++
 *     exception crosses the ABI.  A context is not thread safe; use one
 *     context per stream.
 */
#ifndef TEUK_H
#define TEUK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TEUK_OK 0
#define TEUK_EINVAL (-1)    /* an argument is out of range                     */
#define TEUK_ESTATE (-2)    /* call out of order (e.g. no state bound)         */
#define TEUK_EDEVICE (-3)   /* a HIP call or a host allocation failed; teuk_last_error has the text.
                               No C++ exception leaves any entry point. */
#define TEUK_EUNSTABLE (-4) /* non-finite values found in the state            */
#define TEUK_ENOTSUP (-5)   /* valid request the library does not serve        */

#define TEUK_FP64 64
#define TEUK_FP32 32
#define TEUK_FP32S 48   /* FP32 storage (complex64 state and waveform), FP64 arithmetic and tables */

typedef struct teuk_ctx teuk_ctx;

typedef struct {
    int64_t n_rstar;   /* r* nodes, >= 4                */
    int64_t n_theta;   /* theta cells, >= 4             */
    double rstar_min;  /* first r* node                 */
    double rstar_max;  /* last r* node, > rstar_min     */
} teuk_grid;

/* Create a solver for one (a, M, m, s) mode (Eq. 1, ansatz Eq. 4) with time
 * step dt on grid g.  prec is TEUK_FP64 or TEUK_FP32 (storage and
 * arithmetic), or TEUK_FP32S: FP32 storage of the state and the waveform
 * (complex64, as TEUK_FP32) with each step computed in FP64 from FP64 tables
 * (the FP32 bytes per point, FP64 rounding inside a step; no reverse sweep).
 * hip_stream is a hipStream_t (NULL: the null stream).
 * Requires M > 0, 0 <= a < M, |s| <= 2, dt > 0.  Builds the radial tables
 * (r(r*) from Eq. 2 solved in ln(r - r+)) on the host in FP64 and uploads
 * them.  On success *out receives the context; on failure *out is NULL. */
int teuk_create(const teuk_grid* g, double a, double M, int32_t m, int32_t s, double dt,
                int32_t prec, void* hip_stream, teuk_ctx** out);

/* Release the context and its tables (synchronises its stream first). */
int teuk_destroy(teuk_ctx* ctx);

/* Bind caller-owned device state: phi, pi hold u^n; phi_next, pi_next are
 * the ping-pong partners.  All four must be distinct, n_theta*n_rstar
 * complex elements each.  teuk_step alternates between the two pairs;
 * teuk_current tells which pair holds the latest state.  Binding resets
 * the current pair to (phi, pi). */
int teuk_bind_state(teuk_ctx* ctx, void* phi, void* pi, void* phi_next, void* pi_next);

/* Particle source (stand-in for the paper's T, which it does not print):
 * T_Pi = amp exp(-(r*-r*(r0))^2/(2 sr^2)) exp(-(theta-pi/2)^2/(2 sth^2)) e^{-i m Omega t},
 * T_Phi = 0, with sr = sigma_r_cells dr*, sth = sigma_th_cells dtheta and
 * Omega = sqrt(M)/(r0^{3/2} + a sqrt(M)) (circular equatorial orbit).
 * Requires r0 > r+ and positive widths; amp = 0 switches the source off. */
int teuk_set_source(teuk_ctx* ctx, double r0, double amp, double sigma_r_cells,
                    double sigma_th_cells);

/* Moving source (an inspiralling particle, as in the waveform of the paper's
 * Fig. 1): from the current step on, the source of teuk_set_source (its
 * amplitude and widths) follows the orbit r0_phase, a host array of n_half
 * pairs (r0, phi) giving the orbit radius and phase at t_now + k dt/2,
 * k = 0 .. n_half - 1 (copied).  Step s after this call uses entry 2s at
 * t^n (predictor: centre r*(r0), phase e^{-i m phi}) and entry 2s + 1 at
 * t^n + dt/2 (corrector); teuk_step fails with TEUK_EINVAL past the table.
 * With r0 fixed and phi = Omega t it is the fixed-orbit source up to
 * rounding.  r0_phase = NULL returns to the fixed orbit.  Requires
 * teuk_set_source first (TEUK_ESTATE) and r0 > r+ in every entry.
 * teuk_set_time relabels steps without moving the table; to run again from
 * the table's first entry, set it again.  Its reverse sweep is
 * teuk_adjoint_moving. */
int teuk_set_trajectory(teuk_ctx* ctx, const double* r0_phase, int64_t n_half);

/* Waveform recorder: from now on each step records
 * w_j = (1 - alpha) Phi_{i0,j} + alpha Phi_{i0+1,j}, r*_obs = r*_{i0} + alpha dr*,
 * into wave[k][n_theta] (device, complex, caller-owned) where k counts
 * steps from the current step (row 0 = current state).  Rows at or past
 * capacity_rows are not written.  rstar_obs must lie strictly inside the
 * grid.  wave = NULL switches recording off. */
int teuk_set_observer(teuk_ctx* ctx, double rstar_obs, void* wave, int64_t capacity_rows);

/* Advance n >= 0 steps of Eqs. (13)-(14) with the source fused and the
 * boundary conditions applied; records rows 0..n (relative to the step
 * count at entry) when an observer is set. */
int teuk_step(teuk_ctx* ctx, int64_t n);

/* Write the waveform of the current state at rstar_obs into out
 * (device, n_theta complex). */
int teuk_extract(teuk_ctx* ctx, double rstar_obs, void* out);

/* Host-side time bookkeeping: t = t0 + (step - step0) dt.  teuk_set_time
 * relabels the current step; the observer's rows and the orbit table of
 * teuk_set_trajectory stay attached to the same steps. */
int teuk_get_time(teuk_ctx* ctx, double* t, int64_t* step);
int teuk_set_time(teuk_ctx* ctx, double t, int64_t step);

/* The clock behind those times: the base (t0 at step step0) and the
 * current step.  teuk_set_time(t, step) is teuk_set_clock(t, step, step);
 * it rebases the clock, so the times of the steps after it round
 * differently from those of a run that kept its base.  A run resumed with
 * another run's three clock values forms the same step times (and so the
 * same source phases) bit for bit.  Any output pointer may be NULL;
 * teuk_set_clock moves the observer's rows and the orbit table as
 * teuk_set_time does, and fails with TEUK_EINVAL for a non-finite t0. */
int teuk_get_clock(teuk_ctx* ctx, double* t0, int64_t* step0, int64_t* step);
int teuk_set_clock(teuk_ctx* ctx, double t0, int64_t step0, int64_t step);

/* 0: the latest state is in (phi, pi); 1: in (phi_next, pi_next);
 * negative: error code. */
int teuk_current(teuk_ctx* ctx);

/* Tile shape of the step kernel (performance only; results are bitwise
 * identical for every choice): rows_per_wave theta rows per wavefront
 * (1..4096; 0 restores the default and ignores order) and the launch form:
 * 0: one wavefront runs both fused steps of a tile, tiles theta-chunk-major;
 * 1: the same, r*-strip-group-major; 2: two fused steps on a pair of
 * wavefronts, one step each, handing rows over through LDS (single steps
 * launch as for 0). */
int teuk_set_tiling(teuk_ctx* ctx, int32_t rows_per_wave, int32_t order);
int teuk_get_tiling(teuk_ctx* ctx, int32_t* rows_per_wave, int32_t* order);

/* Temporal blocking: fuse steps_per_launch (1 or 2; default 2) Lax-Wendroff
 * steps in one kernel launch, keeping the intermediate state on chip
 * (performance only: results are bitwise identical to single steps; an odd
 * remainder of teuk_step(n) runs as a single step).  teuk_get_blocking
 * returns the current setting or a negative error code. */
int teuk_set_blocking(teuk_ctx* ctx, int32_t steps_per_launch);
int teuk_get_blocking(teuk_ctx* ctx);

/* Reverse sweep (FP64 contexts only).  The time step of Eqs. (13)-(14) is
 * affine in u = (Phi, Pi), u^{k+1} = K u^k + s^k, with K independent of u
 * and k; s^k carries the source T at t^k and t^k + dt/2.  For a real loss
 * L of the waveform w^k = E u^k (k = 0..n_steps) recorded at rstar_obs
 * (linear interpolation in r*, as teuk_set_observer) from initial data
 * u^0 at time t_start, this returns the gradients of L with respect to the
 * initial data and the source parameters of teuk_set_source:
 *   lambda^n = E^H g^n,  lambda^k = K^H lambda^{k+1} + E^H g^k,
 *   dL/du^0 = lambda^0,  dL/dp = sum_k Re <a_T^k, dT^k/dp>,
 * with a_T^k the adjoints of the source values of step k.  K^H needs no
 * forward state, so no forward steps are stored or recomputed.
 *
 * Complex gradients use the real-view convention g = dL/dRe + i dL/dIm
 * (the convention of torch's complex autograd: for L = |z|^2, g = 2z).
 *   dL_dwave: device, (n_steps + 1) x n_theta complex128, row k = g^k (read).
 *   workspace: device, >= teuk_adjoint_workspace_bytes bytes, 256-byte
 *     aligned, caller-owned; contents are scratch.
 *   dL_dphi0, dL_dpi0: device, n_theta x n_rstar complex128 (written).
 *   dL_dr0, dL_damp: host, may be NULL; both 0 if no source was set.
 * Uses the context's dt, source and reverse-sweep tiling
 * (teuk_set_adjoint_tiling), and neither reads nor changes the bound state
 * or the time.  The workspace size does not depend on the tiling.
 * Synchronous (returns after the sweep).  TEUK_ENOTSUP for FP32 contexts and while an orbit
 * table is set (its sweep is teuk_adjoint_moving); TEUK_EINVAL for
 * misaligned, overlapping or short buffers or rstar_obs outside the grid. */
int64_t teuk_adjoint_workspace_bytes(teuk_ctx* ctx);
int teuk_adjoint(teuk_ctx* ctx, double rstar_obs, const void* dL_dwave, int64_t n_steps, double t_start,
                 void* workspace, int64_t workspace_bytes, void* dL_dphi0, void* dL_dpi0, double* dL_dr0,
                 double* dL_damp);

/* The reverse sweep of teuk_adjoint without a workspace argument, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  It calls no
 * hipMalloc, hipFree or other allocating routine: its workspace is a
 * file-scope device array of teuk_adjoint_noalloc_max_bytes() bytes
 * (40 MiB, enough for a 4096 x 256 grid), which every GPU that runs this
 * call holds until the process ends.  Arguments, results and errors are
 * those of teuk_adjoint, plus TEUK_EINVAL when teuk_adjoint_workspace_bytes
 * exceeds the array.  All calls on one GPU share its array: calls that
 * overlap on one GPU (other streams or threads) race and must be
 * serialised by the caller.  Synchronous, as teuk_adjoint. */
int64_t teuk_adjoint_noalloc_max_bytes(void);
int teuk_adjoint_noalloc(teuk_ctx* ctx, double rstar_obs, const void* dL_dwave, int64_t n_steps, double t_start,
                         void* dL_dphi0, void* dL_dpi0, double* dL_dr0, double* dL_damp);

/* Reverse sweep for a moving source (FP64; the orbit table of
 * teuk_set_trajectory).  As teuk_adjoint, for a forward run of n_steps
 * steps from initial data u^0 that started at the table's first entry, so
 * that step k used entry 2k (predictor, t^k) and entry 2k + 1 (corrector,
 * t^k + dt/2).  With T = amp U, U = exp(-(r* - r*(r0_e))^2 / 2 sr^2)
 * G_theta e^{-i m phi_e} the unit-amplitude source of entry e (the moving
 * source that stands in for the paper's T on a decaying orbit, Fig. 1):
 *   dL/dr0_e  = Re sum conj(a_T) amp U (r* - r*(r0_e)) / sr^2 (d r* / d r)(r0_e),
 *   dL/dphi_e = Re sum conj(a_T) (-i m) amp U,
 *   dL/damp   = Re sum over all entries and points of conj(a_T) U,
 * with d r* / d r = (r^2 + a^2)/Delta (Eq. 2).  The partial sums of every
 * launch are reduced in a fixed order, so results repeat bit for bit.
 *   dL_dtraj: host, 2 n_steps x 2 doubles (written): row e = (dL/dr0_e,
 *     dL/dphi_e); entries from 2 n_steps on are not read by the run and
 *     have zero gradient.
 *   dL_damp: host, may be NULL.
 * Other arguments as teuk_adjoint (no t_start: the table fixes the phases).
 * The workspace size (teuk_adjoint_workspace_bytes) grows with the table,
 * so query it after teuk_set_trajectory.  TEUK_ESTATE without a table;
 * TEUK_EINVAL if 2 n_steps exceeds the table length or for bad buffers;
 * TEUK_ENOTSUP for FP32 contexts. */
int teuk_adjoint_moving(teuk_ctx* ctx, double rstar_obs, const void* dL_dwave, int64_t n_steps, void* workspace,
                        int64_t workspace_bytes, void* dL_dphi0, void* dL_dpi0, double* dL_dtraj, double* dL_damp);

/* Gradient of a real loss of the waveform with respect to one parameter
 * of the problem, with checkpointing (FP64, fixed orbit).  The parameter
 * is the Kerr spin a (TEUK_PARAM_A), the mass M (TEUK_PARAM_M), the orbit
 * radius r0 (TEUK_PARAM_R0) or the source amplitude (TEUK_PARAM_AMP).  a
 * and M enter the operator K of Eqs. (13)-(14) through every coefficient,
 * so unlike teuk_adjoint this needs the forward states:
 *   dL/dp = sum_k Re <lambda^{k+1}, d step(u^k) / dp>,
 * where lambda^{k+1} is the adjoint of u^{k+1} and the derivative of one
 * step at fixed u^k is the central difference
 *   [step_{p+h}(u^k) - step_{p-h}(u^k)] / (2h)
 * of steps under the perturbed parameter (tables, source and Omega built
 * for p +- h; error O(h^2), plus rounding of order eps/h).  The forward run
 * from (phi0, pi0) at t_start keeps every C-th state (checkpoint_interval
 * C; 0 picks ceil(sqrt(n_steps))); the reverse sweep recomputes each
 * segment of C states from its checkpoint, and one launch per reverse step
 * evaluates both perturbed steps on the same u^k and contracts their
 * difference with lambda^{k+1} without storing either.  So memory is
 * ceil(n/C) + C + 1 states (plus the contraction's per-tile parts for the
 * C steps of a segment, summed once per segment), and the cost is about
 * five forward runs.  The forward run takes the context's own launches;
 * the sweep's one-step launches take their own theta rows per wave (1 to
 * 16, from the grid, the device's compute units and the workgroups they
 * hold resident), so the context's tiling changes no bit of the result.
 * Contractions and their sum follow fixed orders (results repeat bit for
 * bit on a device).
 * teuk_param_gradient_workspace_bytes returns TEUK_EINVAL for negative
 * arguments and TEUK_EDEVICE if the device cannot be queried.
 *   dL_dwave: device, (n_steps + 1) x n_theta complex128, as teuk_adjoint.
 *   phi0, pi0: device, n_theta x n_rstar complex128, the initial data (read).
 *   workspace: device, teuk_param_gradient_workspace_bytes(ctx, n_steps, C)
 *     bytes, 256-byte aligned.
 *   dL_dparam: host (written).
 *   dL_dphi0, dL_dpi0: device, may both be NULL; else they receive
 *     lambda^0, as from teuk_adjoint.
 * The context's bound state, time and observer are not touched.
 * TEUK_EINVAL for an unknown parameter, h <= 0, a perturbed value outside
 * the valid range (|a| >= M, r0 <= r+), or bad buffers; TEUK_ESTATE for
 * TEUK_PARAM_R0 or TEUK_PARAM_AMP without a source; TEUK_ENOTSUP for FP32
 * contexts or with an orbit table set. */
#define TEUK_PARAM_A 0
#define TEUK_PARAM_M 1
#define TEUK_PARAM_R0 2
#define TEUK_PARAM_AMP 3
int64_t teuk_param_gradient_workspace_bytes(teuk_ctx* ctx, int64_t n_steps, int64_t checkpoint_interval);
int teuk_param_gradient(teuk_ctx* ctx, int32_t param, double h, double rstar_obs, const void* dL_dwave,
                        int64_t n_steps, double t_start, const void* phi0, const void* pi0,
                        int64_t checkpoint_interval, void* workspace, int64_t workspace_bytes, double* dL_dparam,
                        void* dL_dphi0, void* dL_dpi0);

/* Autotuner (synchronous): times launches_per_trial launches (after one
 * warm-up launch) of every candidate tile shape -- theta rows per wavefront
 * in {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 80, 96, 112, 128, 192, 256}
 * clipped to n_theta, times four launch forms: 1 step per launch, 2 steps
 * on one wavefront in chunk-major or group-major block order, 2 steps on a
 * pair of wavefronts (teuk_set_tiling orders 0, 1 and 2) -- with HIP events
 * on the context's stream, twice (the second pass in the reverse order,
 * each candidate keeping its faster trial), keeps the fastest and reports
 * its rows and steps per launch in *rows_out and *kb_out (either may be
 * NULL; teuk_get_tiling reports the order).  The results of teuk_step are
 * bitwise identical for every candidate, so tuning changes speed only.
 * Needs a bound state; the trial launches read the current pair and write
 * the other one, so the state, time and waveform are unchanged.  The
 * reverse sweep has its own tiling (teuk_set_adjoint_tiling). */
int teuk_autotune(teuk_ctx* ctx, int32_t launches_per_trial, int32_t* rows_out, int32_t* kb_out);

/* Tile shape of the reverse sweep (FP64; performance only: dL/du^0 is
 * bitwise identical for every choice, the source gradients agree to
 * rounding, since their partial sums follow the tiles).  rows_per_wave:
 * theta rows per wavefront, 1..4096, or 0 (the default) to follow the step
 * kernel's rows (teuk_set_tiling, teuk_autotune); steps_per_launch: 1 (the
 * default) or 2 reverse steps per launch.  teuk_get_adjoint_tiling reports
 * the rows in effect.  TEUK_EINVAL outside these ranges. */
int teuk_set_adjoint_tiling(teuk_ctx* ctx, int32_t rows_per_wave, int32_t steps_per_launch);
int teuk_get_adjoint_tiling(teuk_ctx* ctx, int32_t* rows_per_wave, int32_t* steps_per_launch);

/* Autotuner of the reverse sweep (FP64, synchronous): as teuk_autotune
 * (two passes) over its candidate rows but 80 and 112, times 1 or 2
 * reverse steps per launch, timing
 * reverse-step launches that read the bound state's current pair as the
 * adjoint and write the other pair, so the state, time and waveform are
 * unchanged.  Allocates and frees a small device buffer for the trials'
 * gradient partial sums.  Keeps the fastest as the reverse-sweep tiling and
 * reports it (either pointer may be NULL).  TEUK_ENOTSUP for FP32 contexts,
 * TEUK_ESTATE without a bound state. */
int teuk_adjoint_autotune(teuk_ctx* ctx, int32_t launches_per_trial, int32_t* rows_out, int32_t* kb_out);

/* ------------------------------------------------------------- batches
 *
 * After the ansatz of Eq. (4) every azimuthal mode m (and every spin a or s)
 * is an independent 2+1 problem on its own grid (Sec. 2.2).  A batch steps
 * many such instances, of different sizes, together: one persistent kernel
 * launch advances every instance by 1 or 2 steps (the workgroups that fit
 * on the GPU at once walk the batch's tile list), and teuk_batch_step can
 * replay a captured HIP graph of such launches.  Per point the arithmetic
 * is the single-mode step's, so each instance's states and waveform are
 * bitwise identical to a teuk_ctx run with the same parameters started at
 * t = 0, step 0.  FP64 only. */
typedef struct {
    teuk_grid grid;
    double a, M;
    int32_t m, s;
    double dt;
    double r0;              /* source orbit radius (> r+); 0: no source      */
    double amp;             /* source amplitude (see teuk_set_source)        */
    double sigma_r_cells;   /* source widths in cells; <= 0 selects 2        */
    double sigma_th_cells;
    double rstar_obs;       /* extraction radius, strictly inside the grid   */
} teuk_desc;

typedef struct teuk_batch teuk_batch;

/* Create a batch of n instances (1..65535) described by descs, able to take
 * up to max_steps steps in all (the source phase of every step is tabulated
 * on the host at create, 32 B per step and instance).  The same checks as
 * teuk_create apply to each descriptor.  hip_stream: hipStream_t for all
 * work of the batch (graph capture needs a non-null stream).  The library
 * allocates the instances' coefficient and phase tables. */
int teuk_batch_create(int32_t n, const teuk_desc* descs, int64_t max_steps, void* hip_stream, teuk_batch** out);

/* Release the batch (synchronises its stream first). */
int teuk_batch_destroy(teuk_batch* b);

/* Bind instance i's caller-owned device buffers: (phi, pi) hold its current
 * state and (phi_next, pi_next) are the ping-pong partners, each
 * n_theta x n_rstar complex128 (layout as teuk_bind_state); wave (may be
 * NULL) receives its waveform rows [wave_rows][n_theta], row k = the state
 * after k steps of the batch.  Every instance must be bound before the
 * first step. */
int teuk_batch_bind(teuk_batch* b, int32_t i, void* phi, void* pi, void* phi_next, void* pi_next, void* wave,
                    int64_t wave_rows);

/* Moving source for instance i (an inspiral, as for teuk_set_trajectory):
 * r0_phase is a host array of n_half pairs (r0, phi) at t = k dt/2 counted
 * from the batch's step 0, so batch step s uses entries 2s (predictor) and
 * 2s + 1 (corrector); n_half >= 2 max_steps.  The instance keeps its
 * descriptor's amplitude and widths and needs a source (r0 != 0 in its
 * descriptor; TEUK_ESTATE otherwise).  Results equal, bit for bit, a
 * single-mode run given the same table at step 0.  NULL returns the
 * instance to its fixed orbit.  Synchronises the batch's stream.  Batches
 * with a moving instance run a separate build of the batch kernels; when a
 * call switches between the two, a captured graph is dropped
 * (teuk_batch_step then launches directly; capture again for replays).
 * TEUK_EINVAL for a short table or an entry with r0 <= r+ or a non-finite
 * value. */
int teuk_batch_set_trajectory(teuk_batch* b, int32_t i, const double* r0_phase, int64_t n_half);

/* Advance every instance n steps (Eqs. 13-14 with source and boundary
 * conditions): replays of the captured graph while at least its step count
 * remains, then direct launches.  TEUK_EINVAL past max_steps. */
int teuk_batch_step(teuk_batch* b, int64_t n);

/* Capture steps_per_graph steps (a positive multiple of the steps per
 * launch) as a HIP graph that teuk_batch_step replays; 0 drops the graph.
 * The kernels read the step and the current pair from a device-side
 * clock plus per-launch offsets, and one clock advance ends each replay, so
 * every replay continues where the last one stopped.  Changing the tiling
 * drops the graph. */
int teuk_batch_capture_graph(teuk_batch* b, int64_t steps_per_graph);

/* Tile shape for every instance (rows clipped to each n_theta; 0: the
 * per-instance default), steps per launch (1 or 2) and launch form:
 * persistent = 1 launches as many workgroups as stay resident, which walk
 * the batch's tile list (each XCD a contiguous range); 0 launches one
 * workgroup per tile.  Performance only; drops the graph. */
int teuk_batch_set_tiling(teuk_batch* b, int32_t rows_per_wave, int32_t steps_per_launch, int32_t persistent);

/* Autotuner: as teuk_autotune, over the whole batch (one rows value for all
 * instances, clipped to each n_theta) and both launch forms; reports the
 * choice (any out pointer may be NULL).  Trial launches leave the states,
 * the step count and the waveforms unchanged.  Drops the graph. */
int teuk_batch_autotune(teuk_batch* b, int32_t launches_per_trial, int32_t* rows_out, int32_t* kb_out,
                        int32_t* persistent_out);

/* 0: every instance's current state is in its (phi, pi) as bound at step 0;
 * 1: in (phi_next, pi_next).  Negative: error code. */
int teuk_batch_current(teuk_batch* b);
int teuk_batch_get_step(teuk_batch* b, int64_t* step);
int teuk_batch_status(teuk_batch* b);
const char* teuk_batch_last_error(teuk_batch* b);

/* Watchdog of a batch (see teuk_set_watchdog): with on != 0, every
 * teuk_batch_step call ends with a scan of each instance's state for a
 * value not below max_abs in magnitude (max_abs <= 0: non-finite only);
 * graph replays are not split, so the scans follow the calls, not a step
 * interval.  The finding (instance and step) reaches the host without a
 * wait; the next teuk_batch_step or teuk_batch_status turns it into the
 * sticky TEUK_EUNSTABLE, named in teuk_batch_last_error.  A call clears
 * earlier findings (it synchronises the stream); TEUK_EINVAL for max_abs
 * NaN.  Allocates 8 B of device and 8 B of pinned host memory on first use,
 * kept until teuk_batch_destroy. */
int teuk_batch_set_watchdog(teuk_batch* b, int32_t on, double max_abs);

/* Scan the current state for non-finite values (synchronous).  Returns
 * TEUK_OK, TEUK_EUNSTABLE, or the sticky error of an earlier failure. */
int teuk_check_finite(teuk_ctx* ctx);

/* Watchdog for long runs.  The explicit scheme of Eqs. (13)-(14) is stable
 * only while the time step and the grid keep every mode damped; where they
 * do not (a time step far below dr*, a source a few cells wide) a poorly
 * resolved mode can grow without bound.  With every_steps > 0, teuk_step
 * scans the state (Phi and Pi, real and imaginary parts) whenever the step
 * count reaches a multiple of every_steps, for a value whose magnitude is
 * not below max_abs (max_abs <= 0: for non-finite values only).  Launches
 * are split so that each multiple is a launch boundary (results stay
 * bitwise identical; each scan reads the state once).  The scans run on the
 * context's stream and teuk_step stays asynchronous: each call ends by
 * copying the finding into host memory, and the first later teuk_step,
 * teuk_status or teuk_check_finite that sees it sets the sticky
 * TEUK_EUNSTABLE, with the step of the first failing scan in
 * teuk_last_error.  After a stream synchronisation, teuk_status reports
 * every scan of the calls made so far.  every_steps = 0 (the default)
 * turns the watchdog off; a call clears earlier findings (it synchronises
 * the stream).  TEUK_EINVAL for every_steps < 0 or max_abs NaN; allocates
 * 8 B of device memory and 8 B of pinned host memory on first use, kept
 * until teuk_destroy. */
int teuk_set_watchdog(teuk_ctx* ctx, int64_t every_steps, double max_abs);

/* Sticky status of the context (TEUK_OK if no call has failed), including
 * a watchdog finding that has reached the host. */
int teuk_status(teuk_ctx* ctx);

/* Text of the last failure of this context ("" if none). */
const char* teuk_last_error(teuk_ctx* ctx);

/* Name of an error code. */
const char* teuk_strerror(int code);

/* Suggested time step for n_steps steps of the explicit scheme (host only,
 * synchronous).  For data smooth in r* both Lax-Wendroff stages apply the
 * angular terms of S (Eq. 12), which acts on a theta-mode of frequency w as
 * the explicit midpoint rule with |G|^2 = 1 + (w dt)^4 / 4; the rule keeps
 * the growth of the stiffest mode to one e-fold over the run:
 * dt = min(dr* / 2, (8/n_steps)^(1/4) / w_max), with w_max^2 bounded by the
 * Gershgorin bound of the discrete angular operator times max Delta/Sigma^2. */
int teuk_suggest_dt(const teuk_grid* g, double a, double M, int32_t m, int32_t s,
                    int64_t n_steps, double* dt_out);

/* Bandwidth probe (not part of the method): copy `bytes` (a multiple of 16)
 * from src to dst, two non-overlapping 16-byte-aligned device buffers owned by
 * the caller, with a plain streaming kernel on hip_stream (NULL: the null
 * stream); asynchronous.  It measures what HBM delivers to a kernel that
 * only reads and writes, the practical ceiling beside the step kernel's
 * bandwidth, and it is the kernel of known traffic against which hardware
 * byte counters are calibrated.  TEUK_EINVAL for bad sizes, alignment or
 * overlap; TEUK_EDEVICE if the launch fails. */
int teuk_stream_copy(const void* src, void* dst, int64_t bytes, void* hip_stream);

/* Geometry probe (host only): r*(r) from Eq. (2) and its inverse as
 * delta = r - r+. */
double teuk_rstar_of_r(double r, double a, double M);
double teuk_delta_of_rstar(double rstar, double a, double M);

#ifdef __cplusplus
}
#endif

#endif /* TEUK_H */
