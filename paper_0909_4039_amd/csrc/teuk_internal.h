// Internal declarations shared by the host API, the geometry builder and the
// HIP kernels of libteuk.  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/teuk.h"

namespace teuk {

// Radial table fields, stored structure-of-arrays: tab[f * stride + i].
// Two tables exist: at integer nodes r*_i and at half nodes r*_{i+1/2}.
// With w2 = r^2 + a^2, every coefficient of S (Eq. 12) is a radial field
// times at most one angular factor, all over Sigma^2 = w2^2 - a^2 Delta sin^2.
enum RadField : int {
    R_W2 = 0,  // w2
    R_DEL,     // Delta
    R_WBN,     // a^2 Delta [(r-M) w2 - 2 r Delta]       (b b_* = WBN sin^2 / Sigma^4)
    R_CTR,     // 2 s (r Delta - M (r^2 - a^2))          (Sigma^2 Re c_t)
    R_CTI0,    // 4 M a m r                              (Sigma^2 Im c_t = CTI0 + 2 s a cos Delta)
    R_CRR,     // -[6 w2 Delta / r + 2 r Delta + 2 s (r-M) w2]   (Sigma^2 Re c_r; Im c_r = -2 m a w2)
    R_VR,      // -Delta (6 Delta / r^2 + 6 (1+s)(r-M)/r)        (Sigma^2 Re V)
    R_VI,      // -[6 m a Delta / r + 4 s m a (r - M)]           (Sigma^2 Im V)
    R_GR,      // source radial Gaussian exp(-(r* - r*0)^2 / (2 sr^2))
    R_XR,      // (r* - r*0) / sr^2   (d/dr*0 of the Gaussian's exponent)
    R_NFIELDS
};

// Angular table fields per theta row: ang[j * A_STRIDE + f].  The pole
// rows fold the ghost cell (mirror with sign (-1)^|m+s|) into their weights.
enum AngField : int {
    A_SIN2 = 0,  // sin^2 theta
    A_A2S2,      // a^2 sin^2 theta
    A_CS,        // 2 s a cos theta
    A_P,         // weight of f_{j+1}: 1/h^2 + cot/(2h)        (0 on the last row)
    A_M,         // weight of f_{j-1}: 1/h^2 - cot/(2h)        (0 on the first row)
    A_0,         // weight of f_j: -2/h^2 + s - (m + s cos)^2 / sin^2 (+ folded ghost)
    A_GTH,       // source theta Gaussian
    A_AGTH,      // amp x source theta Gaussian
    A_NFIELDS
};
constexpr int A_STRIDE = 8;

struct Geometry {
    int64_t nr = 0, nth = 0;
    double rmin = 0, rmax = 0, dr = 0, dth = 0;
    double a = 0, M = 1;
    int m = 0, s = 0;
    double rp = 0, rm = 0;
    int64_t stride = 0;               // padded nr
    std::vector<double> rad_i, rad_h;  // R_NFIELDS * stride each
    std::vector<double> ang;           // nth * A_STRIDE
};

// Eq. (2): r*(delta) with delta = r - r+ and its inverse (Newton in ln delta).
double rstar_of_delta(double delta, double a, double M);
double delta_of_rstar(double rstar, double a, double M);

// Build the radial and angular tables (source columns left at zero).
void build_geometry(Geometry& g);
// Fill the source columns (R_GR, R_XR, A_GTH) for a source centred at r*0.
void build_source(Geometry& g, double rstar0, double sr, double sth, double amp);
// Gershgorin bound of the discrete angular operator and max Delta/Sigma^2.
double angular_bound(const Geometry& g);
double max_delta_over_sigma2(const Geometry& g);

// Default theta rows per wavefront tile for a grid of nth rows.
int default_rows(int nth, int kblock, int prec);
// Observer column i0 and weight alpha for r*_obs; false outside the open grid.
bool observer_index(const Geometry& g, double rstar_obs, int& i0, double& alpha);
// Argument checks shared by teuk_create, teuk_suggest_dt and teuk_batch_create.
int validate_phys(const teuk_grid* g, double a, double M, int32_t s);
// Omega = sqrt(M) / (r0^{3/2} + a sqrt(M)), circular equatorial orbit.
double orbit_omega(double r0, double a, double M);

// ------------------------------------------------------------------ kernels

constexpr int KB_MAX = 2;   // steps fused per launch (temporal blocking)

template <typename R>
struct StepArgs {
    const R* phi;      // interleaved complex [nth][nr]
    const R* pi;
    R* phi_out;
    R* pi_out;
    const R* rad_i;    // [R_NFIELDS][stride]
    const R* rad_h;
    const R* ang;      // [nth][A_STRIDE]
    int64_t stride;
    int32_t nr, nth;
    int32_t rows;      // theta rows per wavefront tile
    int32_t n_strips;  // r* strips of (64 - 2 kb) output columns
    int32_t n_chunks;  // theta chunks per strip
    int32_t n_tiles;   // n_strips * n_chunks
    int32_t order;     // block order: 0 chunk-major, 1 strip-group-major
    int32_t kb;        // steps in this launch (1 or 2)
    int32_t split;     // kb = 2 on a pair of wavefronts, one step each (lw_step_split_kernel)
    int32_t stream_out;  // 1: the state pair exceeds the last-level cache (FP64 two-step launches then store
                         //    their output rows non-temporally)
    R dt, hdt, inv_dr;
    R m2ma;            // -2 m a  (Sigma^2 Im c_r = m2ma w2)
    // per fused step k: e^{-i m Omega t^{n+k}} and e^{-i m Omega (t^{n+k} + dt/2)}
    R ph[2 * KB_MAX][2];
    // waveform rows of the states entering each fused step (-1: not recorded)
    R* wave;
    int64_t wave_row[KB_MAX];
    int32_t iobs;
    R alpha;
    // moving source: centre r*0 at the predictor (2k) and corrector (2k+1)
    // times of fused step k; the radial factor is exp(-(r* - r*0)^2 / two_sr2)
    int32_t moving;
    R rs0[2 * KB_MAX];
    R two_sr2;
    R rmin, dr;
};

// Arguments of one launch of the reverse sweep (FP64 only).  Stage k of a
// launch reverses forward step g_row[k]: it reads lambda^{g_row[k]+1} and
// writes lambda^{g_row[k]}; t[2k], t[2k+1] and ph[2k], ph[2k+1] are that
// step's predictor and corrector times and source phases.
struct AdjArgs {
    const double* lp;     // lambda^{n+kb}: interleaved complex [nth][nr]
    const double* lq;
    double* lp_out;       // lambda^n
    double* lq_out;
    const double* rad_i;
    const double* rad_h;
    const double* ang;
    int64_t stride;
    int32_t nr, nth;
    int32_t rows, n_strips, n_chunks, kb;
    double dt, hdt, inv_dr, m2ma;
    double ph[2 * KB_MAX][2];
    double t[2 * KB_MAX];
    const double* g;      // dL/dw rows [n + 1][nth]
    int64_t g_row[KB_MAX];
    int32_t iobs;
    double alpha;
    double* slots;        // [blocks][WG_WAVES][3] source-gradient partial sums
    // moving source: r*0 of the orbit-table entry of every stage, [2k] for
    // step k's predictor (half points) and [2k + 1] for its corrector
    // (integer points); per-launch partial sums go to mslots,
    // [tile blocks][WG_WAVES][2 kb][3], written (not added) by every wave.
    // The launch has one block more than tiles: block 0 reduces the previous
    // launch's slots (prev_mslots, NULL for the first launch) into mout.
    int32_t moving;
    double rs0[2 * KB_MAX];
    double inv_sr2, two_sr2, rmin, dr;
    double* mslots;
    const double* prev_mslots;
    int64_t prev_n_slots, prev_top;
    int32_t prev_kb;
    double* mout;         // [table entries][3] per-entry sums
};

// One instance of a batch (FP64): its bound buffers, tables and constants.
// Tiles are numbered instance by instance; first_tile[kb - 1] is the first
// global tile of this instance for launches of kb steps.
struct BatchInst {
    double* buf[2][2];        // [pair][Phi, Pi], interleaved complex [nth][nr]
    const double* rad_i;
    const double* rad_h;
    const double* ang;
    const double* phase;      // [rows][4]: e^{-i m Omega t_k}, e^{-i m Omega (t_k + dt/2)}
    double* wave;             // [wave_cap][nth] or NULL
    int64_t wave_cap;
    int64_t stride;
    int32_t nr, nth, rows, iobs;
    int32_t first_tile[KB_MAX];
    double dt, hdt, inv_dr, m2ma, alpha;
    // moving source: [rows][2] r*0 at t_k and t_k + dt/2 (NULL: fixed orbit),
    // with the Gaussian's 2 sr^2 and the grid's r*_min, dr*
    const double* rs0tab;
    double two_sr2, rmin, dr;
};

// Device clock of a batch: steps taken and launches made (the launch
// parity selects the pair that holds the current states).
struct BatchClock {
    int64_t step;
    int64_t launches;
};

struct BatchArgs {
    const BatchInst* inst;
    const BatchClock* clock;
    int32_t n_inst;
    int32_t n_tiles;          // total tiles at this launch's kb
    int32_t kb;
    int32_t record;           // 0: recorder off (trial launches)
    int32_t persistent;       // 1: resident grid walking the tile list; 0: one workgroup per tile
    int32_t step_off;         // this launch's step and launch count relative to the clock
    int32_t launch_off;
    int32_t moving;           // 1: some instance has a moving source (the kernels built for it)
};

// Context accessors (defined with the context in teuk_api.cpp): the device
// that was current at teuk_create, and recording a failure in the context
// (sticky for TEUK_EDEVICE and TEUK_EUNSTABLE) while returning its code.
int ctx_device(const teuk_ctx* c);
int ctx_fail(teuk_ctx* c, int code, const char* msg);

constexpr int WAVE = 64;
constexpr int WG_WAVES = 4;

void launch_step_fp64(const StepArgs<double>& a, hipStream_t s);
void launch_step_fp32(const StepArgs<float>& a, hipStream_t s);
// FP32 storage with FP64 arithmetic: the state and waveform pointers of `a`
// point to float.
void launch_step_fp32s(const StepArgs<double>& a, hipStream_t s);
void launch_extract_fp64(const double* phi, double* out, int nr, int nth, int iobs, double alpha,
                         hipStream_t s);
void launch_extract_fp32(const float* phi, float* out, int nr, int nth, int iobs, float alpha,
                         hipStream_t s);
void launch_batch_step(const BatchArgs& a, int blocks, hipStream_t s);
void launch_batch_advance(BatchClock* clock, int steps, int launches, hipStream_t s);
void launch_batch_extract(const BatchInst* inst, int n_inst, int max_nth, const BatchClock* clock, hipStream_t s);
int batch_blocks_per_cu(int kb, bool moving);
void launch_adjoint_step(const AdjArgs& a, hipStream_t s);
void launch_adjoint_init(double* lp, double* lq, const double* g_row, int64_t n, int nr, int iobs, double alpha,
                         hipStream_t s);
void launch_fill_zero(double* x, int64_t n, hipStream_t s);
void launch_slot_sum(const double* slots, int64_t n_slots, double* out, hipStream_t s);
void launch_moving_slot_sum(const double* slots, int64_t n_slots, int kb, int64_t top, double* out,
                            hipStream_t s);
// Fused parameter-gradient contraction (lw_pdot_kernel): s[0] and s[1] are
// one-step launches of the contexts built at p + h and p - h on the same
// grid and tiling; the launch writes pdot_parts(s[0]) per-tile parts into
// part, which launch_pdot_sums adds up later.
struct PdotArgs {
    StepArgs<double> s[2];
    const double* lp;   // lambda^{k+1}: interleaved complex [nth][nr]
    const double* lq;
    double* part;
};
int64_t pdot_parts(const StepArgs<double>& a);
// Workgroups per CU that stay resident for lw_pdot_kernel and for the
// one-step FP64 step kernel (at least 1 each).
void sweep_blocks_per_cu(int* pdot, int* step1);
void launch_param_pdot(const PdotArgs& b, const double* phi, const double* pi, hipStream_t s);
// out[i] = the sum, in a fixed order, of the n_parts doubles at
// part + i n_parts, for i < n_steps (one launch).
void launch_pdot_sums(const double* part, int64_t n_parts, int64_t n_steps, double* out, hipStream_t s);
void launch_watch_fp64(const double* x, int64_t n, double lim, int64_t tag, unsigned long long* found,
                       hipStream_t s);
void launch_watch_fp32(const float* x, int64_t n, float lim, int64_t tag, unsigned long long* found,
                       hipStream_t s);
void launch_count_nonfinite_fp64(const double* x, int64_t n, unsigned int* flag, hipStream_t s);
void launch_count_nonfinite_fp32(const float* x, int64_t n, unsigned int* flag, hipStream_t s);

}  // namespace teuk
