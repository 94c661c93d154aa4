// HIP kernels of libteuk for gfx950 (MI355X).
//
// lw_step: one fused two-step Lax-Wendroff update (paper Eqs. 13-14) of the
// first-order m-mode Teukolsky system (Eqs. 8-12), with the particle source
// and the boundary conditions (text after Eq. 14) fused in.
//
// Work decomposition.  A wavefront owns a strip of 64 consecutive r*
// columns (one per lane, r* contiguous in memory so every row load is one
// coalesced 1 KiB (FP64) access per field) and marches upwards through a
// chunk of theta rows.  Lane l holds column c = strip*62 - 1 + l; the
// predictor value at the half point c+1/2 needs column c+1, which comes
// from the neighbouring lane by a DPP wavefront shift; the corrector at c
// needs the half point c-1/2 from the lane below.  Lanes 1..62 therefore
// produce valid outputs and neighbouring strips overlap by two columns.
// Along theta the three-point angular stencil of each stage is served from
// a register window of three rows, so u^n is read from HBM once per row
// (plus a 4-row halo per chunk) and u^{n+1} written once: 64 B per update
// in FP64, 32 B in FP32.  The half-step values never leave registers.
//
// Coefficients.  All coefficients of Eqs. (5)-(12) are separable into
// radial numerators (kept in registers for the lane's column) and angular
// factors (wave-uniform per row, read through the scalar cache); per point
// only Sigma^2 = w2^2 - a^2 Delta sin^2 and one reciprocal square root are
// formed.  The rsqrt starts from the hardware estimate and is refined by
// Newton steps to full precision.
#include <type_traits>

#include "teuk_internal.h"

namespace teuk {

template <typename R>
struct cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

template <typename R> struct vec2;
template <> struct vec2<double> { using T = double2; };
template <> struct vec2<float> { using T = float2; };

template <typename R>
__device__ __forceinline__ cx<R> ldc(const R* base, int64_t idx) {
    typename vec2<R>::T v = reinterpret_cast<const typename vec2<R>::T*>(base)[idx];
    return {v.x, v.y};
}
template <typename R>
__device__ __forceinline__ void stc(R* base, int64_t idx, cx<R> v) {
    typename vec2<R>::T w;
    w.x = v.re;
    w.y = v.im;
    reinterpret_cast<typename vec2<R>::T*>(base)[idx] = w;
}

// Row access with a wave-uniform row base and a 32-bit per-lane byte offset
// (the grid is limited to 2^26 r* nodes, so offsets stay below 2^31).
template <typename R>
__device__ __forceinline__ cx<R> ld_row(const R* __restrict__ base, int64_t row_elem, unsigned boff) {
    const char* p = reinterpret_cast<const char*>(base + 2 * row_elem) + boff;
    typename vec2<R>::T v = *reinterpret_cast<const typename vec2<R>::T*>(p);
    return {v.x, v.y};
}
template <typename R>
__device__ __forceinline__ void st_row(R* __restrict__ base, int64_t row_elem, unsigned boff, cx<R> v) {
    char* p = reinterpret_cast<char*>(base + 2 * row_elem) + boff;
    typename vec2<R>::T w;
    w.x = v.re;
    w.y = v.im;
    *reinterpret_cast<typename vec2<R>::T*>(p) = w;
}

// Row load through a pointer hidden from the optimiser (kept in the global
// address space): its value cannot be rematerialised as a second load
// later (which would miss in L2 and double the HBM reads), so carried rows
// stay in registers.
template <typename R>
__device__ __forceinline__ cx<R> ld_row_once(const R* base, int64_t row_elem, unsigned boff) {
    typedef __attribute__((address_space(1))) const char* gptr;
    gptr p = (gptr)(base + 2 * row_elem);
    asm volatile("" : "+s"(p));
    typedef R v2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(1))) const v2* gvec;
    v2 v = *(gvec)(p + boff);
    return {v.x, v.y};
}

// Cross-lane shifts by one lane with DPP whole-wavefront moves (VALU, no
// LDS round trip): wave_shl:1 gives lane i the value of lane i+1, wave_shr:1
// that of lane i-1.  The lane without a source reads 0 (bound control); in
// the step kernel those are lanes 63 and 0, whose results are never stored.
constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;

template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
    int v = __builtin_bit_cast(int, x);
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
    struct I2 { int lo, hi; };
    I2 v = __builtin_bit_cast(I2, x);
    I2 r;
    r.lo = __builtin_amdgcn_mov_dpp(v.lo, CTRL, 0xf, 0xf, true);
    r.hi = __builtin_amdgcn_mov_dpp(v.hi, CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, r);
}

template <typename R>
__device__ __forceinline__ cx<R> shfl_dn1(cx<R> v) {
    return {dpp_move<DPP_WAVE_SHL1>(v.re), dpp_move<DPP_WAVE_SHL1>(v.im)};
}
template <typename R>
__device__ __forceinline__ cx<R> shfl_up1(cx<R> v) {
    return {dpp_move<DPP_WAVE_SHR1>(v.re), dpp_move<DPP_WAVE_SHR1>(v.im)};
}

// 1/sqrt(x) to full precision: hardware estimate plus Newton steps
// y <- y + y (1/2 - (x/2) y^2).
__device__ __forceinline__ double rsqrt_full(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x;
    double e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
    e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
    return y;
}
__device__ __forceinline__ float rsqrt_full(float x) {
    float y = __builtin_amdgcn_rsqf(x);
    float h = 0.5f * x;
    float e = fmaf(-h * y, y, 0.5f);
    return fmaf(y, e, y);
}

// Blocks are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8);
// remap so that each XCD walks a contiguous range of tiles, keeping the
// neighbouring strips and chunks that share halo rows in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int X = 8;
    int q = nb / X, r = nb % X;
    int x = b % X, k = b / X;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// Radial numerators of one column (one radial location).
template <typename R>
struct Rad {
    R w2, del, wbn, ctr, cti0, crr, vr, vi, gr;
};

// Radial numerators used by the step, in the order they sit in LDS.
constexpr int N_RAD_USED = 9;
__device__ __constant__ const int kRadField[N_RAD_USED] = {R_W2, R_DEL, R_WBN, R_CTR, R_CTI0,
                                                           R_CRR, R_VR, R_VI, R_GR};

// The table is loop invariant; reading it anew at every use (the empty asm
// hides the index from loop-invariant code motion) keeps 2 x 9 values per
// lane out of the register file.
template <typename R>
__device__ __forceinline__ Rad<R> lds_rad(const R (*t)[WAVE], int lane) {
    int z = 0;
    asm volatile("" : "+s"(z));
    lane += z;
    Rad<R> r;
    r.w2 = t[0][lane];
    r.del = t[1][lane];
    r.wbn = t[2][lane];
    r.ctr = t[3][lane];
    r.cti0 = t[4][lane];
    r.crr = t[5][lane];
    r.vr = t[6][lane];
    r.vi = t[7][lane];
    r.gr = t[8][lane];
    return r;
}

// Angular factors of one theta row (wave-uniform: scalar loads).
template <typename R>
struct Ang {
    R sin2, a2s2, cs, wp, wm, w0, agth;
};

template <typename R>
__device__ __forceinline__ Ang<R> load_ang(const R* __restrict__ ang, int row) {
    const R* g = ang + (int64_t)row * A_STRIDE;
    Ang<R> a;
    a.sin2 = g[A_SIN2];
    a.a2s2 = g[A_A2S2];
    a.cs = g[A_CS];
    a.wp = g[A_P];
    a.wm = g[A_M];
    a.w0 = g[A_0];
    a.agth = g[A_AGTH];
    return a;
}

// Non-angular part of one Lax-Wendroff stage at one point.
//
// With w2 = r^2 + a^2 and y = 1/Sigma (Eq. 7), the coefficients of S
// (Eq. 12) are b = w2 y and numerator/Sigma^2 for c_t, c_r, V, with
// b b_* = WBN sin^2 y^4, so that
//   -mu dPhi - V Phi - c_t Pi = -y^2 [CR dPhi + V Phi + CT (Pi - b dPhi)],
//   CR = CRR + WBN sin^2 y^2 + i (-2 m a w2),  CT = CTR + i (CTI0 + 2 s a cos Delta).
// The stage of length tau (dt/2 for the predictor, dt for the corrector)
// then gives, from the means (f, g) of (Phi, Pi) and their r* differences
// (df, dg):
//   Phi' = f0 + tau (g - b df)                         (complete)
//   Pi'  = g0 + tau (b dg + T - y^2 [...])             (without the angular term)
//   D    = tau Delta y^2                               (weight of Lth Phi)
template <typename R>
struct Stage {
    cx<R> phi, pi_part;
    R dw;
};

template <typename R>
__device__ __forceinline__ Stage<R> stage(const Rad<R>& q, const Ang<R>& g, R m2ma, R tau, cx<R> ph,
                                          cx<R> f0, cx<R> g0, cx<R> f, cx<R> gm, cx<R> df, cx<R> dg) {
    R S2 = fma(q.w2, q.w2, -g.a2s2 * q.del);   // Sigma^2
    R y = rsqrt_full(S2);                      // 1/Sigma
    R y2 = y * y;
    R b = q.w2 * y;                            // b, Eq. (6)
    cx<R> X = {fma(-b, df.re, gm.re), fma(-b, df.im, gm.im)};          // Pi - b dPhi
    cx<R> CR = {fma(q.wbn * g.sin2, y2, q.crr), m2ma * q.w2};
    cx<R> CT = {q.ctr, fma(g.cs, q.del, q.cti0)};
    cx<R> V = {q.vr, q.vi};
    cx<R> acc = cmul(CR, df) + cmul(V, f) + cmul(CT, X);
    cx<R> T = (g.agth * q.gr) * ph;
    Stage<R> o;
    o.phi = {fma(tau, X.re, f0.re), fma(tau, X.im, f0.im)};
    cx<R> rhs = {fma(b, dg.re, fma(-y2, acc.re, T.re)), fma(b, dg.im, fma(-y2, acc.im, T.im))};
    o.pi_part = {fma(tau, rhs.re, g0.re), fma(tau, rhs.im, g0.im)};
    o.dw = tau * q.del * y2;
    return o;
}

template <typename R>
__global__ __launch_bounds__(256) void lw_step_kernel(const R* __restrict__ phi, const R* __restrict__ pi,
                                                    R* __restrict__ phi_out, R* __restrict__ pi_out,
                                                    const R* __restrict__ rad_i, const R* __restrict__ rad_h,
                                                    const R* __restrict__ ang, R* __restrict__ wave,
                                                    StepArgs<R> A) {
    const int lane = threadIdx.x & (WAVE - 1);
    // wave-uniform quantities: keep them in scalar registers
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    // A workgroup = WG_WAVES adjacent r* strips at the same theta chunk, so
    // that every row access of the group is one contiguous 4 KiB (FP64)
    // span; blocks run chunk-major so that concurrent groups on an XCD also
    // touch neighbouring columns of the same rows.
    const int ngrp = (A.n_strips + WG_WAVES - 1) / WG_WAVES;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int chunk = blk / ngrp;
    const int strip = (blk - chunk * ngrp) * WG_WAVES + wid;
    if (strip >= A.n_strips) return;  // wave-uniform; the kernel has no barriers
    const int nr = A.nr, nth = A.nth;
    const int c = strip * STRIP_OUT - 1 + lane;
    // Lanes outside the grid read a clamped column: they feed only the
    // half points beyond the r* boundaries, whose outputs are the Dirichlet
    // zeros or are never stored.
    const unsigned cu = (unsigned)min(max(c, 0), nr - 1);
    // radial numerators of this wavefront's columns (each wavefront fills
    // and reads only its own slice, so no barrier is needed)
    __shared__ R srad_all[WG_WAVES][2][N_RAD_USED][WAVE];   // [wave][half/integer][field][lane]
    R (*srad)[N_RAD_USED][WAVE] = srad_all[wid];
    for (int k = 0; k < 2 * N_RAD_USED; ++k) {
        const int loc = k / N_RAD_USED, f = k % N_RAD_USED;
        srad[loc][f][lane] = (loc == 0 ? rad_h : rad_i)[(int64_t)kRadField[f] * A.stride + cu];
    }
    const int j0 = chunk * A.rows;
    const int jend = min(j0 + A.rows, nth);
    const bool out_lane = (c >= 0) && (c < nr) && lane >= 1 && lane <= WAVE - 2;
    const R keep = ((c == 0) || (c == nr - 1)) ? R(0) : R(1);   // Phi = Pi = 0 on the r* boundary
    const unsigned boff = cu * (unsigned)(2 * sizeof(R));          // byte offset of this lane's column
    const unsigned soff = (unsigned)max(c, 0) * (unsigned)(2 * sizeof(R));
    const R dt = A.dt, hdt = A.hdt, idr = A.inv_dr, m2ma = A.m2ma;
    const cx<R> ph0 = {A.ph0_re, A.ph0_im}, ph1 = {A.ph1_re, A.ph1_im};
    const R half = R(0.5);
    const cx<R> zero = {R(0), R(0)};
    const bool rec = (A.wave_row >= 0) && (A.iobs / STRIP_OUT == strip);
    const int wl = A.iobs - strip * STRIP_OUT + 1;

    // Rings indexed by (row - Ls) mod 3, resolved at compile time by the
    // three-way unrolled loop below.
    cx<R> pb[3] = {zero, zero, zero};  // Phi at half points, time n   (rows L-2..L)
    cx<R> phh[3] = {zero, zero, zero}; // Phi at integer points, time n+1/2 (rows L-3..L-1)
    // Each stage is split into its angular part, which needs the next row,
    // and the rest.  Pending (non-angular) parts:
    cx<R> hP = zero, hQp = zero;  // predictor of half row L-1: final Phi, partial Pi
    R hD = R(0);                  // (dt/2) Delta/Sigma^2 at that half row
    cx<R> nQp = zero;             // corrector of row L-2: partial Pi
    R nD = R(0);                  // dt Delta/Sigma^2 at that row

    const int Ls = max(j0 - 2, 0);
    const int Le = min(j0 + A.rows + 1, nth + 1);
    const int Plo = max(j0 - 1, 0), Phi_ = min(j0 + A.rows, nth - 1);
    // prefetch ring, indexed like the other rings (row Ls is always inside
    // the grid; row Ls+1 too unless the grid has a single row chunk edge)
    cx<R> pf_p = ld_row_once(phi, (int64_t)Ls * nr, boff), pf_q = ld_row_once(pi, (int64_t)Ls * nr, boff);
    cx<R> u_p = zero, u_q = zero;   // u^n of the previous row

    // Every stage sits behind a wave-uniform branch; the branches also keep
    // the scheduler from stretching live ranges across stages.
    auto iter = [&](auto PHC, int L) {
        constexpr int S0 = decltype(PHC)::value;   // slot of row L
        constexpr int S1 = (S0 + 2) % 3;          // slot of row L-1
        constexpr int S2 = (S0 + 1) % 3;          // slot of row L-2 (and L-3 -> S0 for phh)
        if (L > Le) return;
        const int P = L - 1, Q = L - 2;
        // Rows L and L+1 were requested by earlier iterations; request row
        // L+2 now into the slot that row L-1 used.  Row P = L-1 stays in
        // registers for the corrector (B2): re-reading it would miss in L2
        // at full occupancy and double the HBM read traffic.
        const cx<R> up = u_p, uq = u_q;
        cx<R> p = pf_p, q = pf_q;
        u_p = p;
        u_q = q;
        if (L + 1 < nth && L + 1 <= Le) {
            const int64_t row = (int64_t)(L + 1) * nr;
            pf_p = ld_row_once(phi, row, boff);
            pf_q = ld_row_once(pi, row, boff);
        }
        __builtin_amdgcn_sched_barrier(0);
        // ---- A1: row L; half-point mean and compact differences at c+1/2
        cx<R> Qb, dP, dQ;   // set when row L exists; read only by A2, which implies it
        if (L < nth) {
            cx<R> p1 = shfl_dn1(p), q1 = shfl_dn1(q);
            pb[S0] = half * (p + p1);
            Qb = half * (q + q1);
            dP = idr * (p1 - p);
            dQ = idr * (q1 - q);
            if (rec && L >= j0 && L < jend) {
                if (lane == wl) stc(wave, A.wave_row * nth + L, (R(1) - A.alpha) * p + A.alpha * p1);
            }
        }
        // ---- B1: finish the predictor (Eq. 13) of half row P and form the
        //      corrector's means and differences at c (time n+1/2)
        cx<R> Qh, dhP, dhQ;  // set by B1; read only by B2, whose rows are a subset
        if (P >= Plo && P <= Phi_) {
            const R* ag = ang + (int64_t)P * A_STRIDE;
            const R wp = ag[A_P], wm = ag[A_M], w0 = ag[A_0];
            cx<R> Lf = wp * pb[S0] + wm * pb[S2] + w0 * pb[S1];
            cx<R> hQ = hQp + hD * Lf;
            cx<R> hPm = shfl_up1(hP), hQm = shfl_up1(hQ);
            phh[S1] = half * (hP + hPm);
            Qh = half * (hQ + hQm);
            dhP = idr * (hP - hPm);
            dhQ = idr * (hQ - hQm);
        }
        // ---- A2: non-angular part of the predictor of half row L
        if (L >= Plo && L <= Phi_) {
            const Ang<R> g = load_ang(ang, L);
            const Rad<R> qh = lds_rad<R>(srad[0], lane);   // half point c+1/2
            Stage<R> o = stage(qh, g, m2ma, hdt, ph0, pb[S0], Qb, pb[S0], Qb, dP, dQ);
            hP = o.phi;
            hQp = o.pi_part;
            hD = o.dw;
        }
        // ---- C: finish the corrector (Eq. 14) of row Q; store its Pi
        if (Q >= j0 && Q < jend) {
            const R* ag = ang + (int64_t)Q * A_STRIDE;
            const R wp = ag[A_P], wm = ag[A_M], w0 = ag[A_0];
            cx<R> Lf = wp * phh[S1] + wm * phh[S0] + w0 * phh[S2];
            cx<R> nQ = keep * (nQp + nD * Lf);
            if (out_lane) st_row(pi_out, (int64_t)Q * nr, soff, nQ);
        }
        // ---- B2: non-angular part of the corrector of row P; its Phi is final
        if (P >= j0 && P < jend) {
            const Ang<R> g = load_ang(ang, P);
            const int64_t row = (int64_t)P * nr;
            const Rad<R> qi = lds_rad<R>(srad[1], lane);   // integer point c
            Stage<R> o = stage(qi, g, m2ma, dt, ph1, up, uq, phh[S1], Qh, dhP, dhQ);
            nQp = o.pi_part;
            nD = o.dw;
            if (out_lane) st_row(phi_out, row, soff, keep * o.phi);
        }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    for (int L = Ls; L <= Le; L += 3) {
        iter(I0{}, L);
        iter(I1{}, L + 1);
        iter(I2{}, L + 2);
    }
}

template <typename R>
static void launch_step(const StepArgs<R>& a, hipStream_t s) {
    int blocks = ((a.n_strips + WG_WAVES - 1) / WG_WAVES) * a.n_chunks;
    hipLaunchKernelGGL(lw_step_kernel<R>, dim3(blocks), dim3(WAVE * WG_WAVES), 0, s, a.phi, a.pi, a.phi_out,
                       a.pi_out, a.rad_i, a.rad_h, a.ang, a.wave, a);
}
void launch_step_fp64(const StepArgs<double>& a, hipStream_t s) { launch_step(a, s); }
void launch_step_fp32(const StepArgs<float>& a, hipStream_t s) { launch_step(a, s); }

// Waveform at r*_obs: w_j = (1 - alpha) Phi_{i0,j} + alpha Phi_{i0+1,j}.
template <typename R>
__global__ void extract_kernel(const R* __restrict__ phi, R* __restrict__ out, int nr, int nth, int i0,
                               R alpha) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nth) return;
    cx<R> p0 = ldc(phi, (int64_t)j * nr + i0);
    cx<R> p1 = ldc(phi, (int64_t)j * nr + i0 + 1);
    stc(out, j, (R(1) - alpha) * p0 + alpha * p1);
}
void launch_extract_fp64(const double* phi, double* out, int nr, int nth, int iobs, double alpha,
                         hipStream_t s) {
    hipLaunchKernelGGL(extract_kernel<double>, dim3((nth + 255) / 256), dim3(256), 0, s, phi, out, nr, nth,
                       iobs, alpha);
}
void launch_extract_fp32(const float* phi, float* out, int nr, int nth, int iobs, float alpha,
                         hipStream_t s) {
    hipLaunchKernelGGL(extract_kernel<float>, dim3((nth + 255) / 256), dim3(256), 0, s, phi, out, nr, nth,
                       iobs, alpha);
}

// Non-finite scan: a lane that sees a NaN or Inf stores 1 into *flag
// (a divergent vector store; every such store writes the same value).
template <typename R>
__global__ void nonfinite_kernel(const R* __restrict__ x, int64_t n, unsigned int* flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t step = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (; i < n; i += step) bad |= !isfinite(x[i]);
    if (bad) *flag = 1u;
}
void launch_count_nonfinite_fp64(const double* x, int64_t n, unsigned int* flag, hipStream_t s) {
    hipLaunchKernelGGL(nonfinite_kernel<double>, dim3(1024), dim3(256), 0, s, x, n, flag);
}
void launch_count_nonfinite_fp32(const float* x, int64_t n, unsigned int* flag, hipStream_t s) {
    hipLaunchKernelGGL(nonfinite_kernel<float>, dim3(1024), dim3(256), 0, s, x, n, flag);
}

}  // namespace teuk
