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
// from the neighbouring lane by a cross-lane shuffle; the corrector at c
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

template <typename R>
__device__ __forceinline__ cx<R> shfl_dn1(cx<R> v) { return {__shfl_down(v.re, 1), __shfl_down(v.im, 1)}; }
template <typename R>
__device__ __forceinline__ cx<R> shfl_up1(cx<R> v) { return {__shfl_up(v.re, 1), __shfl_up(v.im, 1)}; }

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
    R w2, w4, a2d, del, bn, ctr, cti0, cti1, crr, cri, vr, vi, gr;
};

template <typename R>
__device__ __forceinline__ Rad<R> load_rad(const R* __restrict__ t, int64_t stride, int i) {
    Rad<R> r;
    r.w2 = t[R_W2 * stride + i];
    r.w4 = t[R_W4 * stride + i];
    r.a2d = t[R_A2D * stride + i];
    r.del = t[R_DEL * stride + i];
    r.bn = t[R_BN * stride + i];
    r.ctr = t[R_CTR * stride + i];
    r.cti0 = t[R_CTI0 * stride + i];
    r.cti1 = t[R_CTI1 * stride + i];
    r.crr = t[R_CRR * stride + i];
    r.cri = t[R_CRI * stride + i];
    r.vr = t[R_VR * stride + i];
    r.vi = t[R_VI * stride + i];
    r.gr = t[R_GR * stride + i];
    return r;
}

// Point coefficients of S (Eq. 12) assembled from separable parts.
template <typename R>
struct Pt {
    R b, dos2;
    cx<R> mu, V, ct;
};

template <typename R>
__device__ __forceinline__ Pt<R> point(const Rad<R>& q, R sin2, R cs) {
    Pt<R> p;
    R S2 = q.w4 - q.a2d * sin2;          // Sigma^2, Eq. (7)
    R y = rsqrt_full(S2);                // 1/Sigma
    R y2 = y * y;
    p.b = q.w2 * y;                      // b, Eq. (6)
    p.dos2 = q.del * y2;                 // Delta/Sigma^2
    p.ct = {q.ctr * y2, (q.cti0 + q.cti1 * cs) * y2};
    p.V = {q.vr * y2, q.vi * y2};
    R bst = q.bn * sin2 * y2 * y;        // b_* = d b / d r*
    // mu = c_r + b b_* - b c_t
    p.mu = {q.crr * y2 + p.b * bst - p.b * p.ct.re, q.cri * y2 - p.b * p.ct.im};
    return p;
}

template <typename R>
__global__ __launch_bounds__(256) void lw_step_kernel(StepArgs<R> A) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wid = threadIdx.x / WAVE;
    const int tile = xcd_remap(blockIdx.x, gridDim.x) * WG_WAVES + wid;
    if (tile >= A.n_tiles) return;  // wave-uniform; the kernel has no barriers
    const int strip = tile / A.n_chunks;
    const int chunk = tile - strip * A.n_chunks;
    const int nr = A.nr, nth = A.nth;
    const int j0 = chunk * A.rows;
    const int jend = min(j0 + A.rows, nth);
    const int c = strip * STRIP_OUT - 1 + lane;
    const bool inr = (c >= 0) && (c < nr);
    const int cc = min(max(c, 0), nr - 1);
    const bool out_lane = inr && lane >= 1 && lane <= WAVE - 2;
    const bool bc = (c == 0) || (c == nr - 1);
    const Rad<R> qh = load_rad(A.rad_h, A.stride, cc);  // half point c+1/2
    const Rad<R> qi = load_rad(A.rad_i, A.stride, cc);  // integer point c
    const R dt = A.dt, hdt = A.hdt, idr = A.inv_dr, gs = A.ghost;
    const cx<R> ph0 = {A.ph0_re, A.ph0_im}, ph1 = {A.ph1_re, A.ph1_im};
    const R half = R(0.5);
    const cx<R> zero = {R(0), R(0)};
    const bool rec = (A.wave_row >= 0) && (A.iobs / STRIP_OUT == strip);
    const int wl = A.iobs - strip * STRIP_OUT + 1;

    cx<R> Pb0 = zero, Pb1 = zero, Pb2 = zero, Qb1 = zero, Qb2 = zero;
    cx<R> dP1 = zero, dP2 = zero, dQ1 = zero, dQ2 = zero;
    cx<R> Ph0 = zero, Ph1 = zero, Ph2 = zero, Qh1 = zero, Qh2 = zero;
    cx<R> dhP1 = zero, dhP2 = zero, dhQ1 = zero, dhQ2 = zero;
    cx<R> UP0 = zero, UP1 = zero, UP2 = zero, UQ0 = zero, UQ1 = zero, UQ2 = zero;

    const int Ls = max(j0 - 2, 0);
    const int Le = min(j0 + A.rows + 1, nth + 1);
    const int Plo = max(j0 - 1, 0), Phi_ = min(j0 + A.rows, nth - 1);
    for (int L = Ls; L <= Le; ++L) {
        Pb0 = Pb1; Pb1 = Pb2; Qb1 = Qb2; dP1 = dP2; dQ1 = dQ2;
        Ph0 = Ph1; Ph1 = Ph2; Qh1 = Qh2; dhP1 = dhP2; dhQ1 = dhQ2;
        UP0 = UP1; UP1 = UP2; UQ0 = UQ1; UQ1 = UQ2;
        // ---- stage A: load row L, means and compact differences at c+1/2
        if (L < nth) {
            const int64_t k = (int64_t)L * nr + c;
            cx<R> p = inr ? ldc(A.phi, k) : zero;
            cx<R> q = inr ? ldc(A.pi, k) : zero;
            cx<R> p1 = shfl_dn1(p), q1 = shfl_dn1(q);
            Pb2 = half * (p + p1);
            Qb2 = half * (q + q1);
            dP2 = idr * (p1 - p);
            dQ2 = idr * (q1 - q);
            UP2 = p;
            UQ2 = q;
            if (rec && L >= j0 && L < jend && lane == wl) {
                cx<R> w = (R(1) - A.alpha) * p + A.alpha * p1;
                stc(A.wave, A.wave_row * nth + L, w);
            }
        }
        // ---- stage B: predictor (Eq. 13) at half point c+1/2, row P
        const int P = L - 1;
        if (P >= Plo && P <= Phi_) {
            const R* ag = A.ang + (int64_t)P * A_STRIDE;
            const R sin2 = ag[A_SIN2], cs = ag[A_COS], wp = ag[A_P], wm = ag[A_M], w0 = ag[A_0];
            const R gth = ag[A_GTH];
            cx<R> fm = (P == 0) ? gs * Pb1 : Pb0;
            cx<R> fp = (P == nth - 1) ? gs * Pb1 : Pb2;
            Pt<R> k = point(qh, sin2, cs);
            cx<R> Lf = wp * fp + wm * fm + w0 * Pb1;
            cx<R> T = (A.amp * qh.gr * gth) * ph0;
            cx<R> SPi = T - cmul(k.mu, dP1) + k.dos2 * Lf - cmul(k.V, Pb1) - cmul(k.ct, Qb1);
            cx<R> hP = Pb1 - hdt * (k.b * dP1 - Qb1);
            cx<R> hQ = Qb1 + hdt * (k.b * dQ1 + SPi);
            cx<R> hPm = shfl_up1(hP), hQm = shfl_up1(hQ);
            Ph2 = half * (hP + hPm);
            Qh2 = half * (hQ + hQm);
            dhP2 = idr * (hP - hPm);
            dhQ2 = idr * (hQ - hQm);
        }
        // ---- stage C: corrector (Eq. 14) at integer point c, row Q
        const int Q = L - 2;
        if (Q >= j0 && Q < jend) {
            const R* ag = A.ang + (int64_t)Q * A_STRIDE;
            const R sin2 = ag[A_SIN2], cs = ag[A_COS], wp = ag[A_P], wm = ag[A_M], w0 = ag[A_0];
            const R gth = ag[A_GTH];
            cx<R> fm = (Q == 0) ? gs * Ph1 : Ph0;
            cx<R> fp = (Q == nth - 1) ? gs * Ph1 : Ph2;
            Pt<R> k = point(qi, sin2, cs);
            cx<R> Lf = wp * fp + wm * fm + w0 * Ph1;
            cx<R> T = (A.amp * qi.gr * gth) * ph1;
            cx<R> SPi = T - cmul(k.mu, dhP1) + k.dos2 * Lf - cmul(k.V, Ph1) - cmul(k.ct, Qh1);
            cx<R> nP = UP0 - dt * (k.b * dhP1 - Qh1);
            cx<R> nQ = UQ0 + dt * (k.b * dhQ1 + SPi);
            if (bc) { nP = zero; nQ = zero; }
            if (out_lane) {
                const int64_t o = (int64_t)Q * nr + c;
                stc(A.phi_out, o, nP);
                stc(A.pi_out, o, nQ);
            }
        }
    }
}

template <typename R>
static void launch_step(const StepArgs<R>& a, hipStream_t s) {
    int blocks = (a.n_tiles + WG_WAVES - 1) / WG_WAVES;
    hipLaunchKernelGGL(lw_step_kernel<R>, dim3(blocks), dim3(WAVE * WG_WAVES), 0, s, a);
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
