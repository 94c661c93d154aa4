// Device helpers shared by the HIP kernels of libteuk (gfx950): complex
// arithmetic with explicit fused multiply-adds, row loads and stores,
// whole-wavefront DPP lane shifts, a full-precision reciprocal square root,
// the XCD-aware block remap and the coefficient tables' per-point views.
// Not part of the public ABI.
#pragma once

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
// The library is compiled without implicit multiply-add contraction; every
// fused multiply-add below is written out, so that the rounding of each
// point is the same whatever code surrounds it (tile shape, temporal
// blocking, batching).
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)};
}
// a b + c
template <typename R>
__device__ __forceinline__ cx<R> cfma(cx<R> a, cx<R> b, cx<R> c) {
    return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
// conj(a) b
template <typename R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
    return {fma(a.re, b.re, a.im * b.im), fma(a.re, b.im, -(a.im * b.re))};
}
// real s times complex a plus c
template <typename R>
__device__ __forceinline__ cx<R> rfma(R s, cx<R> a, cx<R> c) {
    return {fma(s, a.re, c.re), fma(s, a.im, c.im)};
}
// three-point angular stencil wp f+ + wm f- + w0 f0
template <typename R>
__device__ __forceinline__ cx<R> stencil(R wp, cx<R> fp, R wm, cx<R> fm, R w0, cx<R> f0) {
    return rfma(wp, fp, rfma(wm, fm, w0 * f0));
}

// Conversion between storage and arithmetic precision (identity when equal;
// double to float rounds to nearest).
template <typename T, typename U>
__device__ __forceinline__ cx<T> cvt(cx<U> v) { return {T(v.re), T(v.im)}; }

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

// The same store, non-temporal: the line is not kept in the caches.
template <typename R>
__device__ __forceinline__ void st_row_nt(R* __restrict__ base, int64_t row_elem, unsigned boff, cx<R> v) {
    char* p = reinterpret_cast<char*>(base + 2 * row_elem) + boff;
    typedef R v2 __attribute__((ext_vector_type(2)));
    v2 w;
    w.x = v.re;
    w.y = v.im;
    __builtin_nontemporal_store(w, reinterpret_cast<v2*>(p));
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

// 1/sqrt(x) to full precision.  The hardware estimate y is good to about
// 2^-24; with e = 1 - x y^2, 1/sqrt(x) = y (1 - e)^(-1/2) = y (1 + e/2 +
// 3 e^2/8 + ...), and the terms kept reach 2^-52.7 (measured over 2^20
// arguments, the same as two Newton steps) in five operations and a
// dependency depth of four.
__device__ __forceinline__ double rsqrt_full(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    double p = fma(0.375, e, 0.5);
    return fma(y * e, p, y);
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

// Radial numerators used by the kernels sit in LDS in table order: the
// fields R_W2 .. R_GR are the first N_RAD_USED fields of the tables.
constexpr int N_RAD_USED = 9;
static_assert(R_W2 == 0 && R_GR == N_RAD_USED - 1, "LDS radial fields are the first table fields");

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

// The forward step keeps the radial numerators R_W2 .. R_VI in LDS and the
// source's radial factor separately, per fused step and location, so that
// a moving source can be evaluated at each stage's time.
constexpr int N_RAD_FWD = 8;
static_assert(R_VI == N_RAD_FWD - 1, "forward LDS radial fields are the first table fields");

template <typename R>
__device__ __forceinline__ Rad<R> lds_rad_fwd(const R (*t)[WAVE], int lane) {
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
    r.gr = R(0);   // the forward step reads the source factor from its own slots
    return r;
}

// One LDS value of this lane through a hidden index (see lds_rad).
template <typename R>
__device__ __forceinline__ R lds_lane(const R* t, int lane) {
    int z = 0;
    asm volatile("" : "+s"(z));
    return t[lane + z];
}

// Per-wave LDS of the forward step: radial numerators at half and integer
// points, and the source's radial factor per fused step k at the
// predictor's (half point, t^{n+k}) and the corrector's (integer point,
// t^{n+k} + dt/2) location and time.
template <typename R, int KB>
struct FwdLds {
    R rad[2][N_RAD_FWD][WAVE];
    R src[KB][2][WAVE];
};

// Angular factors of one theta row (wave-uniform: scalar loads).
template <typename R>
struct Ang {
    R sin2, a2s2, cs, wp, wm, w0, agth;
};

// The angular table is read-only while kernels run: it is read through the
// constant address space, so the wave-uniform row reads are scalar loads
// whatever the compiler can prove about the pointer's origin.
template <typename R>
__device__ __forceinline__ R ang_at(const R* ang, int row, int field) {
    typedef __attribute__((address_space(4))) const R* cptr;
    return ((cptr)ang)[(int64_t)row * A_STRIDE + field];
}

template <typename R>
__device__ __forceinline__ Ang<R> load_ang(const R* ang, int row) {
    typedef __attribute__((address_space(4))) const R* cptr;
    const cptr g = (cptr)ang + (int64_t)row * A_STRIDE;
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

}  // namespace teuk
