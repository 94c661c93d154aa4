// HIP kernels of libteuk for gfx950 (MI355X): the forward time step.
//
// lw_step: KB fused two-stage Lax-Wendroff updates (paper Eqs. 13-14) of
// the first-order m-mode Teukolsky system (Eqs. 8-12), with the particle
// source and the boundary conditions (text after Eq. 14) fused in.
//
// Work decomposition.  A wavefront owns a strip of 64 consecutive r*
// columns (one per lane, r* contiguous in memory so every row load is one
// coalesced 1 KiB (FP64) access per field) and marches upwards through a
// chunk of theta rows.  Lane l holds column c = strip*(64 - 2KB) - KB + l;
// the predictor value at the half point c+1/2 needs column c+1, which comes
// from the neighbouring lane by a DPP wavefront shift; the corrector at c
// needs the half point c-1/2 from the lane below.  Each step costs one
// valid column per side, so lanes KB..63-KB produce outputs and
// neighbouring strips overlap by 2KB columns.  Along theta the three-point
// angular stencil of each stage is accumulated as a partial sum (the part
// that needs rows j-1 and j, times the stage's weight D, is added to the
// pending Pi as soon as row j is known; the row j+1 term one row later), so
// u^n is read from HBM once per row (plus 2KB halo rows per side of a chunk)
// and u^{n+KB} written once: 64 B per grid point per launch in FP64, 32 B in
// FP32 (also when FP32 storage is combined with FP64 arithmetic).
// Intermediate values never leave registers.
//
// Coefficients.  All coefficients of Eqs. (5)-(12) are separable into
// radial numerators (per-wave LDS for the lane's column) and angular
// factors (wave-uniform per row, read through the scalar cache); per point
// only Sigma^2 = w2^2 - a^2 Delta sin^2 and one reciprocal square root are
// formed.  The rsqrt starts from the hardware estimate and is refined by
// Newton steps to full precision.
#include <type_traits>

#include "teuk_device.h"

namespace teuk {

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
// The differences arrive unscaled (u_{i+1} - u_i): 1/dr* is folded into b
// (one multiply) and into CR (the radial fields CRR and WBN are scaled when
// the tile loads them, and m2ma_idr = -2 m a / dr*).
//
// The means enter as sums, with no multiply by 1/2: the predictor works
// with twice its values (s = u_i + u_{i+1}, so f = s/2) and produces twice
// the half-step values; the corrector then sees four times its means and
// twice its differences.  The stage is linear, so scaling its inputs by 2
// (predictor) or 4 (corrector) is undone by powers of two folded into
// constants: b and CR carry 2/dr* (idr = 2/dr*), the source slots hold 2T
// (predictor) and 4T (corrector), and the corrector's tau is dt/4.  Powers
// of two scale exactly in binary floating point, so every rounded result
// equals that of the form with explicit means.
template <typename R>
struct Stage {
    cx<R> phi, pi_part;
    R dw;
};

// The coefficients of a stage that depend on the point only: the same for
// every fused step at that point.
template <typename R>
struct Coef {
    R y2, bi, crr, cti;   // 1/Sigma^2, b/dr*, Re CR/dr*, Im CT
};
template <typename R>
__device__ __forceinline__ Coef<R> coef(const Rad<R>& q, const Ang<R>& g, R idr) {
    R S2 = fma(q.w2, q.w2, -g.a2s2 * q.del);   // Sigma^2
    R y = rsqrt_full(S2);                      // 1/Sigma
    Coef<R> k;
    k.y2 = y * y;
    k.bi = (q.w2 * y) * idr;                   // b / dr*, Eq. (6)
    k.crr = fma(q.wbn * g.sin2, k.y2, q.crr);
    k.cti = fma(g.cs, q.del, q.cti0);
    return k;
}

template <bool SRC, typename R>
__device__ __forceinline__ Stage<R> stage(const Coef<R>& k, const Rad<R>& q, R gr, const Ang<R>& g, R m2ma_idr,
                                          R tau, cx<R> ph, cx<R> f0, cx<R> g0, cx<R> f, cx<R> gm, cx<R> df,
                                          cx<R> dg) {
    const R y2 = k.y2, bi = k.bi;
    cx<R> X = {fma(-bi, df.re, gm.re), fma(-bi, df.im, gm.im)};        // Pi - b dPhi
    cx<R> CR = {k.crr, m2ma_idr * q.w2};                              // CR / dr*
    cx<R> CT = {q.ctr, k.cti};
    cx<R> V = {q.vr, q.vi};
    cx<R> acc = cfma(CR, df, cfma(V, f, cmul(CT, X)));
    Stage<R> o;
    o.phi = {fma(tau, X.re, f0.re), fma(tau, X.im, f0.im)};
    cx<R> rhs;
    if constexpr (SRC) {
        cx<R> T = (g.agth * gr) * ph;   // source: amp x theta Gaussian x radial factor x phase
        rhs = {fma(bi, dg.re, fma(-y2, acc.re, T.re)), fma(bi, dg.im, fma(-y2, acc.im, T.im))};
    } else {
        // a tile where T = 0 at every point: the same values up to the sign
        // of a zero
        rhs = {fma(bi, dg.re, -y2 * acc.re), fma(bi, dg.im, -y2 * acc.im)};
    }
    o.pi_part = {fma(tau, rhs.re, g0.re), fma(tau, rhs.im, g0.im)};
    o.dw = tau * q.del * y2;
    return o;
}

// State of one Lax-Wendroff step marching upwards through theta (one
// pipeline stage).  The angular term D (wp f(j+1) + wm f(j-1) + w0 f(j)) of
// each stage is formed in two parts: D times the bracket wm f(j-1) + w0 f(j)
// goes into the pending Pi as soon as row j is known, and the carried weight
// D wp multiplies f(j+1) one row later.  Only one previous row and the
// pending values of each stage are carried.
template <typename R>
struct Pipe {
    cx<R> pb_prev;  // Phi sum (twice the mean) at half point c+1/2, time n, row L-1
    cx<R> ph_prev;  // Phi sum of doubled half values (4x the mean) at c, time n+1/2, row L-2
    // Each Lax-Wendroff stage is split into its angular part, which needs the
    // next row, and the rest.  Pending (non-angular) parts:
    cx<R> hP, hQp;  // predictor of half row L-1, doubled: final Phi, Pi but for the wp term
    R hD;           // (dt/2) (Delta/Sigma^2) wp at that half row: the weight of row L
    cx<R> nQp;      // corrector of row L-2: Pi but for the wp term
    R nD;           // dt (Delta/Sigma^2) wp at that row: the weight of row L-1's half values
    cx<R> up, uq;   // input row L-1 (the u^n term of the corrector)
    int olo, ohi;   // rows [olo, ohi) whose outputs this stage produces
    int ihi;        // input rows end at ihi (they start at olo - 2, clipped at 0)
    int plo, phi;   // half rows [plo, phi] of the predictor
};

template <typename R>
__device__ __forceinline__ void pipe_init(Pipe<R>& st, int olo, int ohi, int nth) {
    const cx<R> zero = {R(0), R(0)};
    st.pb_prev = zero; st.ph_prev = zero;
    st.hP = zero; st.hQp = zero; st.hD = R(0); st.nQp = zero; st.nD = R(0);
    st.up = zero; st.uq = zero;
    st.olo = olo; st.ohi = ohi;
    st.ihi = min(ohi + 2, nth);
    st.plo = max(olo - 1, 0);
    st.phi = min(ohi, nth - 1);
}

// Wavefront-uniform constants shared by the stages.
template <typename R>
struct Consts {
    const R* ang;
    const R (*srad)[N_RAD_FWD][WAVE];
    const R (*ssrc)[2][WAVE];   // source radial factor [fused step][half/integer][lane]
    int lane, nth;
    R keep, idr, qdt, hdt, m2ma_idr;   // idr = 2/dr*, qdt = dt/4 (see stage())
};

// One iteration of a stage at its row index L with input row L = (p, q).
// Returns the stage's finished outputs: Phi at row L-1 (okP) and Pi at row
// L-2 (okQ).  The parts of the iteration sit behind wave-uniform branches,
// which also keep the scheduler from stretching live ranges.  EDGE: the
// tile holds an r* boundary column or a nonzero source value; other tiles
// skip the boundary factor (1 at every column they hold) and the source term
// (0 at every point they hold).
//
// NB: the input row's values at column c+1 arrive in (p1n, q1n), read from
// LDS by the caller, instead of by a lane shift.
template <bool EDGE, bool NB = false, int CM = 0, typename R, typename S>
__device__ __forceinline__ void pipe_iter(Pipe<R>& st, const Consts<R>& K, int ks, int L, cx<R> p, cx<R> q,
                                          cx<R> p1n, cx<R> q1n,
                                          cx<R> ph0, cx<R> ph1, S* wave, int64_t wrow, int wl, int rlo,
                                          int rhi, R alpha, cx<R>& outP, bool& okP, cx<R>& outQ, bool& okQ,
                                          Coef<R>* ch = nullptr, Coef<R>* ci = nullptr) {
    const cx<R> zero = {R(0), R(0)};
    const int P = L - 1, Q = L - 2;
    const cx<R> up = st.up, uq = st.uq;
    st.up = p;
    st.uq = q;
    // ---- A1: input row L; half-point sum and compact differences at c+1/2
    // (rows past the grid keep a zero sum: they meet only zero weights)
    cx<R> pbL = zero, Qb, dP, dQ;   // Qb, dP, dQ are read only by A2, which implies A1 ran
    if (L < st.ihi) {
        cx<R> p1 = p1n, q1 = q1n;
        if constexpr (!NB) {
            p1 = shfl_dn1(p);
            q1 = shfl_dn1(q);
        }
        pbL = p + p1;            // twice the mean (see stage())
        Qb = q + q1;
        dP = p1 - p;             // unscaled: 1/dr* is folded into the stage
        dQ = q1 - q;
        if (wrow >= 0 && L >= rlo && L < rhi) {
            if (K.lane == wl) stc(wave, wrow * K.nth + L, cvt<S>(rfma(alpha, p1, (R(1) - alpha) * p)));
        }
    }
    // ---- B1: finish the predictor (Eq. 13) of half row P and form the
    //      corrector's means and differences at c (time n+1/2)
    cx<R> phL = zero, Qh, dhP, dhQ;  // Qh, dhP, dhQ are read only by B2, whose rows are a subset
    if (P >= st.plo && P <= st.phi) {
        cx<R> hQ = rfma(st.hD, pbL, st.hQp);
        cx<R> hPm = shfl_up1(st.hP), hQm = shfl_up1(hQ);
        phL = st.hP + hPm;       // four times the mean: the half-step values are doubled
        Qh = hQ + hQm;
        dhP = st.hP - hPm;
        dhQ = hQ - hQm;
    }
    // ---- A2: non-angular part of the predictor of half row L and the
    //      bracket of its stencil
    if (L >= st.plo && L <= st.phi) {
        const Ang<R> g = load_ang(K.ang, L);
        const Rad<R> qh = lds_rad_fwd<R>(K.srad[0], K.lane);   // half point c+1/2
        const R gr = EDGE ? lds_lane(K.ssrc[ks][0], K.lane) : R(0);
        Coef<R> kc;
        if constexpr (CM == 2) kc = *ch;
        else kc = coef(qh, g, K.idr);
        if constexpr (CM == 1) *ch = kc;
        Stage<R> o = stage<EDGE>(kc, qh, gr, g, K.m2ma_idr, K.hdt, ph0, pbL, Qb, pbL, Qb, dP, dQ);
        st.hP = o.phi;
        st.hQp = rfma(o.dw, rfma(g.wm, st.pb_prev, g.w0 * pbL), o.pi_part);
        st.hD = o.dw * g.wp;
    }
    st.pb_prev = pbL;
    // ---- C: finish the corrector (Eq. 14) of row Q: its Pi
    okQ = (Q >= st.olo && Q < st.ohi);
    if (okQ) {
        outQ = rfma(st.nD, phL, st.nQp);
        if constexpr (EDGE) outQ = K.keep * outQ;
    }
    // ---- B2: non-angular part of the corrector of row P (its Phi is final)
    //      and the bracket of its stencil
    okP = (P >= st.olo && P < st.ohi);
    if (okP) {
        const Ang<R> g = load_ang(K.ang, P);
        const Rad<R> qi = lds_rad_fwd<R>(K.srad[1], K.lane);   // integer point c
        const R gr = EDGE ? lds_lane(K.ssrc[ks][1], K.lane) : R(0);
        Coef<R> kc;
        if constexpr (CM == 2) kc = *ci;
        else kc = coef(qi, g, K.idr);
        if constexpr (CM == 1) *ci = kc;
        Stage<R> o = stage<EDGE>(kc, qi, gr, g, K.m2ma_idr, K.qdt, ph1, up, uq, phL, Qh, dhP, dhQ);
        st.nQp = rfma(o.dw, rfma(g.wm, st.ph_prev, g.w0 * phL), o.pi_part);
        st.nD = o.dw * g.wp;
        outP = EDGE ? K.keep * o.phi : o.phi;
    }
    st.ph_prev = phL;
}

// The row march of one tile (see step_tile): stage k advances u^{n+k} to
// u^{n+k+1} and consumes row X of stage k-1's output once both its Phi
// (finished one iteration earlier) and its Pi are final, two rows behind.
// S is the storage type of the state and the waveform, R the arithmetic's.
template <typename S, typename R, int KB, bool EDGE, bool NT, typename P>
__device__ __forceinline__ void march(const S* __restrict__ phi, const S* __restrict__ pi,
                                      S* __restrict__ phi_out, S* __restrict__ pi_out, S* __restrict__ wave,
                                      const P& A, const Consts<R>& K, int j0, int jend, unsigned boff,
                                      unsigned soff, bool out_lane, bool rec, int wl) {
    const int nr = A.nr(), nth = A.nth();
    const cx<R> zero = {R(0), R(0)};
    // stage k produces rows [j0 - 2(KB-1-k), jend + 2(KB-1-k)), clipped
    Pipe<R> st[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k)
        pipe_init(st[k], max(j0 - 2 * (KB - 1 - k), 0), min(jend + 2 * (KB - 1 - k), nth), nth);
    const int Ls = max(st[0].olo - 2, 0);          // first input row of stage 0
    const int Le = jend - 1 + 2 * KB;             // last iteration: the last stage's C at row jend-1
    cx<R> held[KB];                               // Phi of stage k's output row L-1, kept one iteration
#pragma unroll
    for (int k = 0; k < KB; ++k) held[k] = zero;

    // input rows of stage 0 in flight two ahead: rows Ls and Ls+1 now,
    // iteration L requests row L+2 into the buffer row L came in
    const cx<S> zs = {S(0), S(0)};
    cx<S> pa_p = ld_row_once(phi, (int64_t)Ls * nr, boff), pa_q = ld_row_once(pi, (int64_t)Ls * nr, boff);
    cx<S> pb_p = zs, pb_q = zs;
    if (Ls + 1 < st[0].ihi && Ls + 1 <= Le) {
        pb_p = ld_row_once(phi, (int64_t)(Ls + 1) * nr, boff);
        pb_q = ld_row_once(pi, (int64_t)(Ls + 1) * nr, boff);
    }

    // Two fused steps in FP32: the second step at a point takes the point's
    // coefficients (Coef) from the first step, which formed them two
    // iterations earlier, through a ring of four slots (the loop is unrolled
    // four times so that no slot is copied).  The same values, so the same
    // results; 20 more VGPRs (118, still 4 waves per SIMD).  FP64 would
    // need 40 and spill.
    constexpr bool CACHE = (KB == 2) && std::is_same<R, float>::value;
    struct Ring {
        Coef<R> h, i;
    };
    Ring r0, r1, r2, r3;
    {
        const Coef<R> z = {R(0), R(0), R(0), R(0)};
        r0.h = r0.i = r1.h = r1.i = r2.h = r2.i = r3.h = r3.i = z;
    }
    // iteration L reads the slot written at L - 2 and writes its own
    auto iter = [&](int L, cx<S>& pf_p, cx<S>& pf_q, Ring& rg, Ring& nw) {
        if (L > Le) return;
        cx<R> p = cvt<R>(pf_p), q = cvt<R>(pf_q);
        if (L + 2 < st[0].ihi && L + 2 <= Le) {
            const int64_t row = (int64_t)(L + 2) * nr;
            pf_p = ld_row_once(phi, row, boff);
            pf_q = ld_row_once(pi, row, boff);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int Lk = L - 2 * k;   // stage k works two rows behind stage k-1
            cx<R> oP, oQ;
            bool okP, okQ;
            const cx<R> ph0 = A.ph(2 * k), ph1 = A.ph(2 * k + 1);
            if constexpr (!CACHE)
                pipe_iter<EDGE>(st[k], K, k, Lk, p, q, p, q, ph0, ph1, wave, rec ? A.wave_row(k) : -1, wl, j0, jend,
                                A.alpha(), oP, okP, oQ, okQ);
            else if (k == 0)
                pipe_iter<EDGE, false, 1>(st[k], K, k, Lk, p, q, p, q, ph0, ph1, wave, rec ? A.wave_row(k) : -1, wl,
                                          j0, jend, A.alpha(), oP, okP, oQ, okQ, &nw.h, &nw.i);
            else
                pipe_iter<EDGE, false, 2>(st[k], K, k, Lk, p, q, p, q, ph0, ph1, wave, rec ? A.wave_row(k) : -1, wl,
                                          j0, jend, A.alpha(), oP, okP, oQ, okQ, &rg.h, &rg.i);
            if (k == KB - 1) {
                if constexpr (NT) {
                    if (okQ && out_lane) st_row_nt(pi_out, (int64_t)(Lk - 2) * nr, soff, cvt<S>(oQ));
                    if (okP && out_lane) st_row_nt(phi_out, (int64_t)(Lk - 1) * nr, soff, cvt<S>(oP));
                } else {
                    if (okQ && out_lane) st_row(pi_out, (int64_t)(Lk - 2) * nr, soff, cvt<S>(oQ));
                    if (okP && out_lane) st_row(phi_out, (int64_t)(Lk - 1) * nr, soff, cvt<S>(oP));
                }
            } else {
                // next stage's input row Lk-2: Phi finished one iteration ago,
                // Pi finished now
                p = held[k];
                q = oQ;
                if (okP) held[k] = oP;
            }
        }
    };
    // unrolled so that the carried values alternate between register sets
    if constexpr (CACHE) {
        for (int L = Ls; L <= Le; L += 4) {
            iter(L, pa_p, pa_q, r2, r0);
            iter(L + 1, pb_p, pb_q, r3, r1);
            iter(L + 2, pa_p, pa_q, r0, r2);
            iter(L + 3, pb_p, pb_q, r1, r3);
        }
    } else {
        for (int L = Ls; L <= Le; L += 2) {
            iter(L, pa_p, pa_q, r0, r0);
            iter(L + 1, pb_p, pb_q, r1, r1);
        }
    }
}

// The tile's share of the coefficient tables, into its wavefront's LDS
// slice (see step_tile).  src_here: a column of this lane meets a nonzero
// source value.
template <typename R, int KB, typename P>
__device__ __forceinline__ void tile_tables(const R* __restrict__ rad_i, const R* __restrict__ rad_h, const P& A,
                                            int strip, FwdLds<R, KB>* lds, bool& src_here) {
    constexpr int SO = WAVE - 2 * KB;   // valid output columns per strip
    const int lane = threadIdx.x & (WAVE - 1);
    const int nr = A.nr();
    const int c = strip * SO - KB + lane;
    // Lanes outside the grid read a clamped column: they feed only the
    // half points beyond the r* boundaries, whose outputs are the Dirichlet
    // zeros or are never stored.
    const unsigned cu = (unsigned)min(max(c, 0), nr - 1);
    // radial numerators of this wavefront's columns (CRR and WBN, which
    // multiply r* differences only, carry the 1/dr* of those differences)
    const R idr = R(2) * A.inv_dr();   // 2/dr*: the stage sees doubled differences (see stage())
    R (*srad)[N_RAD_FWD][WAVE] = lds->rad;
    for (int k = 0; k < 2 * N_RAD_FWD; ++k) {
        const int loc = k / N_RAD_FWD, f = k % N_RAD_FWD;
        const R v = (loc == 0 ? rad_h : rad_i)[(int64_t)f * A.stride() + cu];
        srad[loc][f][lane] = (f == R_CRR || f == R_WBN) ? v * idr : v;
    }
    // source radial factor of each fused step at its predictor (half point,
    // t^{n+k}) and corrector (integer point, t^{n+k} + dt/2): the table's
    // for a fixed orbit, exp(-(r* - r*0(t))^2 / (2 sr^2)) for a moving one
    src_here = false;
#pragma unroll
    for (int k = 0; k < KB; ++k)
        for (int loc = 0; loc < 2; ++loc) {
            R v;
            if (A.moving()) {
                const R x = fma((R)c + (loc == 0 ? R(0.5) : R(0)), A.dr(), A.rmin()) - A.rs0(2 * k + loc);
                v = exp((-x * x) / A.two_sr2());
            } else {
                v = (loc == 0 ? rad_h : rad_i)[(int64_t)R_GR * A.stride() + cu];
            }
            lds->src[k][loc][lane] = v * (loc == 0 ? R(2) : R(4));   // 2T predictor, 4T corrector
            src_here = src_here || (v != R(0) && c >= 0 && c < nr);
        }
}

// The stage constants of a tile whose tables sit in `lds`; c is the lane's
// column.
template <typename R, int KB, typename P>
__device__ __forceinline__ Consts<R> tile_consts(const R* __restrict__ ang, const P& A, FwdLds<R, KB>* lds,
                                                 int lane, int c) {
    const int nr = A.nr();
    const R idr = R(2) * A.inv_dr();   // 2/dr* (see stage())
    Consts<R> K;
    K.ang = ang;
    K.srad = lds->rad;
    K.ssrc = lds->src;
    K.lane = lane;
    K.nth = A.nth();
    K.keep = ((c == 0) || (c == nr - 1)) ? R(0) : R(1);   // Phi = Pi = 0 on the r* boundary
    K.idr = idr;
    K.qdt = R(0.25) * A.dt();
    K.hdt = A.hdt();
    K.m2ma_idr = A.m2ma() * idr;
    return K;
}

// KB Lax-Wendroff steps over one tile (one wavefront's strip of r* columns
// and its chunk of theta rows), the work unit of both the single-mode and
// the batched kernel.  The intermediate states never leave registers.  Each
// stage's arithmetic per point is the same code as for KB = 1, so results
// are bitwise identical to KB single steps whatever the tiling or batching.
// A strip loses one valid column per side and a chunk needs two more halo
// rows per side for each extra stage.  `lds` is this wavefront's own slice
// (no barrier).  S: storage type of the state; R: arithmetic type (FP32
// storage with FP64 arithmetic converts on load and store).
template <typename S, typename R, int KB, bool NT = false, typename P>
__device__ __forceinline__ void step_tile(const S* __restrict__ phi, const S* __restrict__ pi,
                                          S* __restrict__ phi_out, S* __restrict__ pi_out,
                                          const R* __restrict__ rad_i, const R* __restrict__ rad_h,
                                          const R* __restrict__ ang, S* __restrict__ wave, const P& A,
                                          int strip, int chunk, FwdLds<R, KB>* lds) {
    constexpr int SO = WAVE - 2 * KB;   // valid output columns per strip
    const int lane = threadIdx.x & (WAVE - 1);
    const int nr = A.nr(), nth = A.nth();
    const int c = strip * SO - KB + lane;
    const unsigned cu = (unsigned)min(max(c, 0), nr - 1);
    bool src_here;
    tile_tables<R, KB>(rad_i, rad_h, A, strip, lds, src_here);
    const int j0 = chunk * A.rows();
    const int jend = min(j0 + A.rows(), nth);
    const bool out_lane = (c >= 0) && (c < nr) && lane >= KB && lane <= WAVE - 1 - KB;
    const unsigned boff = cu * (unsigned)(2 * sizeof(S));          // byte offset of this lane's column
    const unsigned soff = (unsigned)max(c, 0) * (unsigned)(2 * sizeof(S));
    const Consts<R> K = tile_consts<R, KB>(ang, A, lds, lane, c);
    // recorder: the strip holding columns iobs and iobs+1 among its lanes
    const bool rec = (A.iobs() / SO == strip);
    const int wl = A.iobs() - strip * SO + KB;
    // Tiles with an r* boundary column or a nonzero source value take the
    // general code; all others skip the boundary factor and the source term.
    const bool edge = __ballot(K.keep == R(0) || src_here) != 0;
    if (edge)
        march<S, R, KB, true, NT>(phi, pi, phi_out, pi_out, wave, A, K, j0, jend, boff, soff, out_lane, rec, wl);
    else
        march<S, R, KB, false, NT>(phi, pi, phi_out, pi_out, wave, A, K, j0, jend, boff, soff, out_lane, rec, wl);
}

// Per-tile constants of the single-mode kernel: its kernel argument (the
// compiler reloads kernel arguments where that frees registers).
template <typename R>
struct ArgParams {
    const StepArgs<R>& A;
    __device__ int nr() const { return A.nr; }
    __device__ int nth() const { return A.nth; }
    __device__ int rows() const { return A.rows; }
    __device__ int64_t stride() const { return A.stride; }
    __device__ int iobs() const { return A.iobs; }
    __device__ R dt() const { return A.dt; }
    __device__ R hdt() const { return A.hdt; }
    __device__ R inv_dr() const { return A.inv_dr; }
    __device__ R m2ma() const { return A.m2ma; }
    __device__ R alpha() const { return A.alpha; }
    __device__ cx<R> ph(int i) const { return {A.ph[i][0], A.ph[i][1]}; }
    __device__ int64_t wave_row(int k) const { return A.wave_row[k]; }
    __device__ bool moving() const { return A.moving != 0; }
    __device__ R rs0(int i) const { return A.rs0[i]; }
    __device__ R two_sr2() const { return A.two_sr2; }
    __device__ R rmin() const { return A.rmin; }
    __device__ R dr() const { return A.dr; }
};

// Single-mode launch: one tile per wavefront, WG_WAVES adjacent strips of
// the same theta chunk per workgroup.  S: storage type of the state and the
// waveform; R: arithmetic type.  The FP64 body fits 3 waves per SIMD (168
// VGPRs); the hint keeps the allocator there.
template <typename S, typename R, int KB, bool NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void lw_step_kernel(
    const S* __restrict__ phi, const S* __restrict__ pi, S* __restrict__ phi_out, S* __restrict__ pi_out,
    const R* __restrict__ rad_i, const R* __restrict__ rad_h, const R* __restrict__ ang, S* __restrict__ wave,
    StepArgs<R> A) {
    // wave-uniform quantities: keep them in scalar registers
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    // Every row access of a workgroup is one contiguous 4 KiB (FP64) span.
    // Block order (a tuning choice): chunk-major lets the groups that run
    // together touch neighbouring columns of the same rows; group-major
    // keeps a strip group's chunks together so their halo rows are served
    // by L2.  Blocks take tiles in dispatch order, which deals consecutive
    // blocks to the 8 XCDs in turn: all XCDs then stream the same rows,
    // and the partial last chunk's cheap tiles come last.  Giving each XCD
    // a contiguous range of tiles instead measured the same on 32768 x 1024
    // and up to 17 % slower on 8192 x 256 at small chunks.
    const int ngrp = (A.n_strips + WG_WAVES - 1) / WG_WAVES;
    const int blk = (int)blockIdx.x;
    int chunk, grp;
    if (A.order == 0) {  // chunk-major: concurrent groups read the same rows
        chunk = blk / ngrp;
        grp = blk - chunk * ngrp;
    } else {             // group-major: adjacent chunks share their halo rows in L2
        grp = blk / A.n_chunks;
        chunk = blk - grp * A.n_chunks;
    }
    const int strip = grp * WG_WAVES + wid;
    if (strip >= A.n_strips) return;  // wave-uniform; the kernel has no barriers
    __shared__ FwdLds<R, KB> lds_all[WG_WAVES];   // one slice per wavefront
    const ArgParams<R> P{A};
    step_tile<S, R, KB, NT>(phi, pi, phi_out, pi_out, rad_i, rad_h, ang, wave, P, strip, chunk, &lds_all[wid]);
}


// Two fused steps on a pair of wavefronts.  The single-wave tile above keeps
// both steps' pipelines in one wavefront's registers (3 waves per SIMD in
// FP64).  Here a workgroup of two wavefronts takes one strip and one theta
// chunk: wave 0 runs the first step's pipeline over the rows of u^n read
// from HBM, wave 1 the second step's over the rows of u^{n+1} that wave 0
// hands over through an LDS ring, and writes u^{n+2}.  Each wave carries one
// pipeline, and the two share the strip's radial tables.  The arithmetic per
// point is step_tile's (the same stage code), so results are bitwise
// identical to it and to single steps.
//
// Wave 0 finishes Phi of row L-1 and Pi of row L-2 at its iteration L and
// puts them in ring slot (row & 3).  Wave 1 takes row L-3 at iteration L, so
// a row is complete one iteration before it is read; both waves meet at one
// barrier per iteration, and a slot is rewritten only after two more
// barriers.  Wave 1 reads column c+1 of its input row from the ring instead
// of shifting lanes.
constexpr int RING = 4;

template <typename R>
struct SplitLds {
    R rad[2][N_RAD_FWD][WAVE];
    R src[2][2][WAVE];
    cx<R> ring[RING][2][WAVE + 1];   // [slot][Phi, Pi][lane]; lane 64 feeds only lane 63
};

// LDS barrier of the pair: LDS and scalar operations complete, then s_barrier.
// Vector memory is not waited for (the pair shares no global data).
__device__ __forceinline__ void pair_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <typename S, typename R, bool EDGE, typename P>
__device__ __forceinline__ void split_march(const S* __restrict__ phi, const S* __restrict__ pi,
                                            S* __restrict__ phi_out, S* __restrict__ pi_out, S* __restrict__ wave,
                                            const P& A, const Consts<R>& K, SplitLds<R>* lds, int wid, int j0,
                                            int jend, unsigned boff, unsigned soff, bool out_lane, bool rec,
                                            int wl) {
    const int nr = A.nr(), nth = A.nth();
    const int Ls = max(j0 - 4, 0);     // first input row of the first step
    const int Le = jend + 3;           // the second step's C at row jend-1 comes at L = Le + 1
    const int lane = K.lane;
    if (wid == 0) {
        Pipe<R> st;
        pipe_init(st, max(j0 - 2, 0), min(jend + 2, nth), nth);
        const cx<R> ph0 = A.ph(0), ph1 = A.ph(1);
        const int64_t wrow = rec ? A.wave_row(0) : -1;
        const cx<S> zs = {S(0), S(0)};
        cx<S> pa_p = ld_row_once(phi, (int64_t)Ls * nr, boff), pa_q = ld_row_once(pi, (int64_t)Ls * nr, boff);
        cx<S> pb_p = zs, pb_q = zs;
        if (Ls + 1 < st.ihi) {
            pb_p = ld_row_once(phi, (int64_t)(Ls + 1) * nr, boff);
            pb_q = ld_row_once(pi, (int64_t)(Ls + 1) * nr, boff);
        }
        auto it = [&](int L, cx<S>& pf_p, cx<S>& pf_q) {
            cx<R> p = cvt<R>(pf_p), q = cvt<R>(pf_q);
            if (L + 2 < st.ihi) {
                const int64_t row = (int64_t)(L + 2) * nr;
                pf_p = ld_row_once(phi, row, boff);
                pf_q = ld_row_once(pi, row, boff);
            }
            __builtin_amdgcn_sched_barrier(0);
            cx<R> oP, oQ;
            bool okP, okQ;
            pipe_iter<EDGE>(st, K, 0, L, p, q, p, q, ph0, ph1, wave, wrow, wl, j0, jend, A.alpha(), oP, okP, oQ,
                            okQ);
            if (okP) lds->ring[(L - 1) & (RING - 1)][0][lane] = oP;
            if (okQ) lds->ring[(L - 2) & (RING - 1)][1][lane] = oQ;
            pair_barrier();
        };
        int L = Ls;
        for (; L + 1 <= Le + 1; L += 2) {
            it(L, pa_p, pa_q);
            it(L + 1, pb_p, pb_q);
        }
        if (L <= Le + 1) it(L, pa_p, pa_q);
    } else {
        Pipe<R> st;
        pipe_init(st, j0, jend, nth);
        const cx<R> ph0 = A.ph(2), ph1 = A.ph(3);
        const int64_t wrow = rec ? A.wave_row(1) : -1;
        for (int L = Ls; L <= Le + 1; ++L) {
            const int X = L - 3;     // this step's input row
            const int slot = X & (RING - 1);
            const cx<R> p = lds->ring[slot][0][lane], q = lds->ring[slot][1][lane];
            const cx<R> p1 = lds->ring[slot][0][lane + 1], q1 = lds->ring[slot][1][lane + 1];
            cx<R> oP, oQ;
            bool okP, okQ;
            pipe_iter<EDGE, true>(st, K, 1, X, p, q, p1, q1, ph0, ph1, wave, wrow, wl, j0, jend, A.alpha(), oP, okP,
                                  oQ, okQ);
            if (okQ && out_lane) st_row(pi_out, (int64_t)(X - 2) * nr, soff, cvt<S>(oQ));
            if (okP && out_lane) st_row(phi_out, (int64_t)(X - 1) * nr, soff, cvt<S>(oP));
            pair_barrier();
        }
    }
}

// Grid: one workgroup (two wavefronts) per tile, tiles chunk-major in
// dispatch order (consecutive tiles go to the 8 XCDs in turn, as in
// lw_step_kernel).  One contiguous tile range per XCD measured 26 % slower
// for FP64 on 32768 x 1024 (0.657 against 0.485 ms per launch at 64 rows)
// and within 3 % either way for FP32.  4 pairs per SIMD need at most 128
// VGPRs.
template <typename S, typename R>
__global__ __launch_bounds__(2 * WAVE) __attribute__((amdgpu_waves_per_eu(4))) void lw_step_split_kernel(
    const S* __restrict__ phi, const S* __restrict__ pi, S* __restrict__ phi_out, S* __restrict__ pi_out,
    const R* __restrict__ rad_i, const R* __restrict__ rad_h, const R* __restrict__ ang, S* __restrict__ wave,
    StepArgs<R> A) {
    constexpr int KB = 2, SO = WAVE - 2 * KB;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int lane = threadIdx.x & (WAVE - 1);
    const int tile = (int)blockIdx.x;
    const int chunk = tile / A.n_strips, strip = tile - chunk * A.n_strips;
    __shared__ SplitLds<R> lds;
    const ArgParams<R> P{A};
    const int nr = P.nr(), nth = P.nth();
    const int c = strip * SO - KB + lane;
    const unsigned cu = (unsigned)min(max(c, 0), nr - 1);
    const R idr = R(2) * P.inv_dr();
    // the strip's radial numerators: each wave writes half of the fields
    for (int k = wid; k < 2 * N_RAD_FWD; k += 2) {
        const int loc = k / N_RAD_FWD, f = k % N_RAD_FWD;
        const R v = (loc == 0 ? rad_h : rad_i)[(int64_t)f * P.stride() + cu];
        lds.rad[loc][f][lane] = (f == R_CRR || f == R_WBN) ? v * idr : v;
    }
    // source radial factors of both steps (each wave its own step's), and
    // whether any column of the strip meets the source (both waves alike)
    bool src_here = false;
#pragma unroll
    for (int k = 0; k < KB; ++k)
        for (int loc = 0; loc < 2; ++loc) {
            R v;
            if (P.moving()) {
                const R x = fma((R)c + (loc == 0 ? R(0.5) : R(0)), P.dr(), P.rmin()) - P.rs0(2 * k + loc);
                v = exp((-x * x) / P.two_sr2());
            } else {
                v = (loc == 0 ? rad_h : rad_i)[(int64_t)R_GR * P.stride() + cu];
            }
            if (k == wid) lds.src[k][loc][lane] = v * (loc == 0 ? R(2) : R(4));
            src_here = src_here || (v != R(0) && c >= 0 && c < nr);
        }
    // The ring starts at zero: wave 1's pipeline reads rows before the first
    // one wave 0 hands over (their values meet only zero weights, as the
    // zero-initialised carried rows of the single-wave tile do).
    {
        const cx<R> zero = {R(0), R(0)};
        for (int k = 0; k < RING; ++k) {
            lds.ring[k][wid][lane] = zero;
            if (lane == 0) lds.ring[k][wid][WAVE] = zero;
        }
    }
    pair_barrier();
    const int j0 = chunk * P.rows();
    const int jend = min(j0 + P.rows(), nth);
    const bool out_lane = (c >= 0) && (c < nr) && lane >= KB && lane <= WAVE - 1 - KB;
    const unsigned boff = cu * (unsigned)(2 * sizeof(S));
    const unsigned soff = (unsigned)max(c, 0) * (unsigned)(2 * sizeof(S));
    Consts<R> K;
    K.ang = ang;
    K.srad = lds.rad;
    K.ssrc = lds.src;
    K.lane = lane;
    K.nth = nth;
    K.keep = ((c == 0) || (c == nr - 1)) ? R(0) : R(1);
    K.idr = idr;
    K.qdt = R(0.25) * P.dt();
    K.hdt = P.hdt();
    K.m2ma_idr = P.m2ma() * idr;
    const bool rec = (P.iobs() / SO == strip);
    const int wl = P.iobs() - strip * SO + KB;
    const bool edge = __ballot(K.keep == R(0) || src_here) != 0;
    if (edge)
        split_march<S, R, true>(phi, pi, phi_out, pi_out, wave, P, K, &lds, wid, j0, jend, boff, soff, out_lane, rec,
                                wl);
    else
        split_march<S, R, false>(phi, pi, phi_out, pi_out, wave, P, K, &lds, wid, j0, jend, boff, soff, out_lane,
                                 rec, wl);
}

// S: storage type; the state and waveform pointers of `a` point to S.
template <typename S, typename R>
static void launch_step(const StepArgs<R>& a, hipStream_t s) {
    int blocks = ((a.n_strips + WG_WAVES - 1) / WG_WAVES) * a.n_chunks;
    const S* phi = reinterpret_cast<const S*>(a.phi);
    const S* pi = reinterpret_cast<const S*>(a.pi);
    S* phi_out = reinterpret_cast<S*>(a.phi_out);
    S* pi_out = reinterpret_cast<S*>(a.pi_out);
    S* wave = reinterpret_cast<S*>(a.wave);
    if (a.kb == 2 && a.split)
        hipLaunchKernelGGL((lw_step_split_kernel<S, R>), dim3(a.n_strips * a.n_chunks), dim3(2 * WAVE), 0, s, phi, pi,
                           phi_out, pi_out, a.rad_i, a.rad_h, a.ang, wave, a);
    else if (a.kb == 2) {
        // FP64 states too large to stay in the last-level cache: the build
        // with non-temporal output stores (FP32 gained nothing from it)
        if constexpr (std::is_same<S, double>::value && std::is_same<R, double>::value) {
            if (a.stream_out) {
                hipLaunchKernelGGL((lw_step_kernel<S, R, 2, true>), dim3(blocks), dim3(WAVE * WG_WAVES), 0, s, phi,
                                   pi, phi_out, pi_out, a.rad_i, a.rad_h, a.ang, wave, a);
                return;
            }
        }
        hipLaunchKernelGGL((lw_step_kernel<S, R, 2, false>), dim3(blocks), dim3(WAVE * WG_WAVES), 0, s, phi, pi,
                           phi_out, pi_out, a.rad_i, a.rad_h, a.ang, wave, a);
    } else {
        hipLaunchKernelGGL((lw_step_kernel<S, R, 1, false>), dim3(blocks), dim3(WAVE * WG_WAVES), 0, s, phi, pi,
                           phi_out, pi_out, a.rad_i, a.rad_h, a.ang, wave, a);
    }
}
void launch_step_fp64(const StepArgs<double>& a, hipStream_t s) { launch_step<double>(a, s); }
void launch_step_fp32(const StepArgs<float>& a, hipStream_t s) { launch_step<float>(a, s); }
void launch_step_fp32s(const StepArgs<double>& a, hipStream_t s) { launch_step<float>(a, s); }

// Parameter gradients: the contraction of the adjoint state lambda^{k+1}
// with the difference of two forward steps of u^k, one under coefficients
// built at p + h and one at p - h,
//   Re sum conj(lambda) (step_{p+h}(u) - step_{p-h}(u))   over Phi and Pi,
// without writing the two stepped states.  A tile runs both steps on the
// same input rows (two stage pipelines, each with its own tables, one step
// each) and adds lambda times the difference of their outputs.  The
// differences are those of the step kernel's outputs bit for bit; the sum
// runs over lanes, then tiles, in fixed orders.
template <bool EDGE>
__device__ __forceinline__ void march_pdot(const double* __restrict__ phi, const double* __restrict__ pi,
                                           const double* __restrict__ lp, const double* __restrict__ lq,
                                           const ArgParams<double>& Ap, const ArgParams<double>& Am,
                                           const Consts<double>& Kp, const Consts<double>& Km, int j0, int jend,
                                           unsigned boff, bool out_lane, double& acc) {
    const int nr = Ap.nr(), nth = Ap.nth();
    const cx<double> zero = {0.0, 0.0};
    Pipe<double> sp, sm;
    pipe_init(sp, j0, jend, nth);
    pipe_init(sm, j0, jend, nth);
    const int Ls = max(sp.olo - 2, 0);   // first input row
    const int Le = jend + 1;             // last iteration: C of row jend - 1
    // Input rows and the lambda rows of an iteration's outputs (Pi at row
    // L - 2, Phi at row L - 1) are in flight two iterations ahead, in the
    // buffer set of the iteration's parity.
    struct Rows {
        cx<double> p, q, lq, lp;
    };
    auto request = [&](int L, Rows& b) {
        b.p = b.q = b.lq = b.lp = zero;
        if (L < sp.ihi) {
            b.p = ld_row_once(phi, (int64_t)L * nr, boff);
            b.q = ld_row_once(pi, (int64_t)L * nr, boff);
        }
        if (L - 2 >= sp.olo && L - 2 < sp.ohi) b.lq = ld_row_once(lq, (int64_t)(L - 2) * nr, boff);
        if (L - 1 >= sp.olo && L - 1 < sp.ohi) b.lp = ld_row_once(lp, (int64_t)(L - 1) * nr, boff);
    };
    Rows ra, rb;
    request(Ls, ra);
    if (Ls + 1 <= Le) request(Ls + 1, rb);
    double* const nowave = nullptr;
    auto iter = [&](int L, Rows& b) {
        if (L > Le) return;
        const Rows cur = b;
        if (L + 2 <= Le) request(L + 2, b);
        __builtin_amdgcn_sched_barrier(0);
        cx<double> oPp, oQp, oPm, oQm;
        bool okP, okQ, okPm, okQm;
        pipe_iter<EDGE>(sp, Kp, 0, L, cur.p, cur.q, cur.p, cur.q, Ap.ph(0), Ap.ph(1), nowave, -1, 0, j0, jend, 0.0,
                        oPp, okP, oQp, okQ);
        pipe_iter<EDGE>(sm, Km, 0, L, cur.p, cur.q, cur.p, cur.q, Am.ph(0), Am.ph(1), nowave, -1, 0, j0, jend, 0.0,
                        oPm, okPm, oQm, okQm);
        // Re conj(l) d = l.re d.re + l.im d.im
        if (okQ && out_lane) {
            acc = fma(cur.lq.re, oQp.re - oQm.re, acc);
            acc = fma(cur.lq.im, oQp.im - oQm.im, acc);
        }
        if (okP && out_lane) {
            acc = fma(cur.lp.re, oPp.re - oPm.re, acc);
            acc = fma(cur.lp.im, oPp.im - oPm.im, acc);
        }
    };
    for (int L = Ls; L <= Le; L += 2) {
        iter(L, ra);
        iter(L + 1, rb);
    }
}

// One wavefront per tile, four adjacent strips of one theta chunk per
// workgroup (chunk-major, as lw_step_kernel's order 0); one step per tile.
// part[chunk * n_strips + strip] receives the tile's sum.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void lw_pdot_kernel(
    const double* __restrict__ phi, const double* __restrict__ pi, PdotArgs B) {
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const StepArgs<double>& A = B.s[0];
    const int ngrp = (A.n_strips + WG_WAVES - 1) / WG_WAVES;
    const int blk = (int)blockIdx.x;   // dispatch order, as lw_step_kernel
    const int chunk = blk / ngrp;
    const int strip = (blk - chunk * ngrp) * WG_WAVES + wid;
    if (strip >= A.n_strips) return;   // wave-uniform; the kernel has no barriers
    __shared__ FwdLds<double, 1> lds_all[WG_WAVES][2];   // the + and - tables of each wavefront
    const ArgParams<double> Ap{B.s[0]}, Am{B.s[1]};
    const int lane = threadIdx.x & (WAVE - 1);
    const int nr = A.nr, nth = A.nth;
    const int c = strip * (WAVE - 2) - 1 + lane;
    const unsigned cu = (unsigned)min(max(c, 0), nr - 1);
    bool src_p, src_m;
    tile_tables<double, 1>(B.s[0].rad_i, B.s[0].rad_h, Ap, strip, &lds_all[wid][0], src_p);
    tile_tables<double, 1>(B.s[1].rad_i, B.s[1].rad_h, Am, strip, &lds_all[wid][1], src_m);
    const int j0 = chunk * A.rows;
    const int jend = min(j0 + A.rows, nth);
    const bool out_lane = (c >= 0) && (c < nr) && lane >= 1 && lane <= WAVE - 2;
    const unsigned boff = cu * 16u;
    const Consts<double> Kp = tile_consts<double, 1>(B.s[0].ang, Ap, &lds_all[wid][0], lane, c);
    const Consts<double> Km = tile_consts<double, 1>(B.s[1].ang, Am, &lds_all[wid][1], lane, c);
    const bool edge = __ballot(Kp.keep == 0.0 || src_p || src_m) != 0;
    double acc = 0.0;
    if (edge)
        march_pdot<true>(phi, pi, B.lp, B.lq, Ap, Am, Kp, Km, j0, jend, boff, out_lane, acc);
    else
        march_pdot<false>(phi, pi, B.lp, B.lq, Ap, Am, Kp, Km, j0, jend, boff, out_lane, acc);
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, WAVE);
    if (lane == 0) B.part[(int64_t)chunk * A.n_strips + strip] = acc;
}

// Sums of the tiles' parts in a fixed order: workgroup b adds the n parts
// at part + b n into out[b].
__global__ __launch_bounds__(256) void pdot_sum_kernel(const double* __restrict__ part, int64_t n,
                                                       double* __restrict__ out) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    part += (int64_t)blockIdx.x * n;
    double s = 0.0;
    for (int64_t i = t; i < n; i += 256) s += part[i];
    red[t] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) out[blockIdx.x] = red[0];
}

int64_t pdot_parts(const StepArgs<double>& a) { return (int64_t)a.n_strips * a.n_chunks; }

void sweep_blocks_per_cu(int* pdot, int* step1) {
    int n = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, lw_pdot_kernel, WAVE * WG_WAVES, 0);
    *pdot = (e == hipSuccess && n > 0) ? n : 1;
    n = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, lw_step_kernel<double, double, 1, false>, WAVE * WG_WAVES, 0);
    *step1 = (e == hipSuccess && n > 0) ? n : 1;
}

void launch_param_pdot(const PdotArgs& b, const double* phi, const double* pi, hipStream_t s) {
    const StepArgs<double>& a = b.s[0];
    const int blocks = ((a.n_strips + WG_WAVES - 1) / WG_WAVES) * a.n_chunks;
    hipLaunchKernelGGL(lw_pdot_kernel, dim3(blocks), dim3(WAVE * WG_WAVES), 0, s, phi, pi, b);
}

void launch_pdot_sums(const double* part, int64_t n_parts, int64_t n_steps, double* out, hipStream_t s) {
    if (n_steps > 0)
        hipLaunchKernelGGL(pdot_sum_kernel, dim3((unsigned)n_steps), dim3(256), 0, s, part, n_parts, out);
}

// Batched launches: every instance of a batch advances kb steps in one
// launch.  Tiles are numbered instance by instance; the step and the
// current pair are the batch's device clock plus the launch's offsets, so a
// captured graph of launches followed by one clock advance replays
// correctly.  Each tile runs step_tile, so batched
// results are bitwise identical to single-mode runs.  Descriptors and clock
// are read-only during a launch and are read through the constant address
// space (wave-uniform scalar loads).
typedef __attribute__((address_space(4))) const BatchInst* cinst;
typedef __attribute__((address_space(4))) const BatchClock* cclock;
typedef __attribute__((address_space(4))) const double* cdbl;

// Per-tile constants of a batched launch, read from the instance's
// descriptor, phase table and the clock (constant memory: reloaded where
// that frees registers).
template <bool MOV>
struct InstParams {
    cinst I;
    cclock clk;
    int record;
    int step_off;
    __device__ int nr() const { return I->nr; }
    __device__ int nth() const { return I->nth; }
    __device__ int rows() const { return I->rows; }
    __device__ int64_t stride() const { return I->stride; }
    __device__ int iobs() const { return I->iobs; }
    __device__ double dt() const { return I->dt; }
    __device__ double hdt() const { return I->hdt; }
    __device__ double inv_dr() const { return I->inv_dr; }
    __device__ double m2ma() const { return I->m2ma; }
    __device__ double alpha() const { return I->alpha; }
    // i = 2 q + (0: t, 1: t + dt/2) for fused step q
    __device__ cx<double> ph(int i) const {
        const cdbl p = (cdbl)I->phase + 4 * (clk->step + step_off + (i >> 1)) + 2 * (i & 1);
        return {p[0], p[1]};
    }
    __device__ int64_t wave_row(int q) const {
        const int64_t row = clk->step + step_off + q;
        return (record && I->wave != nullptr && row < I->wave_cap) ? row : -1;
    }
    // moving source (compiled in only for batches that have one): i as for ph
    __device__ bool moving() const { return MOV && I->rs0tab != nullptr; }
    __device__ double rs0(int i) const { return I->rs0tab[2 * (clk->step + step_off + (i >> 1)) + (i & 1)]; }
    __device__ double two_sr2() const { return I->two_sr2; }
    __device__ double rmin() const { return I->rmin; }
    __device__ double dr() const { return I->dr; }
};

template <int KB, bool MOV>
__device__ __forceinline__ void batch_tile(cinst I, cclock clk, int t, int wid, const BatchArgs& B,
                                           FwdLds<double, KB>* lds) {
    constexpr int SO = WAVE - 2 * KB;
    const InstParams<MOV> P{I, clk, B.record, B.step_off};
    const int src = (int)((clk->launches + B.launch_off) & 1);
    const int n_strips = (I->nr + SO - 1) / SO;
    const int ngrp = (n_strips + WG_WAVES - 1) / WG_WAVES;
    const int local = t - I->first_tile[KB - 1];
    const int chunk = local / ngrp;
    const int strip = (local - chunk * ngrp) * WG_WAVES + wid;
    if (strip < n_strips)
        step_tile<double, double, KB>(I->buf[src][0], I->buf[src][1], I->buf[1 - src][0], I->buf[1 - src][1], I->rad_i,
                              I->rad_h, I->ang, I->wave, P, strip, chunk, lds);
}

// Persistent form: the grid holds as many workgroups as stay resident and
// the 8 XCDs each walk a contiguous range of the tile list, so strips that
// share halo columns and rows stay in one L2.  MOV: the batch has instances
// with a moving source (a separate build, so fixed-orbit batches keep the
// registers of the kernel without it).
template <int KB, bool MOV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void lw_batch_kernel(BatchArgs B) {
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    __shared__ FwdLds<double, KB> lds_all[WG_WAVES];
    const cinst insts = (cinst)B.inst;
    const cclock clk = (cclock)B.clock;
    const int X = 8;
    const int x = blockIdx.x % X, kx = blockIdx.x / X, nbx = gridDim.x / X;
    const int t_lo = (int)((int64_t)B.n_tiles * x / X), t_hi = (int)((int64_t)B.n_tiles * (x + 1) / X);
    int i = 0;
    for (int t = t_lo + kx; t < t_hi; t += nbx) {
        while (i + 1 < B.n_inst && insts[i + 1].first_tile[KB - 1] <= t) ++i;
        batch_tile<KB, MOV>(insts + i, clk, t, wid, B, &lds_all[wid]);
    }
}

// Grid form: one workgroup per tile (XCD-aware order); the instance is
// found by bisection over the tiles' prefix.
template <int KB, bool MOV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void lw_batch_grid_kernel(BatchArgs B) {
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    __shared__ FwdLds<double, KB> lds_all[WG_WAVES];
    const cinst insts = (cinst)B.inst;
    const cclock clk = (cclock)B.clock;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    int lo = 0, hi = B.n_inst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (insts[mid].first_tile[KB - 1] <= t) lo = mid;
        else hi = mid - 1;
    }
    batch_tile<KB, MOV>(insts + lo, clk, t, wid, B, &lds_all[wid]);
}

// Resident workgroups per CU of the persistent kernel, per kb and form
// (index 2 (kb - 1) + moving).
int batch_blocks_per_cu(int kb, bool moving) {
    int n = 0;
    auto k = kb == 2 ? (moving ? lw_batch_kernel<2, true> : lw_batch_kernel<2, false>)
                     : (moving ? lw_batch_kernel<1, true> : lw_batch_kernel<1, false>);
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, WAVE * WG_WAVES, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

void launch_batch_step(const BatchArgs& a, int blocks, hipStream_t s) {
    const bool mv = a.moving != 0;
    if (a.persistent) {
        auto k = a.kb == 2 ? (mv ? lw_batch_kernel<2, true> : lw_batch_kernel<2, false>)
                           : (mv ? lw_batch_kernel<1, true> : lw_batch_kernel<1, false>);
        hipLaunchKernelGGL(k, dim3(blocks), dim3(WAVE * WG_WAVES), 0, s, a);
    } else {
        auto k = a.kb == 2 ? (mv ? lw_batch_grid_kernel<2, true> : lw_batch_grid_kernel<2, false>)
                           : (mv ? lw_batch_grid_kernel<1, true> : lw_batch_grid_kernel<1, false>);
        hipLaunchKernelGGL(k, dim3(a.n_tiles), dim3(WAVE * WG_WAVES), 0, s, a);
    }
}

// The clock advances after a run of batched launches (one lane, vector store).
__global__ void batch_advance_kernel(BatchClock* clock, int steps, int launches) {
    if (threadIdx.x == 0) {
        clock->step += steps;
        clock->launches += launches;
    }
}
void launch_batch_advance(BatchClock* clock, int steps, int launches, hipStream_t s) {
    hipLaunchKernelGGL(batch_advance_kernel, dim3(1), dim3(64), 0, s, clock, steps, launches);
}

// Waveform row of the current state of every recording instance (the row
// of the step the clock shows), as the single-mode extract does.
__global__ void batch_extract_kernel(const BatchInst* __restrict__ inst, const BatchClock* __restrict__ clock) {
    const BatchInst* I = &inst[blockIdx.y];
    const int64_t row = clock->step;
    const int src = (int)(clock->launches & 1);
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (I->wave == nullptr || row >= I->wave_cap || j >= I->nth) return;
    const double* phi = I->buf[src][0];
    cx<double> p0 = ldc(phi, (int64_t)j * I->nr + I->iobs);
    cx<double> p1 = ldc(phi, (int64_t)j * I->nr + I->iobs + 1);
    stc(I->wave, row * I->nth + j, rfma(I->alpha, p1, (1.0 - I->alpha) * p0));
}
void launch_batch_extract(const BatchInst* inst, int n_inst, int max_nth, const BatchClock* clock, hipStream_t s) {
    hipLaunchKernelGGL(batch_extract_kernel, dim3((max_nth + 255) / 256, n_inst), dim3(256), 0, s, inst, clock);
}

// Waveform at r*_obs: w_j = (1 - alpha) Phi_{i0,j} + alpha Phi_{i0+1,j}.
template <typename R>
__global__ void extract_kernel(const R* __restrict__ phi, R* __restrict__ out, int nr, int nth, int i0,
                               R alpha) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nth) return;
    cx<R> p0 = ldc(phi, (int64_t)j * nr + i0);
    cx<R> p1 = ldc(phi, (int64_t)j * nr + i0 + 1);
    stc(out, j, rfma(alpha, p1, (R(1) - alpha) * p0));
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
