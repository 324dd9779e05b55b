// Ambiguity-function segment processor and persistent kernel template (gfx950).
//
// One persistent kernel per mode walks a work queue of segments; a segment
// is a contiguous range of non-negative lags of one waveform.  For each lag
// tau >= 0 the kernel forms the shifted lag product
//     r'[m] = s[m + tau] * conj(s[m]),  m in [0, N - tau)
// whose spectrum Y' = DFT_M(r') gives both AF rows (paper Sec. 4.1, Eqs.
// 7-12, aperiodic lags, Doppler sign e^{-j}):
//     chi(tau, k)  = exp(-j 2pi k tau / M) Y'[k]
//     chi(-tau, k) = conj(Y'[-k])
// so |chi(+-tau, .)| need one transform per lag pair.  Since r' is zero on
// [M/2, M) when M >= 2N, Y'[2k'] = DFT_{M/2}(r')[k'] and
// Y'[2k'+1] = DFT_{M/2}(r' w_M^m)[k']: two independent half transforms.
//
// Backward (Sec. 4.2, Eqs. 13-15): every loss here depends on chi only
// through |chi|, so dL/d conj(chi) = c * chi with real c per cell, and the
// upstream of Y' is H[k] = (c(tau,k) + c(-tau,-k)) Y'[k] (tau > 0; c(0,k)
// Y'[k] for tau = 0).  Q' = IDFT_M(H) (unnormalised, e^{+j}) is needed only on
// [0, N - tau) and splits the same way:
//     Q'[m] = IDFT_{M/2}(H_even)[m] + w_M^{-m} IDFT_{M/2}(H_odd)[m].
// The lag-product adjoint then adds, for every lag tau >= 0,
//     g[p] += conj(Q'[p]) s[p + tau]    (p < N - tau)
//     g[p] += Q'[p - tau] s[p - tau]    (p >= tau)
// into per-thread accumulators owned by the work group.  Each segment writes
// its own slab, and a second kernel sums slabs in a fixed order and adds
// dL/dE * s (dE/d conj(s) = s): no atomics touch the gradient, so results are
// bitwise reproducible.
#pragma once
#include "af_device.h"
#include "af_internal.h"

#include <math.h>

#include <type_traits>

namespace graf {

constexpr float kLog2e = 1.4426950408889634f;

// Soft-PSL sums use the shift a_ref = sqrt(1 + eps), an upper bound of every
// a (|chi| <= E by Cauchy-Schwarz, so p <= 1).  When a_ref log2(e) / T < 100
// no term exp((a - a_ref)/T), a >= 0, leaves the normal float range, and the
// fixed shift replaces the running maximum: plain sums, no rescaling.  Smaller
// temperatures fall back to per-iteration maxima merged pairwise.
__device__ __forceinline__ float lse_ref(float eps) { return __builtin_amdgcn_sqrtf(1.f + eps); }
__device__ __forceinline__ bool lse_fixed_shift(float eps, float inv_t2) { return lse_ref(eps) * inv_t2 < 100.f; }

// 2^x without the denormal-range fix-up (results below 2^-126 flush to zero,
// which only drops terms far below the float resolution of the sums)
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// ----------------------------------------------------------- reductions --
__device__ __forceinline__ float wave_sum(float v) { return wave_allsum(v); }
__device__ __forceinline__ double wave_sum(double v) { return wave_allsum(v); }

// log-sum-exp pair (max, sum of exp((x - max)/T)) merge; inv_t2 = log2(e)/T
__device__ __forceinline__ void lse_merge(float& m, double& s, float m2, double s2, float inv_t2) {
    if (m2 == m) {  // same shift (always so with the fixed shift): a plain sum
        s += s2;
        return;
    }
    float mn = fmaxf(m, m2);
    if (mn == -INFINITY) return;
    s = s * (double)exp2f((m - mn) * inv_t2) + s2 * (double)exp2f((m2 - mn) * inv_t2);
    m = mn;
}

__device__ __forceinline__ void wave_lse(float& m, double& s, float inv_t2) { wave_lse_pair(m, s, inv_t2); }

// Sum over the work group in a fixed order: wavefront butterflies, then the
// per-wave results in wave order.  Every thread receives the total.
template <int WGS, typename Tv>
__device__ Tv block_sum(Tv v, double* scratch) {
    constexpr int NW = WGS / 64;
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[w] = (double)v;
    __syncthreads();
    Tv t = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) t += (Tv)scratch[i];
    return t;
}

// ------------------------------------------------------- band weights ----
// separable ISL shaping weight u[floor(31|tau|/N)] * v[floor(31|k_c|/(M/2+1))]
__device__ __forceinline__ int floor_div_small(int a, int d) {
    // exact floor(a / d) for 0 <= a < 2^24, d > 0
    int q = (int)((float)a * (1.0f / (float)d));
    if ((q + 1) * d <= a) ++q;
    if (q * d > a) --q;
    return q;
}

// ------------------------------------------------------- one segment -----
// Thread layout: lane groups of L = MH/P lanes.  SPLIT = 1: the even and the
// odd half transform of a lag run on two neighbouring groups (2L threads per
// lag).  SPLIT = 0: one group runs both halves in turn (L threads per lag).
// In SPLIT mode the magnitude / upstream rows of a lag are staged through the
// lag's two transform buffers (2 * (MH + MH/32) complex >= 2 rows of M floats)
// so that global traffic is coalesced 16-byte row accesses.
// Per-waveform state a work group keeps across the segments it runs: the
// energy, the soft-PSL normaliser (backward of the loss) and the samples
// staged in LDS.
struct WaveState {
    int wave;
    float E;
    float glob_m, glob_inv_s;
};

// Fill the pass tables that follow the half table w_M^i (i < MH, already in
// LDS and visible to every thread) from it: w_M^i = -w_M^(i - MH) for i >= MH.
template <int WGS, int MH, int P>
__device__ __forceinline__ void build_pass_tables(float2* twl, int tid) {
    constexpr int NP = PassTables<MH, P>::total();
    for (int e = tid; e < NP; e += WGS) {
        const int src = pass_table_source<MH, P>(e);
        const float2 w = twl[src & (MH - 1)];
        twl[MH + e] = src < MH ? w : make_float2(-w.x, -w.y);
    }
}

// Stage waveform `wave` (N <= MH samples) into LDS and compute its energy;
// with twl != nullptr also copy this size's twiddles w_M^i (i < 2 MH) from the
// global table; for the loss backward also merge the forward pass records
// into the soft-PSL normaliser.  Every global load is issued before the first
// barrier, so one memory round trip covers all of them.  CIRC (periodic AF,
// N = MH): the samples are staged twice, s_lds[p] = s[p mod N] for p < 2 N,
// so that the lag product reads s[(m + tau) mod N] as s_lds[m + tau].
// UNPAD (aperiodic): MH + 1 entries, zero from N on, and the lag product
// clamps its shifted index to MH instead of reading a zero-padded copy.
template <int MODE, int WGS, int MH, bool CIRC = false, int P = 16, bool UNPAD = false>
__device__ void stage_wave(const AfArgs& a, const WaveDesc& w, int wave, float2* s_lds, bool s_in_lds,
                           double* scratch, WaveState& st, float2* twl, int twsh) {
    constexpr int NPT = (MH + WGS - 1) / WGS;
    constexpr int TPT = (MH + WGS - 1) / WGS;  // the half table w_M^i, i < MH
    constexpr int PPT = 4;  // records per thread merged from registers
    constexpr bool MERGE = MODE == MODE_BWD_LOSS;
    int tid = threadIdx.x;
    // opaque, as in process_segment: the sample indices below are not
    // hoisted out of the persistent item loop
    asm volatile("" : "+v"(tid));
    float2 tx[TPT];
    if (twl) {
#pragma unroll
        for (int i = 0; i < TPT; ++i) {
            const int j = tid + i * WGS;
            tx[i] = j < MH ? a.tw[j << twsh] : make_float2(0.f, 0.f);
        }
    }
    const float2* __restrict__ sg_s = a.s + w.s_off;
    float2 sx[NPT];
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
        const int p = tid + i * WGS;
        sx[i] = p < w.n ? sg_s[p] : make_float2(0.f, 0.f);
    }
    const bool merge = MERGE && a.w_psl != 0.f;
    float pm[MERGE ? PPT : 1];
    double ps[MERGE ? PPT : 1];
    if (merge) {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int j = tid + i * WGS;
            pm[i] = -INFINITY;
            ps[i] = 0.0;
            if (j < w.seg_count) {
                pm[i] = a.parts[w.seg_begin + j].lse_m;
                ps[i] = a.parts[w.seg_begin + j].lse_s;
            }
        }
    }
    __syncthreads();  // the previous segment is done with s_lds and scratch
    float e = 0.f;
#pragma unroll
    for (int i = 0; i < NPT; ++i) e += cabs2(sx[i]);
    if (CIRC && s_in_lds) {
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int p = tid + i * WGS;
            if (p < MH) {
                s_lds[p] = sx[i];
                s_lds[p + MH] = sx[i];
            }
        }
    } else if (UNPAD && s_in_lds) {
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int p = tid + i * WGS;
            if (p < MH) s_lds[p] = sx[i];  // zero from N on
        }
        if (tid == 0) s_lds[MH] = make_float2(0.f, 0.f);
    } else if (s_in_lds) {
        // 2 MH entries, zero from N on: every lag product index m + tau
        // (m < MH, tau <= N) reads a sample or a zero
#pragma unroll
        for (int i = 0; i < 2 * NPT; ++i) {
            const int p = tid + i * WGS;
            if (p < 2 * MH) s_lds[p] = (i < NPT && p < w.n) ? sx[i < NPT ? i : 0] : make_float2(0.f, 0.f);
        }
    }
    if (twl) {
#pragma unroll
        for (int i = 0; i < TPT; ++i) {
            const int j = tid + i * WGS;
            if (j < MH) twl[j] = tx[i];
        }
    }
    st.wave = wave;
    st.glob_m = 0.f;
    st.glob_inv_s = 0.f;
    if (!merge) {
        st.E = block_sum<WGS, float>(e, scratch);
    } else {
        // energy and the global soft-PSL normaliser in one fixed-order
        // reduction: thread-strided records, wavefront butterflies, waves in order
        const float inv_t2 = kLog2e / a.temp;
        const bool fixed = lse_fixed_shift(a.eps, inv_t2);
        float m = -INFINITY;
        double s = 0.0;
        if (fixed) {
            // every record carries the shift a_ref
            m = lse_ref(a.eps);
#pragma unroll
            for (int i = 0; i < (MERGE ? PPT : 1); ++i) s += ps[i];
            for (int j = tid + PPT * WGS; j < w.seg_count; j += WGS) s += a.parts[w.seg_begin + j].lse_s;
            s = wave_sum(s);
        } else {
#pragma unroll
            for (int i = 0; i < (MERGE ? PPT : 1); ++i) lse_merge(m, s, pm[i], ps[i], inv_t2);
            for (int j = tid + PPT * WGS; j < w.seg_count; j += WGS) {
                const Part pr = a.parts[w.seg_begin + j];
                lse_merge(m, s, pr.lse_m, pr.lse_s, inv_t2);
            }
            wave_lse(m, s, inv_t2);
        }
        e = wave_sum(e);
        if ((tid & 63) == 0) {
            scratch[3 * (tid >> 6)] = (double)m;
            scratch[3 * (tid >> 6) + 1] = s;
            scratch[3 * (tid >> 6) + 2] = (double)e;
        }
        __syncthreads();
        m = fixed ? lse_ref(a.eps) : -INFINITY;
        s = 0.0;
        float et = 0.f;
        for (int i = 0; i < WGS / 64; ++i) {
            if (fixed)
                s += scratch[3 * i + 1];
            else
                lse_merge(m, s, (float)scratch[3 * i], scratch[3 * i + 1], inv_t2);
            et += (float)scratch[3 * i + 2];
        }
        st.E = et;
        st.glob_m = m;
        st.glob_inv_s = (float)(1.0 / s);
    }
    // the block sums above passed barriers after the half table's stores
    if (twl) build_pass_tables<WGS, MH, P>(twl, tid);
    __syncthreads();
}

// Copy this size's twiddles from the global table to LDS as the half table
// w_M^i (i < MH) and the transform's pass tables (classes with several
// waveforms, before their first item).
template <int WGS, int MH, int P>
__device__ void stage_twiddles(const AfArgs& a, float2* twl, int twsh) {
    constexpr int TPT = (MH + WGS - 1) / WGS;
    float2 tx[TPT];
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
        const int j = threadIdx.x + i * WGS;
        tx[i] = j < MH ? a.tw[j << twsh] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
        const int j = threadIdx.x + i * WGS;
        if (j < MH) twl[j] = tx[i];
    }
    __syncthreads();
    build_pass_tables<WGS, MH, P>(twl, threadIdx.x);
    __syncthreads();
}

// Copy the two short twiddle tables of TwSplit (lo: w_M^j, j < 2^b; hi:
// w_M^(h 2^b), h < M / 2^b) and, with p1 (non-null only for M >= 256), the
// first-pass table w_256^(r k) from the global table w_M^(i << twsh), then
// synchronise.
template <int WGS, int MH, int B>
__device__ void stage_split_twiddles(const AfArgs& a, float2* hi, float2* lo, float2* p1, int twsh) {
    constexpr int M = 2 * MH;
    constexpr int NLO = 1 << B, NHI = M >> B;
    const int np1 = (p1 && M >= 256) ? kPass1Entries : 0;
    for (int j = threadIdx.x; j < NLO + NHI + np1; j += WGS) {
        if (j < NLO) {
            lo[j] = a.tw[j << twsh];
        } else if (j < NLO + NHI) {
            hi[j - NLO] = a.tw[((j - NLO) << B) << twsh];
        } else {
            const int e = j - NLO - NHI, r = e / 16 + 1, k = e % 16;
            p1[e] = a.tw[((r * k * (M / 256)) & (M - 1)) << twsh];
        }
    }
    __syncthreads();
}

// CIRC: the periodic AF of N = MH samples (lag index modulo N, N Doppler
// bins).  Its N-point spectrum of the lag product is the even half of the
// aperiodic M = 2N split, so every lane group takes a lag of its own; one
// transform gives rows tau and N - tau of the [N][N] grid (tau = 0 and
// tau = N/2 give one row each), and the lag product and its adjoint index
// samples modulo N.
// instances that take the extended epilogue terms (hard-PSL maximum,
// L_match, mainlobe width, cell weights): the forward and the fused ISL
// passes built with EXTK (split variants); the plain instances of both
// carry none of that code
template <int MODE, bool EXTK>
constexpr bool EXT_MODE() {
    return (MODE == MODE_FWD || MODE == MODE_FUSED_ISL) && EXTK;
}

// MAGONLY (forward): a and spectra only, no loss sums and no chi rows, so the
// instance carries a single family of epilogue copies (the halves-in-turn
// variant then keeps every value in its 128 registers)
// HARDONLY (extended forward): the hard-PSL maximum is the only extended term
template <int MODE, int MH, int P, int SPLIT, int WGS, int NACC, bool CIRC, bool EXTK, bool MAGONLY = false,
          bool UNPAD = false, bool HARDONLY = false, typename Tw>
__device__ __forceinline__ void process_segment(const AfArgs& a, const SegDesc sg, float2* lds, const Tw& twl,
                                                const float2* s_lds, bool s_in_lds, double* scratch,
                                                const WaveState& ws) {
    constexpr int L = MH / P;
    constexpr int G = WGS / L;
    constexpr int LPI = (SPLIT && !CIRC) ? G / 2 : G;  // lags per iteration
    constexpr int BUF = LdsSize<MH>::value;
    constexpr int TPL = (SPLIT && !CIRC) ? 2 * L : L;  // threads per lag
    constexpr int M_ = 2 * MH;
    constexpr int RL = CIRC ? MH : M_;  // grid row length (Doppler bins)
    static_assert(!CIRC || SPLIT, "periodic AF needs a split variant");
    constexpr bool NEEDS_INV = MODE != MODE_FWD;
    constexpr bool HAS_MAG_OUT = MODE == MODE_FWD || MODE == MODE_FUSED_ISL || MODE == MODE_LOSS;
    constexpr bool FWD_SUMS = MODE == MODE_FWD || MODE == MODE_LOSS;  // soft-PSL partials
    static_assert(L >= 1 && G >= (SPLIT ? 2 : 1), "group does not fit the work group");
    static_assert(!SPLIT || (2 * BUF * 2 >= 2 * M_), "row staging does not fit");

    int tid = threadIdx.x;
    // an opaque lane index per item: the lane-dependent expressions below
    // are not hoisted out of a persistent kernel's item loop, where one
    // kernel serving several transform sizes would keep every size's copies
    // live across its items
    asm volatile("" : "+v"(tid));
    const int grp = tid / L;
    int l = tid - grp * L;
    const int lam = (SPLIT && !CIRC) ? (grp >> 1) : grp;
    const int hsel = (SPLIT && !CIRC) ? ((L % 64 == 0) ? __builtin_amdgcn_readfirstlane(grp & 1) : (grp & 1)) : 0;
    const int t2 = tid - lam * TPL;  // thread index among the lag's threads
    float2* buf = lds + grp * BUF;
    float* rowbuf = reinterpret_cast<float*>(lds + ((SPLIT && !CIRC) ? 2 * lam : lam) * BUF);

    const WaveDesc w = a.single ? a.w0 : a.waves[sg.wave];
    const int N = w.n, T = w.T;
    constexpr int M = M_;
    const int tshift = a.log2_mmax - w.log2m;  // w_M^i = tw[i << tshift]
    const float2* __restrict__ sg_s = a.s + w.s_off;
    const float2* __restrict__ tw = a.tw;
    // transform passes exchange data only inside the lane group: when the
    // group lies within one wavefront (L divides 64), ordering the
    // wavefront's own LDS accesses suffices
    auto sync = []() {
        if constexpr (L <= 64) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __syncthreads();
        }
    };

    const float E = ws.E;
    if (sg.tau_begin == 0 && tid == 0) a.energy[sg.wave] = E;
    const float invE = 1.0f / E;
    const float invE2 = invE * invE;
    const float2* __restrict__ sv = s_in_lds ? s_lds : sg_s;
    const float inv_t2 = kLog2e / a.temp;
    const bool want_lse = !MAGONLY && FWD_SUMS && a.w_psl != 0.f;
    const bool lse_fixed = lse_fixed_shift(a.eps, inv_t2);
    const float aref_t2 = lse_ref(a.eps) * inv_t2;
    const float glob_m = ws.glob_m, glob_inv_s = ws.glob_inv_s;
    const bool banded = a.band_w != nullptr && w.band_off >= 0;
    const float* bu = banded ? a.band_w + w.band_off : nullptr;
    const float* bv = banded ? a.band_w + w.band_off + 31 : nullptr;
    const bool mag_out = HAS_MAG_OUT && a.mag != nullptr;
    const bool chi_out = !MAGONLY && MODE == MODE_FWD && a.chi != nullptr;

    // gradient accumulators: registers, or (halves in turn, long waveforms)
    // the segment's own slab in global memory, which only this group touches
    constexpr bool GACC = !SPLIT;
    float2 acc[(NEEDS_INV && !GACC) ? NACC : 1];
#pragma unroll
    for (int i = 0; i < ((NEEDS_INV && !GACC) ? NACC : 1); ++i) acc[i] = make_float2(0.f, 0.f);
    float2* const slab = NEEDS_INV ? a.slabs + w.slab_off + (int64_t)(sg.rec - w.seg_begin) * N : nullptr;
    // global samples (variants without samples in LDS) and the slab of the
    // halves-in-turn variants through buffer resources over exactly N values
    const Rsrc s_rs = make_rsrc(sg_s, (unsigned)N * 8u);
    const Rsrc slab_rs = make_rsrc(slab, NEEDS_INV ? (unsigned)N * 8u : 0u);
    if (NEEDS_INV && GACC) {
        for (int p = tid; p < N; p += WGS) buf_store2(slab_rs, p * 8, make_float2(0.f, 0.f));
    }
    // lag-product adjoint of lag tj from Q' in LDS (qa, plus qa + BUF when the
    // two halves sit in two buffers)
    // (to_dst true: accumulate into gdst[p] instead; a compile-time choice so
    // that the register accumulators stay in registers)
    auto gather = [&](const float2* qa, bool two, int tj, auto to_dst, float2* gdst) {
        constexpr bool TO_DST = decltype(to_dst)::value;
        if constexpr (CIRC) {
            // conj(Q[p]) s[(p + tj) mod N] + Q[(p - tj) mod N] s[(p - tj) mod N]
            // (samples staged twice: s_lds[p + tj] is s[(p + tj) mod N])
#pragma unroll
            for (int i = 0; i < NACC; ++i) {
                const int p = tid + WGS * i;
                if (p < N) {
                    float2 sum = TO_DST ? gdst[p] : acc[TO_DST ? 0 : i];
                    sum = cadd(sum, cmul(cconj(qa[lds_index(p)]), sv[p + tj]));
                    const int m = p >= tj ? p - tj : p - tj + N;
                    sum = cadd(sum, cmul(qa[lds_index(m)], sv[m]));
                    if (TO_DST)
                        gdst[p] = sum;
                    else
                        acc[TO_DST ? 0 : i] = sum;
                }
            }
            return;
        }
        const int Sj = N - tj;
#pragma unroll
        for (int i = 0; i < NACC; ++i) {
            const int p = tid + WGS * i;
            if (p < N) {
                float2 sum = TO_DST ? gdst[p] : (GACC ? buf_load2(slab_rs, p * 8) : acc[(GACC || TO_DST) ? 0 : i]);
                if (p < Sj) {
                    float2 Q = qa[lds_index(p)];
                    if (two) Q = cadd(Q, qa[BUF + lds_index(p)]);
                    sum = cadd(sum, cmul(cconj(Q), s_in_lds ? sv[p + tj] : buf_load2(s_rs, (p + tj) * 8)));
                }
                const int m = p - tj;
                if (m >= 0) {
                    float2 Q = qa[lds_index(m)];
                    if (two) Q = cadd(Q, qa[BUF + lds_index(m)]);
                    sum = cadd(sum, cmul(Q, s_in_lds ? sv[m] : buf_load2(s_rs, m * 8)));
                }
                if (TO_DST)
                    gdst[p] = sum;
                else if (GACC)
                    buf_store2(slab_rs, p * 8, sum);
                else
                    acc[(GACC || TO_DST) ? 0 : i] = sum;
            }
            // slab accumulation: bound the loads the scheduler keeps in flight
            if (GACC && (i & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
    };
    const bool compl_isl = a.band_w == nullptr && w.full_window != 0;
    // MODE_LOSS: the ISL gradient lives on the mainlobe cells (complement
    // form); segments holding mainlobe lags collect it in their second slab
    const bool isl_seg = MODE == MODE_LOSS && compl_isl && a.w_isl != 0.f && sg.tau_begin <= w.h_tau;
    float2* const slab2 = isl_seg ? a.slabs2 + w.slab2_off + (int64_t)(sg.rec - w.seg_begin) * N : nullptr;
    // With few mainlobe bins, Q of the ISL part is evaluated directly from
    // H on those bins (2 h_k + 1 per lag, kept in scratch) instead of a
    // second transform pair; its first iteration then initialises the slab.
    const int n_mb = 2 * w.h_k + 1;
    const bool direct_isl = isl_seg && LPI * n_mb <= 64;
    if (isl_seg && !direct_isl) {
        for (int p = tid; p < N; p += WGS) slab2[p] = make_float2(0.f, 0.f);
    }
    float2* const mlb = reinterpret_cast<float2*>(scratch);
    double isl = 0.0, ls = 0.0, dle = 0.0, mt = 0.0;
    // L_match against a target power grid, the soft mainlobe width, a
    // per-cell weight grid and the hard-PSL maximum (forward and fused ISL
    // modes; the extended epilogue copy)
    constexpr bool EXT_OK = EXT_MODE<MODE, EXTK>();
    const bool match = EXT_OK && a.match_t != nullptr;
    const bool width = EXT_OK && a.w_width != 0.f;
    const bool cellw = EXT_OK && a.cell_w != nullptr;
    // the extensions' arguments read once per segment into uniform locals:
    // read through the argument struct inside the cell loops, they came from
    // a stack copy of it, each read a memory round trip that also waited for
    // the target reads in flight
    const float* const x_match_t = a.match_t;
    const float* const x_cell_w = a.cell_w;
    const float x_w_match = a.w_match, x_w_width = a.w_width, x_gamma = a.gamma, x_w_cell = a.w_cell;
    // likewise the loss weights and eps that the cell loops use
    const float x_w_isl = a.w_isl, x_w_psl = a.w_psl, x_eps = a.eps;
    const bool hard_rt = EXT_OK && a.psl_hard != 0;
    const bool ext_full = match || width || cellw;  // beyond the hard-PSL maximum
    const bool ext_rt = ext_full || hard_rt;
    // hard PSL: this lane's largest sidelobe power and its cell (tau >= 0 row)
    float hp = -1.f;
    int hi = 0;
    float lm = (want_lse && (lse_fixed || MODE == MODE_LOSS)) ? lse_ref(x_eps) : -INFINITY;

    // the odd half's factor w_M^m at the lane's points m = l + r L: w_M^l,
    // read once per lane (returned here), times the constant
    // w_M^(r L) = exp(-j 2 pi r / 2P).  The 1024-thread variant (128
    // registers) keeps one table read per point: the constants' extra live
    // values cost its backward more than the reads
    constexpr bool FOLD = WGS < 1024;
    auto odd_base = [&](int h) { return (FOLD && h) ? twl.low(l) : make_float2(1.f, 0.f); };
    // Y' of lag tau, half h, in the exit layout v[q] = Y'[2 (l + qL) + h]
    auto lag_spectrum = [&](float2* v, int h, int tau, bool active) {
        if (CIRC) {
            // r'[m] = s[(m + tau) mod N] conj(s[m]), m < N = MH; an inactive
            // lag (tau may lie past N/2 + 1) reads lag 0 and gives zero
            const int tz = active ? tau : 0;
#pragma unroll
            for (int r = 0; r < P; ++r) {
                const int m = l + r * L;
                const float2 x = cmulc(sv[m + tz], sv[m]);
                v[r] = active ? x : make_float2(0.f, 0.f);
                if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
            }
        } else if (s_in_lds) {
            // zero-padded samples: r'[m] = 0 for m >= N - tau comes out of
            // the product itself; an inactive lag reads zeros
            const int tz = active ? tau : N;
            const float2 c = odd_base(h);
#pragma unroll
            for (int r = 0; r < P; ++r) {
                const int m = l + r * L;
                // UNPAD: entry MH is zero, as is every entry from N on
                float2 x = cmulc(sv[UNPAD ? min(m + tz, MH) : m + tz], sv[m]);
                if (h) x = cmul(x, c);
                v[r] = x;
                if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
            }
            if (h) twist_const<2 * P, -1, P>(v);
        } else {
            // samples through the buffer resource over [0, N): the range
            // check zeroes s[m + tau] for m >= N - tau; an inactive lag reads
            // only zeros
            const int tz = active ? tau : N;
            const float2 c = odd_base(h);
#pragma unroll
            for (int r = 0; r < P; ++r) {
                const int m = l + r * L;
                float2 x = cmulc(buf_load2(s_rs, (m + tz) * 8), buf_load2(s_rs, m * 8));
                if (h) x = cmul(x, FOLD ? c : twl.low(m));
                v[r] = x;
                // bound how many loads the scheduler keeps in flight
                if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
            }
            if (FOLD && h) twist_const<2 * P, -1, P>(v);
        }
        fft_group<MH, P, -1, (WGS >= 1024)>(v, buf, l, twl, sync);
    };
    // Q' of half h: inverse transform, w_M^{-m} on the odd half, stored to
    // this group's buffer in natural order
    auto inverse_to_lds = [&](float2* v, int h) {
        fft_group<MH, P, +1, (WGS >= 1024)>(v, buf, l, twl, sync);
        if (h) {
            const float2 c = odd_base(h);
#pragma unroll
            for (int q = 0; q < P; ++q) v[q] = cmulc(v[q], FOLD ? c : twl.low(l + q * L));
            if (FOLD) twist_const<2 * P, +1, P>(v);
        }
        if constexpr (L % 32 == 0) {
            const int bi = lds_index(l);
#pragma unroll
            for (int q = 0; q < P; ++q) buf[bi + lds_off(q * L)] = v[q];
        } else {
#pragma unroll
            for (int q = 0; q < P; ++q) buf[lds_index(l + q * L)] = v[q];
        }
    };

    for (int t0 = sg.tau_begin; t0 < sg.tau_end; t0 += LPI) {
        // lane groups of whole wavefronts: the lag is wave-uniform
        const int tau = (L % 64 == 0) ? __builtin_amdgcn_readfirstlane(t0 + lam) : t0 + lam;
        const bool active = tau < sg.tau_end;
        // does lag tau have a distinct partner row -tau (periodic: N - tau)?
        const bool two_rows = CIRC ? (tau > 0 && 2 * tau != N) : (tau > 0);
        const float mult = two_rows ? 2.f : 1.f;
        const bool main_tau = tau <= w.h_tau;
        const float wu = (banded && active) ? bu[(31 * tau) / N] : 1.f;
        const int tz = active ? tau : 0;
        const int64_t row_p = CIRC ? w.grid_off + (int64_t)tz * RL : w.grid_off + (int64_t)(T + tz) * M;
        const int64_t row_n = CIRC ? w.grid_off + (int64_t)(tz ? N - tz : 0) * RL : w.grid_off + (int64_t)(T - tz) * M;
        // rows tau and -tau of the halves-in-turn epilogue (empty when inactive)
        const unsigned row_bytes = active ? (unsigned)RL * 4u : 0u;
        const Rsrc mag_p = make_rsrc(HAS_MAG_OUT && a.mag ? a.mag + row_p : nullptr, HAS_MAG_OUT && a.mag ? row_bytes : 0u);
        const Rsrc mag_n = make_rsrc(HAS_MAG_OUT && a.mag ? a.mag + row_n : nullptr, HAS_MAG_OUT && a.mag ? row_bytes : 0u);
        const Rsrc gm_p = make_rsrc(MODE == MODE_BWD_MAG ? a.grad_mag + row_p : nullptr, MODE == MODE_BWD_MAG ? row_bytes : 0u);
        const Rsrc gm_n = make_rsrc(MODE == MODE_BWD_MAG ? a.grad_mag + row_n : nullptr, MODE == MODE_BWD_MAG ? row_bytes : 0u);

        // prefetch the two upstream rows (tau, -tau) while the transform runs
        constexpr int NPF = (MODE == MODE_BWD_MAG && SPLIT) ? (2 * RL / 4) / TPL : 1;
        float4 gpre[NPF];
        if (MODE == MODE_BWD_MAG && SPLIT) {
#pragma unroll
            for (int i = 0; i < NPF; ++i) {
                const int f = t2 + i * TPL;  // float4 index over both rows
                const int r = f >= RL / 4;
                const int64_t base = r ? row_n : row_p;
                gpre[i] = (active && (two_rows || !r))
                              ? *reinterpret_cast<const float4*>(a.grad_mag + base + 4 * (f - r * (RL / 4)))
                              : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }

        // magnitude-only forward of the halves-in-turn variant: the even
        // half's magnitudes wait in registers for the odd half's, so that
        // each row goes out in whole lines (one half alone would leave every
        // other 4-byte bin of a line to a later write).  Reading the
        // backward's upstream rows in pairs the same way measured slower:
        // the held values push its 128 registers into spills
        constexpr bool PAIR = !SPLIT && MAGONLY;
        float hold[PAIR ? P : 1];
#pragma unroll 1
        for (int hh = 0; hh < (SPLIT ? 1 : 2); ++hh) {
            const int h = SPLIT ? hsel : hh;
            // have every lane-index expression (LDS and row offsets, bin
            // numbers) recomputed in the loop from an opaque lane index:
            // cheap integer arithmetic, where hoisting it out of the loop
            // keeps dozens of values live and spills them
            asm volatile("" : "+v"(l), "+v"(tid));
            float2 v[P];
            if (NEEDS_INV && a.load_store) {
                // an inactive lag gets an empty range: zeros
                const Rsrc ys = make_rsrc(a.ystore + w.store_off + (int64_t)(active ? tau : 0) * (CIRC ? MH : M) + h * MH,
                                          active ? (unsigned)MH * 8u : 0u);
#pragma unroll
                for (int q = 0; q < P; ++q) v[q] = buf_load2(ys, (l + q * L) * 8);
            } else {
                lag_spectrum(v, h, tau, active);
            }
            // v[q] = Y'[2 (l + qL) + h]
            if (MODE == MODE_FWD && a.ystore && active) {
                const Rsrc ys = make_rsrc(a.ystore + w.store_off + (int64_t)tau * (CIRC ? MH : M) + h * MH,
                                          (unsigned)MH * 8u);
#pragma unroll
                for (int q = 0; q < P; ++q) buf_store2(ys, (l + q * L) * 8, v[q]);
            }
            if constexpr (SPLIT) {
                if (mag_out || MODE == MODE_BWD_MAG || chi_out) __syncthreads();  // transform buffers free
                if (MODE == MODE_BWD_MAG) {
                    float4* rb4 = reinterpret_cast<float4*>(rowbuf);
#pragma unroll
                    for (int i = 0; i < NPF; ++i) rb4[t2 + i * TPL] = gpre[i];
                    __syncthreads();
                }
            }

            // ---------------------------------------------- epilogue --
            // p = |Y'|^2/E^2, a = sqrt(p + eps); the sidelobe test and the
            // weight are symmetric under (tau, k) -> (-tau, -k).  Sums over
            // the lane's bins run in float, then fold into float64.
            float isl_f = 0.f, dle_f = 0.f, mloc = -INFINITY, sl_f = 0.f;
            float mt_f = 0.f, dlm_f = 0.f;  // L_match: both cells of the pair explicitly
            float wd_f = 0.f;               // soft mainlobe width
            float cw_f = 0.f;               // per-cell weights: sum W p
            float avs[(MODE == MODE_FWD) ? P : 1];
            // One straight-line copy per loss configuration (shift rule,
            // banded weights, mainlobe complement, soft-PSL on/off): every
            // condition left inside is per lane and becomes a select.
            // MAIN: the lag may hold mainlobe cells (tau <= h_tau); without
            // them every mainlobe test is compiled out
            // EXT: the rarely used extensions, each behind a uniform runtime
            // test: 1 the hard-PSL maximum alone, 2 also L_match, the mainlobe
            // width and the cell weights
            auto epilogue = [&](auto fixed_c, auto banded_c, auto compl_c, auto psl_c, auto main_c, auto ext_c) {
                constexpr bool FIXED = decltype(fixed_c)::value;
                constexpr bool BANDED = decltype(banded_c)::value;
                constexpr bool COMPL = decltype(compl_c)::value;
                constexpr bool PSL = decltype(psl_c)::value;
                constexpr bool MAIN = decltype(main_c)::value;
                constexpr int EXT = decltype(ext_c)::value;  // 0, 1: hard PSL only, 2: every extension
                const float c_main = -mult * x_w_isl * invE2;  // d(M - mainlobe power)/d conj(chi)
                // the per-cell reads of L_match and the cell weights (both cells
                // of the pair; the -tau row only with a distinct partner) go
                // out together before the cells' arithmetic, so one memory
                // round trip serves the lane's P cells.  Plain per-lane
                // pointers: the lag, and so the row, differs between the lane
                // groups of a wavefront.  The halves-in-turn variant (128
                // registers) reads each cell's values where it uses them.
                constexpr bool BATCH = EXT == 2 && SPLIT;
                constexpr int XR = BATCH ? P : 1;
                float tg_p[XR], tg_n[XR], cw_p[XR], cw_n[XR];
                if constexpr (BATCH) {
#pragma unroll
                    for (int q = 0; q < P; ++q) {
                        const int k = CIRC ? l + q * L : 2 * (l + q * L) + h;
                        const int kn = k ? RL - k : 0;
                        tg_p[q] = tg_n[q] = cw_p[q] = cw_n[q] = 0.f;
                        if (match) {
                            tg_p[q] = active ? x_match_t[row_p + k] : 0.f;
                            tg_n[q] = (active && two_rows) ? x_match_t[row_n + kn] : 0.f;
                        }
                        if (cellw) {
                            cw_p[q] = active ? x_cell_w[row_p + k] : 0.f;
                            cw_n[q] = (active && two_rows) ? x_cell_w[row_n + kn] : 0.f;
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    // bin of the grid row (periodic: v[q] is bin l + qL of N)
                    const int k = CIRC ? l + q * L : 2 * (l + q * L) + h;
                    const int kn = k ? RL - k : 0;
                    const int kc = k < (RL >> 1) ? k : RL - k;  // |centred bin|
                    const float pw = cabs2(v[q]) * invE2;
                    // a = sqrt(x) and 1/a = rsqrt(x): modes that need both take
                    // one reciprocal square root and a multiply
                    constexpr bool NEED_IA = MODE == MODE_BWD_MAG || MODE == MODE_LOSS ||
                                             (MODE == MODE_BWD_LOSS && PSL);
                    const float xa = pw + x_eps;
                    const float ia = NEED_IA ? __builtin_amdgcn_rsqf(xa) : 0.f;
                    const float av = NEED_IA ? xa * ia : __builtin_amdgcn_sqrtf(xa);
                    const bool main_cell = MAIN && active && main_tau && kc <= w.h_k;
                    const bool sd = active && !main_cell;
                    if (EXT >= 1 && hard_rt) {
                        // largest power, then the smallest cell index
                        const int ci = tau * RL + k;
                        const bool better = sd && (pw > hp || (pw == hp && ci < hi));
                        hp = better ? pw : hp;
                        hi = better ? ci : hi;
                    }
                    float wt = 1.f;
                    if constexpr (BANDED) {
                        // the band index is in [0, 30] for every bin
                        wt = wu * bv[floor_div_small(31 * kc, (RL >> 1) + 1)];
                    }
                    if (HAS_MAG_OUT) {
                        if (mag_out) {
                            if (SPLIT) {
                                rowbuf[k] = av;
                                rowbuf[RL + kn] = av;
                            } else if constexpr (PAIR) {
                                if (h == 0) {
                                    hold[PAIR ? q : 0] = av;
                                } else if (active) {
                                    // bins k - 1 (even) and k of row tau as one pair;
                                    // row -tau holds them at M - k + 1 and M - k
                                    buf_store2(mag_p, (k - 1) * 4, make_float2(hold[PAIR ? q : 0], av));
                                    if (tau > 0) {
                                        buf_store1(mag_n, (k == 1 ? 0 : RL - k + 1) * 4, hold[PAIR ? q : 0]);
                                        buf_store1(mag_n, (RL - k) * 4, av);
                                    }
                                }
                            } else if (active) {
                                buf_store1(mag_p, k * 4, av);
                                if (tau > 0) buf_store1(mag_n, kn * 4, av);
                            }
                        }
                        if constexpr (COMPL)
                            isl_f -= main_cell ? pw : 0.f;  // mainlobe power
                        else
                            isl_f = fmaf(sd ? wt : 0.f, pw, isl_f);
                    }
                    // exp((a - a_ref)/T): the fixed-shift soft-PSL term
                    const float e = (FWD_SUMS && PSL && FIXED) ? fast_exp2(fmaf(av, inv_t2, -aref_t2)) : 0.f;
                    if constexpr (FWD_SUMS && PSL) {
                        if constexpr (FIXED) {
                            sl_f += sd ? e : 0.f;
                        } else {
                            avs[q] = sd ? av : -INFINITY;
                            mloc = fmaxf(mloc, avs[q]);
                        }
                    }
                    // L_match: (p - p_t)^2 for the cell (tau, k) and, with a
                    // distinct partner, (-tau, -k); coefficient and energy
                    // term per cell, not through the pair multiplier
                    float cm = 0.f;
                    // Eq. 21: the k = 0 cells of rows tau and -tau (equal
                    // powers) weigh |tau| sigma(gamma (p - 1/2)), since
                    // p(0, 0) = 1 for every waveform; upstream
                    // |tau| gamma sigma' per cell, energy term -2 p / E
                    if (EXT == 2 && width && k == 0) {
                        const float ld = (float)(CIRC ? min(tau, N - tau) : tau);
                        const float sg = 1.f / (1.f + fast_exp2(-kLog2e * x_gamma * (pw - 0.5f)));
                        wd_f += active ? mult * ld * sg : 0.f;
                        if constexpr (NEEDS_INV) {
                            const float u = active ? mult * x_w_width * ld * x_gamma * sg * (1.f - sg) : 0.f;
                            cm += u * invE2;
                            dlm_f = fmaf(-2.f * u * pw, invE, dlm_f);
                        }
                    }
                    if (EXT == 2 && cellw) {
                        // W p on both cells of the pair, each with its own weight
                        const float wp = BATCH ? cw_p[BATCH ? q : 0] : (active ? x_cell_w[row_p + k] : 0.f);
                        const float wn = BATCH ? cw_n[BATCH ? q : 0]
                                               : ((active && two_rows) ? x_cell_w[row_n + kn] : 0.f);
                        cw_f = fmaf(wp + wn, pw, cw_f);
                        if constexpr (NEEDS_INV) {
                            cm += x_w_cell * (wp + wn) * invE2;
                            dlm_f = fmaf(-2.f * x_w_cell * (wp + wn) * pw, invE, dlm_f);
                        }
                    }
                    if (EXT == 2 && match) {
                        const float tp = BATCH ? tg_p[BATCH ? q : 0] : (active ? x_match_t[row_p + k] : 0.f);
                        const float tn = BATCH ? tg_n[BATCH ? q : 0]
                                               : ((active && two_rows) ? x_match_t[row_n + kn] : 0.f);
                        const float dp = active ? pw - tp : 0.f;
                        const float dn = (active && two_rows) ? pw - tn : 0.f;
                        mt_f = fmaf(dp, dp, fmaf(dn, dn, mt_f));
                        if constexpr (NEEDS_INV) {
                            cm += 2.f * x_w_match * (dp + dn) * invE2;
                            dlm_f = fmaf(-4.f * x_w_match * pw * invE, dp + dn, dlm_f);
                        }
                    }
                    if constexpr (NEEDS_INV) {
                        float c = 0.f;
                        if constexpr (MODE == MODE_BWD_MAG) {
                            float g;
                            if (SPLIT) {
                                g = rowbuf[k];
                                if (two_rows) g += rowbuf[RL + kn];
                            } else {
                                g = buf_load1(gm_p, k * 4);
                                if (tau > 0) g += buf_load1(gm_n, kn * 4);
                            }
                            g = active ? g : 0.f;
                            c = 0.5f * g * invE2 * ia;
                            dle_f = fmaf(-g * pw * invE, ia, dle_f);
                        } else if constexpr (MODE == MODE_BWD_LOSS) {
                            float cs = COMPL ? 0.f : x_w_isl * wt * invE2;
                            if constexpr (PSL) {
                                const float qq = fast_exp2((av - glob_m) * inv_t2) * glob_inv_s;
                                    cs = fmaf(x_w_psl * qq * 0.5f * invE2, ia, cs);
                                dle_f = fmaf(sd ? -x_w_psl * qq * pw * invE : 0.f, ia, dle_f);
                            }
                            c = sd ? mult * cs : ((COMPL && main_cell) ? c_main : 0.f);
                        } else if constexpr (MODE == MODE_LOSS) {
                            if (direct_isl && main_cell) {
                                // H of the ISL part on this mainlobe bin
                                const int ks = k < (RL >> 1) ? k : k - RL;
                                mlb[lam * n_mb + ks + w.h_k] = cscale(v[q], -mult * x_w_isl * invE2);
                            }
                            // soft-PSL part without the normaliser 1/S
                            c = sd ? mult * x_w_psl * e * 0.5f * invE2 * ia : 0.f;
                            dle_f = fmaf(sd ? -x_w_psl * e * pw * invE : 0.f, ia, dle_f);
                        } else {  // MODE_FUSED_ISL
                            if constexpr (COMPL)
                                c = main_cell ? c_main : 0.f;
                            else
                                c = sd ? mult * x_w_isl * wt * invE2 : 0.f;
                        }
                        v[q] = cscale(v[q], c + cm);
                    }
                }
            };
            using T_ = std::integral_constant<bool, true>;
            using F_ = std::integral_constant<bool, false>;
            auto by_loss = [&](auto fixed_c, auto psl_c, auto main_c, auto ext_c) {
                if (banded)
                    epilogue(fixed_c, T_{}, F_{}, psl_c, main_c, ext_c);
                else if (compl_isl)
                    epilogue(fixed_c, F_{}, T_{}, psl_c, main_c, ext_c);
                else
                    epilogue(fixed_c, F_{}, F_{}, psl_c, main_c, ext_c);
            };
            // the hot fused passes also get a copy without mainlobe logic for
            // the lags beyond the mainlobe (tau > h_tau: all but a few)
            // of the extended copies, the hard-PSL maximum alone (the
            // experiment loss's forward pass) keeps a copy without the other
            // extensions' per-cell tests
            auto ext_copy = [&]() {
                if constexpr (HARDONLY) {
                    by_loss(T_{}, F_{}, T_{}, std::integral_constant<int, 1>{});
                } else {
                    if (ext_full)
                        by_loss(T_{}, F_{}, T_{}, std::integral_constant<int, 2>{});
                    else
                        by_loss(T_{}, F_{}, T_{}, std::integral_constant<int, 1>{});
                }
            };
            if constexpr (MODE == MODE_FWD && MAGONLY) {
                by_loss(T_{}, F_{}, T_{}, F_{});
            } else if constexpr (MODE == MODE_FWD) {
                if (!want_lse && ext_rt)
                    ext_copy();
                else if (!want_lse)
                    by_loss(T_{}, F_{}, T_{}, F_{});
                else if (lse_fixed)
                    by_loss(T_{}, T_{}, T_{}, F_{});
                else
                    by_loss(F_{}, T_{}, T_{}, F_{});
            } else if constexpr (MODE == MODE_BWD_LOSS) {
                if (x_w_psl != 0.f)
                    by_loss(T_{}, T_{}, T_{}, F_{});
                else
                    by_loss(T_{}, F_{}, T_{}, F_{});
            } else if constexpr (MODE == MODE_BWD_MAG) {
                epilogue(T_{}, F_{}, F_{}, F_{}, F_{}, F_{});
            } else if constexpr (MODE == MODE_LOSS) {
                if (compl_isl && main_tau)
                    epilogue(T_{}, F_{}, T_{}, T_{}, T_{}, F_{});
                else if (compl_isl)
                    epilogue(T_{}, F_{}, T_{}, T_{}, F_{}, F_{});
                else if (main_tau)
                    epilogue(T_{}, F_{}, F_{}, T_{}, T_{}, F_{});
                else
                    epilogue(T_{}, F_{}, F_{}, T_{}, F_{}, F_{});
            } else if constexpr (EXTK) {
                ext_copy();
            } else if (main_tau) {
                by_loss(T_{}, F_{}, T_{}, F_{});
            } else {
                by_loss(T_{}, F_{}, F_{}, F_{});
            }
            isl += (double)(mult * isl_f);
            dle += (double)((MODE == MODE_BWD_MAG ? 1.f : mult) * dle_f + dlm_f);
            if (match || width || cellw)
                mt += (double)fmaf(x_w_match, mt_f, fmaf(x_w_width, wd_f, x_w_cell * cw_f));
            if (FWD_SUMS && want_lse && (lse_fixed || MODE == MODE_LOSS)) {
                ls += (double)(mult * sl_f);
            } else if (MODE == MODE_FWD && want_lse && mloc > -INFINITY) {
                // this iteration's sidelobe cells, two per bin for tau > 0
                float sl = 0.f;
#pragma unroll
                for (int q = 0; q < P; ++q) sl += fast_exp2((avs[q] - mloc) * inv_t2);
                lse_merge(lm, ls, mloc, (double)(mult * sl), inv_t2);
            }

            if constexpr (SPLIT) {
                if (mag_out) {
                    // coalesced row stores: rows tau and -tau (tau = 0: one row)
                    __syncthreads();
                    const float4* rb4 = reinterpret_cast<const float4*>(rowbuf);
                    if (active) {
                        for (int f = t2; f < 2 * (RL / 4); f += TPL) {
                            const int r = f >= RL / 4;
                            if (r && !two_rows) break;
                            float4* dst = reinterpret_cast<float4*>(a.mag + (r ? row_n : row_p)) + (f - r * (RL / 4));
                            *dst = rb4[f];
                        }
                    }
                }
                if (chi_out) {
                    // complex AF rows from the spectrum staged in natural order
                    __syncthreads();
                    float2* yb = reinterpret_cast<float2*>(rowbuf);
#pragma unroll
                    for (int q = 0; q < P; ++q) yb[CIRC ? l + q * L : 2 * (l + q * L) + h] = v[q];
                    __syncthreads();
                    if (active) {
                        for (int k = t2; k < RL; k += TPL) {
                            // w_RL^{k tau} = w_M^{(M / RL) k tau}
                            const int ti = (int)(((int64_t)k * tau * (M / RL)) & (M - 1));
                            a.chi[row_p + k] = cmul(yb[k], tw[ti << tshift]);
                            if (two_rows) a.chi[row_n + k] = cconj(yb[k ? RL - k : 0]);
                        }
                    }
                }
                if (NEEDS_INV && (mag_out || MODE == MODE_BWD_MAG || chi_out)) __syncthreads();
            } else {
                if (chi_out && active) {
#pragma unroll 1
                    for (int q = 0; q < P; ++q) {
                        float2 y = make_float2(0.f, 0.f);
#pragma unroll
                        for (int qq = 0; qq < P; ++qq)
                            if (qq == q) y = v[qq];
                        const int k = 2 * (l + q * L) + h;
                        const int ti = (int)(((int64_t)k * tau) & (M - 1));
                        a.chi[row_p + k] = cmul(y, tw[ti << tshift]);
                        if (tau > 0) a.chi[row_n + (k ? M - k : 0)] = cconj(y);
                    }
                }
            }

            if constexpr (NEEDS_INV) {
                inverse_to_lds(v, h);
                if constexpr (!SPLIT) {
                    // halves in turn: this half's share of every lag's adjoint
                    __syncthreads();
                    for (int j = 0; j < LPI; ++j) {
                        if (t0 + j >= sg.tau_end) break;
                        gather(lds + j * BUF, false, t0 + j, std::false_type{}, nullptr);
                    }
                    __syncthreads();
                }
            }
        }

        if constexpr (NEEDS_INV && SPLIT) {
            __syncthreads();
            // lag-product adjoint for every lag of this iteration
            for (int j = 0; j < LPI; ++j) {
                if (t0 + j >= sg.tau_end) break;
                if (CIRC)
                    gather(lds + j * BUF, false, t0 + j, std::false_type{}, nullptr);
                else
                    gather(lds + 2 * j * BUF, true, t0 + j, std::false_type{}, nullptr);
            }
        }
        __syncthreads();
        if constexpr (MODE == MODE_LOSS && SPLIT) {
            if (direct_isl && t0 <= w.h_tau) {
                // ISL part of the mainlobe lags: Q[m] = sum over the mainlobe
                // bins of H[k] exp(+j 2 pi k m / M), into each lag's buffer
                for (int j = 0; j < LPI; ++j) {
                    const int tj = t0 + j;
                    if (tj >= sg.tau_end || tj > w.h_tau) break;
                    float2* qb = lds + (CIRC ? j : 2 * j) * BUF;
                    const float2* hb = mlb + j * n_mb;
                    for (int m = tid; m < (CIRC ? N : N - tj); m += WGS) {
                        float2 qv = make_float2(0.f, 0.f);
                        for (int b = 0; b < n_mb; ++b) {
                            // exp(+j 2 pi k m / RL) = conj(w_M^{(M / RL) k m})
                            const int ti = ((b - w.h_k) * m * (M / RL)) & (M - 1);
                            qv = cadd(qv, cmulc(hb[b], twl(ti)));
                        }
                        qb[lds_index(m)] = qv;
                    }
                }
                __syncthreads();
                // adjoint of every mainlobe lag of the iteration in registers,
                // then one write (or update) of the second slab
                float2 acc2[NACC];
#pragma unroll
                for (int i = 0; i < NACC; ++i) acc2[i] = make_float2(0.f, 0.f);
                for (int j = 0; j < LPI; ++j) {
                    const int tj = t0 + j;
                    if (tj >= sg.tau_end || tj > w.h_tau) break;
                    const float2* qa = lds + (CIRC ? j : 2 * j) * BUF;
#pragma unroll
                    for (int i = 0; i < NACC; ++i) {
                        const int p = tid + WGS * i;
                        if (CIRC) {
                            if (p < N) {
                                acc2[i] = cadd(acc2[i], cmul(cconj(qa[lds_index(p)]), sv[p + tj]));
                                const int m = p >= tj ? p - tj : p - tj + N;
                                acc2[i] = cadd(acc2[i], cmul(qa[lds_index(m)], sv[m]));
                            }
                        } else {
                            if (p < N - tj) acc2[i] = cadd(acc2[i], cmul(cconj(qa[lds_index(p)]), sv[p + tj]));
                            if (p < N && p >= tj) acc2[i] = cadd(acc2[i], cmul(qa[lds_index(p - tj)], sv[p - tj]));
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < NACC; ++i) {
                    const int p = tid + WGS * i;
                    if (p < N) slab2[p] = (t0 == sg.tau_begin) ? acc2[i] : cadd(slab2[p], acc2[i]);
                }
                __syncthreads();
            } else if (isl_seg && t0 <= w.h_tau) {
                // ISL part of the mainlobe lags: the spectrum again, times
                // d(M - mainlobe power)/d conj(chi) = -w_isl/E^2 on mainlobe
                // cells (both signs of tau for tau > 0), into the second slab
                float2 v[P];
                lag_spectrum(v, hsel, tau, active);
                const float c_main = -mult * x_w_isl * invE2;
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const int k = CIRC ? l + q * L : 2 * (l + q * L) + hsel;
                    const int kc = k < (RL >> 1) ? k : RL - k;
                    const bool main_cell = active && main_tau && kc <= w.h_k;
                    v[q] = cscale(v[q], main_cell ? c_main : 0.f);
                }
                inverse_to_lds(v, hsel);
                __syncthreads();
                for (int j = 0; j < LPI; ++j) {
                    if (t0 + j >= sg.tau_end) break;
                    if (CIRC)
                        gather(lds + j * BUF, false, t0 + j, std::true_type{}, slab2);
                    else
                        gather(lds + 2 * j * BUF, true, t0 + j, std::true_type{}, slab2);
                }
                __syncthreads();
            }
        }
    }

    // ------------------------------------------- segment results -------
    // one fixed-order reduction of (ISL, soft-PSL pair, dL/dE) over the group
    // wavefront sums in float (each lane's partial already folds its cells in
    // float64; 64 float terms keep the 1e-4 loss and gradient bars with room),
    // wave totals combined in float64 below
    if (FWD_SUMS) {
        if (lse_fixed || MODE == MODE_LOSS)
            ls = (double)wave_sum((float)ls);
        else
            wave_lse(lm, ls, inv_t2);
    }
    isl = (double)wave_sum((float)isl);
    if (MODE != MODE_FWD) dle = (double)wave_sum((float)dle);
    if (match || width || cellw) mt = (double)wave_sum((float)mt);
    // hard PSL: the wavefront's largest power, then its smallest cell index
    const bool hard = hard_rt;
    if (hard) {
        const float wmx = wave_allmax(hp);
        hi = wave_allmin_int(hp == wmx ? hi : 0x7fffffff);
        hp = wmx;
    }
    __syncthreads();
    if ((tid & 63) == 0) {
        scratch[4 * (tid >> 6) + 0] = isl;
        scratch[4 * (tid >> 6) + 1] = (double)lm;
        scratch[4 * (tid >> 6) + 2] = ls;
        scratch[4 * (tid >> 6) + 3] = dle;
        if (hard) {
            scratch[64 + 2 * (tid >> 6)] = (double)hp;
            scratch[65 + 2 * (tid >> 6)] = (double)hi;
        }
        scratch[96 + (tid >> 6)] = mt;
    }
    __syncthreads();
    if (tid == 0) {
        Part pr;
        pr.isl = 0.0;
        pr.lse_s = 0.0;
        pr.dle = 0.0;
        pr.lse_m = -INFINITY;
        pr.ext = 0.0;
        pr.psl_p = -1.f;
        pr.psl_i = 0;
        pr.pad = 0;
        for (int i = 0; i < WGS / 64; ++i) {
            pr.isl += scratch[4 * i + 0];
            if (FWD_SUMS) lse_merge(pr.lse_m, pr.lse_s, (float)scratch[4 * i + 1], scratch[4 * i + 2], inv_t2);
            pr.dle += scratch[4 * i + 3];
            pr.ext += scratch[96 + i];
            if (hard) {
                // waves in order: larger power, then the smaller cell index
                const float p = (float)scratch[64 + 2 * i];
                const int c = (int)scratch[65 + 2 * i];
                if (p > pr.psl_p || (p == pr.psl_p && c < pr.psl_i)) {
                    pr.psl_p = p;
                    pr.psl_i = c;
                }
            }
        }
        if (MODE == MODE_BWD_LOSS)
            a.parts[sg.rec].dle = pr.dle;
        else
            a.parts[sg.rec] = pr;
    }
    if constexpr (NEEDS_INV) {
        if (!GACC) {
#pragma unroll
            for (int i = 0; i < NACC; ++i) {
                const int p = tid + WGS * i;
                if (p < N) slab[p] = acc[GACC ? 0 : i];
            }
        }
    }
    __syncthreads();
}

// ------------------------------------------------- variants and kernels --
// A variant fixes points per lane P, the half-transform split, the work-group
// size and the occupancy target; each kernel instance covers one transform
// size MH = M/2 = 2^LG.  Gradient accumulators per thread: NACC = MH / WGS
// (N <= M/2 = MH), at least one.
template <int P_, int SPLIT_, int WGS_, int WAVES_, int LO_, int HI_, int S_LDS_, int TW_LDS_>
struct Variant {
    static constexpr int P = P_, SPLIT = SPLIT_, WGS = WGS_, WAVES = WAVES_, LO = LO_, HI = HI_, S_LDS = S_LDS_;
    static constexpr int TW_LDS = TW_LDS_;  // twiddle table copied to LDS
    static constexpr int nacc(int lg) { return (1 << lg) / WGS > 1 ? (1 << lg) / WGS : 1; }
    static constexpr bool fits(int lg) {
        return lg >= LO && lg <= HI && (1 << lg) >= P &&
               (SPLIT ? 2 * ((1 << lg) / P) <= WGS : ((1 << lg) / P) <= WGS);
    }
    // dynamic LDS of one instance: transform buffers, then the twiddle table
    // w_M^i for i < M = 2^(lg+1), or (TW_LDS = 0) its two short factors
    static constexpr int split_bits(int lg) { return (lg + 2) / 2; }
    static constexpr int split_lds_bytes(int lg) { return (((2 << lg) >> split_bits(lg)) + (1 << split_bits(lg))) * 8; }
    static constexpr int buf_lds_bytes(int lg) { return (WGS / ((1 << lg) / P)) * ((1 << lg) + ((1 << lg) >> 5)) * 8; }
    // two-factor variants with 16-point passes also keep the first-pass table
    static constexpr int p1_lds_bytes() { return (!TW_LDS && P == 16) ? kPass1Entries * 8 : 0; }
    static constexpr int fft_lds_bytes(int lg) {
        return buf_lds_bytes(lg) + (TW_LDS ? (2 << lg) * 8 : split_lds_bytes(lg) + p1_lds_bytes());
    }
};

//                 P  split WGS waves LG range  s, twiddles in LDS
using V0 = Variant<16, 1, 256, 2, 6, 11, 1, 1>;  // M 128..4096
using V1 = Variant<16, 1, 512, 2, 12, 12, 1, 0>; // M 8192
using V2 = Variant<16, 0, 1024, 4, 13, 14, 0, 0>; // M 16384..32768, halves in turn
using V3 = Variant<8, 1, 256, 2, 6, 10, 1, 1>;   // more lanes per lag, M <= 2048
using V4 = Variant<32, 1, 256, 1, 8, 11, 1, 1>;  // fewer passes, M 512..4096
using V5 = Variant<32, 1, 256, 1, 12, 12, 1, 0>; // M 8192: 32 points per lane, one wave per SIMD

// Persistent kernel over one size class: work group g runs items g, g + grid,
// g + 2 grid, ... of the class's list, which the planner sorted longest first
// (a static, deterministic assignment).
template <int MODE, typename V, int LG, bool CIRC = false, bool EXTK = false, bool MAGONLY = false,
          bool HARDONLY = false>
__global__ __launch_bounds__(V::WGS, V::WAVES) void af_kernel(AfArgs a) {
    static_assert(!CIRC || (V::SPLIT && V::S_LDS), "periodic AF: split variants with samples in LDS");
    static_assert(!V::TW_LDS || (1 << LG) + PassTables<(1 << LG), V::P>::total() <= (2 << LG),
                  "half table and pass tables exceed the twiddle area");
    extern __shared__ float2 dyn[];
    // block reductions; [64, 96) holds the per-wave hard-PSL records,
    // [96, 112) the per-wave sums of the cell-wise extension terms
    __shared__ double scratch[112];
    constexpr int MH = 1 << LG;
    float2* lds = dyn;
    float2* s_lds = V::S_LDS ? dyn + V::fft_lds_bytes(LG) / 8 : nullptr;
    float2* tw_lds = V::TW_LDS ? dyn + V::buf_lds_bytes(LG) / 8 : nullptr;
    const int twsh_global = a.log2_mmax - (LG + 1);
    constexpr int TB = V::split_bits(LG);
    float2* tw_lo = dyn + V::buf_lds_bytes(LG) / 8;
    float2* tw_hi = tw_lo + (1 << TB);
    using Tw = std::conditional_t<V::TW_LDS != 0, TwPass, TwSplit>;
    Tw twl;
    if constexpr (V::TW_LDS) {
        twl = TwPass{tw_lds, tw_lds + MH, MH};
    } else {
        float2* tw_p1 = (V::p1_lds_bytes() > 0 && MH >= 128) ? tw_hi + ((2 << LG) >> TB) : nullptr;
        twl = TwSplit{tw_hi, tw_lo, TB, tw_p1};
        if (blockIdx.x < a.n_segs) stage_split_twiddles<V::WGS, MH, TB>(a, tw_hi, tw_lo, tw_p1, twsh_global);
    }
    WaveState st;
    st.wave = -1;
    // the first item's descriptor travels with the staging loads; each later
    // one is fetched while the previous item runs
    SegDesc next;
    if (blockIdx.x < a.n_segs) next = a.segs[blockIdx.x];
    if (blockIdx.x < a.n_segs) {
        if (a.single) {
            // one waveform: its samples, the twiddles and the first item's
            // descriptor travel in the same memory round trip
            stage_wave<MODE, V::WGS, MH, CIRC, V::P>(a, a.w0, a.w0_index, s_lds, V::S_LDS != 0, scratch, st,
                                                     tw_lds, twsh_global);
        } else if (tw_lds) {
            stage_twiddles<V::WGS, MH, V::P>(a, tw_lds, twsh_global);
        }
    }
    for (int item = blockIdx.x; item < a.n_segs; item += gridDim.x) {
        const SegDesc sg = next;
        if (item + (int)gridDim.x < a.n_segs) next = a.segs[item + gridDim.x];
        if (sg.wave != st.wave) {
            // a class with one waveform carries its descriptor in the arguments
            const WaveDesc w = a.single ? a.w0 : a.waves[sg.wave];
            stage_wave<MODE, V::WGS, MH, CIRC, V::P>(a, w, sg.wave, s_lds, V::S_LDS != 0, scratch, st, nullptr, 0);
        }
        process_segment<MODE, MH, V::P, V::SPLIT, V::WGS, V::nacc(LG), CIRC, EXTK, MAGONLY, false, HARDONLY>(
            a, sg, lds, twl, s_lds, V::S_LDS != 0, scratch, st);
    }
}

// ------------------------------------------------- one-launch kernel -----
// Every size class of a plan in one persistent launch: 512-thread work
// groups, 16 points per lane, split halves, samples in LDS, the twiddles of
// each class read from the two short tables of the plan's largest transform
// and, for the passes of stride 16 and 256, from the tables of those passes.
// The LDS of the transform buffers is the same for every size (WGS P (1 +
// 1/32) complex values), so one allocation serves all classes; items come
// from one work queue sorted longest first, taken with an atomic ticket.
//
// LDS: transform buffers, short tables, first-pass table, then one region
// that holds (aperiodic) the stride-256 pass table and the samples, or
// (periodic) the samples staged twice.  The aperiodic samples of the largest
// size do not fit beside that table zero-padded to M, so that size stages
// MH + 1 entries and clamps the lag product's index (UNPAD).
using VU = Variant<16, 1, 512, 2, 6, 12, 1, 0>;
constexpr int kUnionP2Bytes = kPass2Entries * 8;
__host__ __device__ constexpr bool union_unpad(int lg) { return lg == VU::HI; }
__host__ __device__ constexpr int union_region_bytes(int lg) {
    const int circ = 8 * (2 << lg);
    const int aper = kUnionP2Bytes + 8 * (union_unpad(lg) ? (1 << lg) + 2 : (2 << lg));
    return circ > aper ? circ : aper;
}

template <int MODE, int LG, bool CIRC, bool EXTK, typename Tw>
__device__ __forceinline__ void union_item(const AfArgs& a, const SegDesc& sg, WaveState& st, float2* lds,
                                           float2* s_lds, double* scratch, const Tw& twl) {
    if constexpr (VU::fits(LG)) {
        constexpr int MH = 1 << LG;
        constexpr bool UNPAD = !CIRC && union_unpad(LG);
        if (sg.wave != st.wave) {
            const WaveDesc w = a.waves[sg.wave];
            stage_wave<MODE, VU::WGS, MH, CIRC, VU::P, UNPAD>(a, w, sg.wave, s_lds, true, scratch, st, nullptr, 0);
        }
        process_segment<MODE, MH, VU::P, VU::SPLIT, VU::WGS, VU::nacc(LG), CIRC, EXTK, false, UNPAD>(
            a, sg, lds, twl, s_lds, true, scratch, st);
    }
}

template <int MODE, bool CIRC = false, bool EXTK = false>
__global__ __launch_bounds__(VU::WGS, VU::WAVES) void af_union_kernel(AfArgs a) {
    extern __shared__ float2 dyn[];
    __shared__ double scratch[112];
    __shared__ int ticket;
    constexpr int LGMAX = VU::HI;
    float2* lds = dyn;
    // short tables sized for the largest transform the kernel takes; the
    // plan's largest M = 2^log2_mmax sets the split actually used
    float2* tw_lo = dyn + VU::buf_lds_bytes(LGMAX) / 8;
    float2* tw_hi = tw_lo + (1 << VU::split_bits(LGMAX));
    float2* tw_p1 = tw_hi + ((2 << LGMAX) >> VU::split_bits(LGMAX));
    float2* region = dyn + VU::fft_lds_bytes(LGMAX) / 8;
    float2* tw_p2 = CIRC ? nullptr : region;
    float2* s_lds = CIRC ? region : region + kPass2Entries;
    const int b = (a.log2_mmax + 1) / 2;  // split bits of the plan's largest M
    const int mmax = 1 << a.log2_mmax;
    const int nlo = 1 << b, nhi = mmax >> b;
    const int np1 = mmax >= 256 ? kPass1Entries : 0;  // first-pass table (classes with M >= 256)
    // stride-256 pass table (classes with M >= 1024): w_4096^(r k) where
    // r k M_max / 4096 is a whole index of the plan's table; the entries a
    // transform of M <= M_max reads are all of that kind
    const int np2 = (!CIRC && mmax >= 1024) ? kPass2Entries : 0;
    if (threadIdx.x == 0) ticket = atomicAdd(a.queue, 1);
    for (int j = threadIdx.x; j < nlo + nhi + np1 + np2; j += VU::WGS) {
        if (j < nlo) {
            tw_lo[j] = a.tw[j];
        } else if (j < nlo + nhi) {
            tw_hi[j - nlo] = a.tw[(j - nlo) << b];
        } else if (j < nlo + nhi + np1) {
            const int e = j - nlo - nhi, r = e / 16 + 1, k = e % 16;
            tw_p1[e] = a.tw[(r * k * (mmax / 256)) & (mmax - 1)];
        } else {
            const int e = j - nlo - nhi - np1, r = e / 256 + 1, k = e % 256;
            const int t = r * k * mmax;
            tw_p2[e] = (t & 4095) == 0 ? a.tw[(t >> 12) & (mmax - 1)] : make_float2(0.f, 0.f);
        }
    }
    __syncthreads();
    WaveState st;
    st.wave = -1;
    using Tw = TwSplitSh<!CIRC>;
    for (;;) {
        const int item = ticket;  // the same for every thread of the group
        if (item >= a.n_segs) break;
        const SegDesc sg = a.segs[item];
        const int log2m = a.waves[sg.wave].log2m;
        const Tw twl{tw_hi, tw_lo, b, a.log2_mmax - log2m, tw_p1, tw_p2};
        switch (log2m - 1) {
            case 6: union_item<MODE, 6, CIRC, EXTK>(a, sg, st, lds, s_lds, scratch, twl); break;
            case 7: union_item<MODE, 7, CIRC, EXTK>(a, sg, st, lds, s_lds, scratch, twl); break;
            case 8: union_item<MODE, 8, CIRC, EXTK>(a, sg, st, lds, s_lds, scratch, twl); break;
            case 9: union_item<MODE, 9, CIRC, EXTK>(a, sg, st, lds, s_lds, scratch, twl); break;
            case 10: union_item<MODE, 10, CIRC, EXTK>(a, sg, st, lds, s_lds, scratch, twl); break;
            case 11: union_item<MODE, 11, CIRC, EXTK>(a, sg, st, lds, s_lds, scratch, twl); break;
            case 12: union_item<MODE, 12, CIRC, EXTK>(a, sg, st, lds, s_lds, scratch, twl); break;
            default: break;
        }
        // every thread has read this item's ticket (process_segment ends
        // with a barrier); take the next
        __syncthreads();
        if (threadIdx.x == 0) ticket = atomicAdd(a.queue, 1);
        __syncthreads();
    }
}

}  // namespace graf
