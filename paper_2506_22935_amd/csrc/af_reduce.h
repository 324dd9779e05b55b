// Gradient reduction of the reduction kernels: segment records merged in a
// fixed order, per-segment slabs summed in a fixed order (no atomics touch
// the gradient), dL/dE * s added, optionally one Adam step on the phases.
#pragma once
#include "af_device.h"
#include "af_internal.h"

#include <math.h>

namespace graf {

constexpr float kLog2eR = 1.4426950408889634f;

__device__ __forceinline__ void lse_merge_r(float& m, double& s, float m2, double s2, float inv_t2) {
    if (m2 == m) {  // same shift: a plain sum
        s += s2;
        return;
    }
    float mn = fmaxf(m, m2);
    if (mn == -INFINITY) return;
    s = s * (double)exp2f((m - mn) * inv_t2) + s2 * (double)exp2f((m2 - mn) * inv_t2);
    m = mn;
}

// --------------------------------------------------------------- reduce --
__device__ __forceinline__ double wave_sum_d(double v) { return wave_allsum(v); }

__device__ __forceinline__ void wave_lse_r(float& m, double& s, float inv_t2) { wave_lse_pair(m, s, inv_t2); }

struct WaveTotals {
    double isl_raw, lse_s, dle, ext;
    float lse_m;
};

// Totals of a waveform's segment records, merged by the 256-thread block in
// a fixed order (thread-strided, wavefront butterflies, waves in order).
__device__ WaveTotals wave_totals(const ReduceArgs& a, const WaveDesc& w, double* sh) {
    const float inv_t2 = kLog2eR / a.temp;
    double isl = 0.0, s = 0.0, dle = 0.0, mt = 0.0;
    float m = -INFINITY;
    for (int j = threadIdx.x; j < w.seg_count; j += 256) {
        const Part pr = a.parts[w.seg_begin + j];
        isl += pr.isl;
        dle += pr.dle;
        mt += pr.ext;
        lse_merge_r(m, s, pr.lse_m, pr.lse_s, inv_t2);
    }
    isl = wave_sum_d(isl);
    dle = wave_sum_d(dle);
    if (a.ext_cells) mt = wave_sum_d(mt);
    wave_lse_r(m, s, inv_t2);
    const int wv = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        sh[4 * wv + 0] = isl;
        sh[4 * wv + 1] = dle;
        sh[4 * wv + 2] = (double)m;
        sh[4 * wv + 3] = s;
        sh[16 + wv] = mt;
    }
    __syncthreads();
    WaveTotals t{0.0, 0.0, 0.0, 0.0, -INFINITY};
    for (int i = 0; i < 4; ++i) {
        t.isl_raw += sh[4 * i + 0];
        t.dle += sh[4 * i + 1];
        t.ext += sh[16 + i];
        lse_merge_r(t.lse_m, t.lse_s, (float)sh[4 * i + 2], sh[4 * i + 3], inv_t2);
    }
    return t;
}

// Sum over the waveform's slabs for this block's samples: thread t adds
// slabs t>>pb_log, (t>>pb_log) + SG, ... of sample t & (PB-1); the SG
// subgroup sums meet in LDS and are added in subgroup order.
// The first U slabs of every thread are loaded before the segment records are
// merged (slab_first), so both memory round trips overlap; slab_sum adds them
// and any further slabs in the same order.
constexpr int kSlabU = 32;
struct SlabFirst {
    float2 x[kSlabU];
};
__device__ __forceinline__ void slab_first(const ReduceArgs& a, const WaveDesc& w, int p, SlabFirst& f) {
    const int sub = threadIdx.x >> (8 - a.sg_log);
    const int SG = 1 << a.sg_log;
    const bool ok = !a.skip_slabs && p < w.n;
    const float2* sl = a.slabs + w.slab_off + p;
#pragma unroll
    for (int u = 0; u < kSlabU; ++u) {
        const int j = sub + u * SG;
        f.x[u] = (ok && j < w.seg_count) ? sl[(int64_t)j * w.n] : make_float2(0.f, 0.f);
    }
}
__device__ __forceinline__ float2 slab_sum(const ReduceArgs& a, const WaveDesc& w, int p, const SlabFirst& f,
                                           float2* sh2) {
    const int pb_log = 8 - a.sg_log;
    const int sub = threadIdx.x >> pb_log;
    const int SG = 1 << a.sg_log;
    float2 sum = make_float2(0.f, 0.f);
#pragma unroll
    for (int u = 0; u < kSlabU; ++u) sum = cadd(sum, f.x[u]);
    if (!a.skip_slabs && p < w.n) {
        const float2* sl = a.slabs + w.slab_off + p;
        for (int j = sub + kSlabU * SG; j < w.seg_count; j += SG) sum = cadd(sum, sl[(int64_t)j * w.n]);
    }
    sh2[threadIdx.x] = sum;
    __syncthreads();
    float2 g = make_float2(0.f, 0.f);
    if (sub == 0) {
        const int lane = threadIdx.x;
        for (int k = 0; k < SG; ++k) g = cadd(g, sh2[(k << pb_log) + lane]);
    }
    return g;
}

// dL/dE from the totals: the ISL part is -2 w_isl (collected sum) / E in
// both forms
__device__ __forceinline__ float total_dlde(const ReduceArgs& a, const WaveTotals& t, float E) {
    return (float)(-2.0 * (double)a.w_isl * t.isl_raw / (double)E + t.dle);
}
// the loss terms (one thread per waveform writes them): (L, ISL, PSL term,
// E) with the soft PSL, or the hard PSL from vals; the spectral variance,
// var(|s|) and the smoothness term from vals, the cell-wise extension terms
// from the records
__device__ __forceinline__ float4 loss_terms(const ReduceArgs& a, const WaveDesc& w, int wave, const WaveTotals& t,
                                             float E) {
    // complement waveforms carry ISL - M (Moyal: the full grid holds M E^2;
    // N E^2 for the periodic AF)
    const double isl = t.isl_raw + ((a.uniform_w && w.full_window) ? (double)w.moyal : 0.0);
    const float psl = a.psl_hard ? a.vals[4 * wave]
                                 : ((t.lse_s > 0.0) ? (float)((double)t.lse_m + (double)a.temp * log(t.lse_s)) : 0.f);
    double loss = (double)a.w_isl * isl + (a.w_psl != 0.f ? (double)a.w_psl * (double)psl : 0.0);
    if (a.w_spec != 0.f) loss += (double)a.w_spec * (double)a.vals[4 * wave + 1];
    if (a.w_const != 0.f) loss += (double)a.w_const * (double)a.vals[4 * wave + 2];
    if (a.w_smooth != 0.f) loss += (double)a.w_smooth * (double)a.vals[4 * wave + 3];
    if (a.ext_cells) loss += t.ext;
    return make_float4((float)loss, (float)isl, psl, E);
}

// Sum of a waveform's second slabs (fused loss pass: the ISL part of the
// segments that hold mainlobe lags) at sample p, in segment order.
__device__ __forceinline__ float2 second_slabs(const ReduceArgs& a, const WaveDesc& w, int p) {
    float2 sum = make_float2(0.f, 0.f);
    const float2* sl = a.slabs2 + w.slab2_off + p;
    for (int j = 0; j < w.isl_segs; ++j) sum = cadd(sum, sl[(int64_t)j * w.n]);
    return sum;
}

__device__ __forceinline__ RBlock reduce_block(const ReduceArgs& a, int blk) {
    RBlock b;
    if (a.single) {
        b.w = a.w0;
        b.wave = 0;
        b.p0 = blk * (256 >> a.sg_log);
    } else {
        b = a.blocks[blk];
    }
    return b;
}

// One block of the reduction (the first 256 threads of the work group; any
// further threads only pass the barriers): the gradient of its samples,
// dL/dE * s added, the loss terms from the block holding sample 0, and with
// ADAM one Adam step on the phases (Sec. 6.2's update with the Sec. 7.1.2
// optimiser, dL/dphi = 2 Im(conj(s) g)) using step t_prev + 1.
template <bool ADAM>
__device__ void reduce_chunk(const ReduceArgs& a, int blk, int t_prev, double* sh, float2* sh2) {
    const RBlock b = reduce_block(a, blk);
    const WaveDesc& w = b.w;
    const int p = b.p0 + (int)(threadIdx.x & ((256 >> a.sg_log) - 1));
    const bool mine = (int)threadIdx.x < (256 >> a.sg_log) && p < w.n;
    const int64_t i = w.s_off + (mine ? p : 0);
    // every load this block needs goes out before the first reduction
    const float E = a.energy[b.wave];
    float2 sp = make_float2(0.f, 0.f);
    float m = 0.f, v = 0.f, ph0 = 0.f;
    if (mine) {
        sp = a.s[i];
        if (ADAM) {
            m = a.adam_m[i];
            v = a.adam_v[i];
            ph0 = a.phi[i];
        }
    }
    SlabFirst f;
    slab_first(a, w, p, f);
    const bool isl2 = a.psl_scaled && a.uniform_w && w.full_window && a.w_isl != 0.f && mine;
    const float2 s2 = isl2 ? second_slabs(a, w, p) : make_float2(0.f, 0.f);
    const WaveTotals tt = wave_totals(a, w, sh);
    float2 g = slab_sum(a, w, p, f, sh2);
    float dLdE;
    if (a.psl_scaled) {
        // fused loss pass: main slabs and dL/dE records carry the soft-PSL
        // part without 1/S; the mainlobe ISL part sits in the second slabs
        const double inv_s = tt.lse_s > 0.0 ? 1.0 / tt.lse_s : 0.0;
        g.x = fmaf((float)inv_s, g.x, s2.x);
        g.y = fmaf((float)inv_s, g.y, s2.y);
        dLdE = (float)(-2.0 * (double)a.w_isl * tt.isl_raw / (double)E + tt.dle * inv_s);
    } else {
        dLdE = total_dlde(a, tt, E);
    }
    if (mine) {
        g.x = fmaf(dLdE, sp.x, g.x);
        g.y = fmaf(dLdE, sp.y, g.y);
        if (a.g_extra) g = cadd(g, a.g_extra[i]);
        if (ADAM) {
            const float dphi = 2.f * (sp.x * g.y - sp.y * g.x);
            const float t = (float)(t_prev + 1);
            m = fmaf(a.beta1, m, (1.f - a.beta1) * dphi);
            v = fmaf(a.beta2, v, (1.f - a.beta2) * dphi * dphi);
            const float mh = m / (1.f - powf(a.beta1, t));
            const float vh = v / (1.f - powf(a.beta2, t));
            const float ph = ph0 - a.lr * mh / (sqrtf(vh) + a.adam_eps);
            a.adam_m[i] = m;
            a.adam_v[i] = v;
            a.phi[i] = ph;
            float sn, cs;
            sincosf(ph, &sn, &cs);
            a.s_next[i] = make_float2(cs, sn);
        } else if (a.grad) {
            a.grad[i] = g;
        }
    }
    if (b.p0 == 0 && threadIdx.x == 0 && a.terms)
        reinterpret_cast<float4*>(a.terms)[b.wave] = loss_terms(a, w, b.wave, tt, E);
}

}  // namespace graf
