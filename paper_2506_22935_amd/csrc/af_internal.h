// Types shared by the host planner (af_api.hip) and the kernels (af_segment.h
// via af_variant.hip, af_reduce.hip).  Not part of the public C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace graf {

// One waveform of a batch, as the kernels see it.
struct WaveDesc {
    int n, m, T, log2m;       // length, Doppler bins, lag half-width, log2(M)
    int64_t s_off;            // first sample in the packed complex64 input
    int64_t grid_off;         // first element of its [2T+1][M] grids
    int64_t store_off;        // first element of its [T+1][M] spectrum store
    int64_t slab_off;         // first complex64 of its slabs ([segs][N])
    int seg_begin, seg_count; // its segments (consecutive partial records)
    int h_tau, h_k;           // mainlobe half-widths (lags, bins)
    int band_off;             // first of its 62 shaping weights, or -1
    int full_window;          // T = N - 1: with uniform ISL weights the ISL is
                              // taken as M - (mainlobe power), Moyal's identity
    int isl_segs;             // its segments that hold mainlobe lags (tau <= h_tau)
    int64_t slab2_off;        // first complex64 of their second slabs
    int circ;                 // periodic AF: N = M/2 bins, lag pairs tau, N - tau
                              // for tau in [0, T = N/2], grid [N][N]
    int moyal;                // sum of p over the whole grid with a full window:
                              // M (aperiodic) or N (periodic)
};

// One work item: lags [tau_begin, tau_end) (tau >= 0) of one waveform.
struct SegDesc {
    int wave, tau_begin, tau_end, rec;  // rec = slab / partial-record index
};

// Per-segment partial results, accumulated in float64 where they are sums
// over many cells.  isl: the segment's share of the ISL (for a complement
// waveform, minus its mainlobe power: ISL = M + sum of these); lse_m, lse_s:
// soft-PSL log-sum-exp pair (max a, sum exp((a - max)/T)); dle: dL/dE share;
// psl_p, psl_i: the largest sidelobe power of the segment and its cell
// tau * (row length) + k on the tau >= 0 row (hard PSL; the smallest index
// among equal powers; psl_p = -1 without a sidelobe cell).
struct Part {
    double isl;
    double lse_s;
    double dle;
    double ext;    // weighted cell-wise extension terms over the segment's cells:
                   // w_match (p - p_target)^2 + w_width |tau| sigma(gamma (p(tau, 0) - 1/2))
                   // + w_cell W_cell p
    float lse_m;
    float psl_p;
    int psl_i;
    int pad;
};

enum Mode : int {
    MODE_FWD = 0,       // spectra -> magnitude / AF / stored spectra / loss parts
    MODE_BWD_MAG = 1,   // upstream dL/da grid -> gradient slabs
    MODE_BWD_LOSS = 2,  // ISL + soft-PSL loss -> gradient slabs (needs MODE_FWD parts)
    MODE_FUSED_ISL = 3, // ISL loss forward and backward in one pass
    MODE_LOSS = 4,      // ISL (mainlobe complement) + soft-PSL (fixed shift) loss,
                        // forward and backward in one pass; the soft-PSL
                        // gradient is left unnormalised for the reduction
    MODE_FUSED_EXT = 5, // launch id only: the MODE_FUSED_ISL pass in its own
                        // instance with the extended epilogue terms (hard-PSL
                        // maximum, L_match, mainlobe width; split variants), so
                        // that the plain fused pass keeps its registers
    MODE_FWD_EXT = 6,   // launch id only: the MODE_FWD pass with the extended
                        // epilogue terms, likewise; the plain forward carries
                        // none of their code and keeps every value in registers
    MODE_FWD_MAG = 7,   // launch id only: af_forward without chi rows: a grid and
                        // spectra only (its own instance in the halves-in-turn
                        // variant, whose full forward does not fit 128 registers;
                        // MODE_FWD elsewhere)
    MODE_FWD_HARD = 8   // launch id only: the MODE_FWD pass recording the hard-PSL
                        // maximum and no other extended term (the experiment
                        // loss's pass), in an instance without the per-cell
                        // code of the other terms
};
constexpr int kNumModes = 9;
// launch ids that run the extended epilogue
constexpr bool is_ext_mode(int mode) {
    return mode == MODE_FUSED_EXT || mode == MODE_FWD_EXT || mode == MODE_FWD_HARD;
}

struct AfArgs {
    WaveDesc w0;          // the waveform of a one-waveform class (single != 0)
    int single;
    int w0_index;
    const float2* s;
    const WaveDesc* waves;
    const SegDesc* segs;  // this launch's items in execution order
    int n_segs;
    int log2_mmax;
    const float2* tw;     // exp(-j 2 pi i / MMAX), i < MMAX
    float eps;
    float w_isl, w_psl, temp;
    const float* band_w;  // [62] per waveform, or null
    float* mag;           // [grid] fp32, nullable (MODE_FWD, MODE_FUSED_ISL)
    float2* chi;          // [grid] complex64, nullable (MODE_FWD)
    float2* ystore;       // spectra store [T+1][M], nullable
    int load_store;       // backward reads spectra from ystore instead of recomputing
    const float* grad_mag;  // [grid] (MODE_BWD_MAG)
    Part* parts;          // [records]
    float2* slabs;        // [sum segs*N]
    float2* slabs2;       // [sum isl_segs*N] ISL part of MODE_LOSS
    float* energy;        // [B], written by the segment holding lag 0
    int psl_hard;         // MODE_FWD_EXT / MODE_FUSED_EXT: record the hard-PSL maximum
    const float* match_t; // target power grid of L_match (MODE_FWD_EXT / MODE_FUSED_EXT), nullable
    float w_match;
    float w_width, gamma; // soft mainlobe width on the k = 0 column (MODE_FWD_EXT / MODE_FUSED_EXT)
    const float* cell_w;  // per-cell weight grid (MODE_FWD_EXT / MODE_FUSED_EXT), nullable
    float w_cell;
    int* queue;           // one-launch plans: the work-queue ticket counter (zero at launch)
};

// The slab reduction runs 256-thread blocks over (256 >> sg_log) samples of
// one waveform; the threads split the waveform's slabs into 2^sg_log
// interleaved subgroups and add the subgroup sums in a fixed order
// (deterministic, no atomics).  sg_log is 0, 2 or 4, picked by the planner.

// One block of the gradient reduction: samples [p0, p0 + 256 >> sg_log) of
// waveform `wave`, with that waveform's descriptor alongside so that a block
// needs one load before its data loads.
struct RBlock {
    WaveDesc w;
    int wave, p0;
};

struct ReduceArgs {
    const float2* s;
    const RBlock* blocks;
    int n_blocks;
    WaveDesc w0;          // one-waveform plans: blocks are implicit (single != 0)
    int single;
    int psl_scaled;       // slabs and dL/dE records carry the soft-PSL part
                          // without 1/S (MODE_LOSS); the ISL part is in slabs2
    const float2* slabs2;
    int sg_log;           // log2 of the slab subgroups per block
    const Part* parts;
    const float2* slabs;
    const float* energy;
    float w_isl, w_psl, temp;
    float2* grad;         // dL/d conj(s), packed like s; nullable
    float* terms;         // [B][4] = loss, ISL, soft-PSL, E; nullable
    int skip_slabs;       // loss only: do not read gradient slabs
    int uniform_w;        // no shaping weights: full-window ISL uses the complement
    // fused Adam on phases (grad == null then): phi, m, v packed like s
    float* phi;
    float* adam_m;
    float* adam_v;
    float2* s_next;       // exp(j phi_new)
    int* step;            // device step counter (1-based after increment)
    float lr, beta1, beta2, adam_eps;
    // per-waveform terms from extra_kernel and the cell-wise extension terms
    int ext_cells;        // add the segment records' ext (already weighted)
    int psl_hard;         // the PSL term is the hard maximum (vals[4b])
    float w_spec;         // weight of the spectral variance (vals[4b + 1])
    float w_const;        // weight of var(|s|) (vals[4b + 2])
    float w_smooth;       // weight of the phase-smoothness term (vals[4b + 3])
    const float2* g_extra;  // their gradient, packed like s; nullable
    const float* vals;    // [B][4] = hard PSL, spectral variance, var(|s|), smoothness
};

// Per-waveform terms: the hard-PSL maximum of the experiment loss
// (Sec. 7.1.1) from the segment records, chi at that cell and its
// single-cell adjoint; the spectral variance of the N-point spectrum with
// its gradient; var(|s|) and the phase-smoothness term of the composite loss
// (Sec. 5.2); one 256-thread block per waveform.
struct ExtraArgs {
    const float2* s;
    const WaveDesc* waves;
    const Part* parts;
    const float* energy;
    const float2* tw;     // exp(-j 2 pi i / MMAX)
    int log2_mmax;
    int psl;              // compute the hard-PSL part
    float w_psl;
    int spec;             // compute the spectral part
    float w_spec;
    int wterms;           // compute var(|s|) and the smoothness term
    float w_const, w_smooth;
    float2* g_extra;      // gradient out (the weighted sum of the parts); nullable
    float* vals;          // [B][4] out
    float* spec_out;      // [B] spectral variance out (nullable)
};
hipError_t launch_extra(const ExtraArgs& a, int batch, int max_n, hipStream_t st);
// Spectral-mask projection (Sec. 6.2): out = IDFT_N(mask . DFT_N(s)), then,
// with unit, out / |out|; mask null: only the unit-circle projection.  One
// 256-thread block per waveform; out may alias s.
struct ProjectArgs {
    const float2* s;
    const WaveDesc* waves;
    const float* mask;    // packed like s, nullable
    int unit;
    float2* out;
};
hipError_t launch_project(const ProjectArgs& a, int batch, int max_n, hipStream_t st);
// out[i] = sum_s lambdas[s] grids[s * cells + i], in scenario order
hipError_t launch_combine(const float* grids, const float* lambdas, int n_scen, int64_t cells, float* out,
                          hipStream_t st);

// Cross-ambiguity of s and u (af_cross.hip), over the plan's segments of one
// size class; slabs and records are laid out like the auto-AF's
struct CrossArgs {
    const float2* s;
    const float2* u;
    const WaveDesc* waves;
    const SegDesc* segs;
    const float2* tw;     // exp(-j 2 pi i / MMAX)
    int log2_mmax;
    float eps;
    float* mag;           // forward: [grid] a, nullable
    float2* chi;          // forward: [grid] chi_su, nullable
    float* energy;        // [B][2] = E_s, E_u (written by the segment holding lag 0), nullable in the forward
    const float* grad_mag;  // backward: [grid] dL/da
    float2* slab_s;       // backward: per-segment dL/d conj(s) slabs
    float2* slab_u;       // backward: per-segment dL/d conj(u) slabs
    double* part;         // backward: per-segment sum of g_a p / a
    float2* grad_s;       // reduction outputs, packed like s
    float2* grad_u;
};
bool cross_lg_supported(int lg, int circ);
hipError_t launch_cross(int mode, int lg, int circ, const CrossArgs& a, int grid, hipStream_t st);
hipError_t launch_cross_reduce(const CrossArgs& a, int batch, int max_n, hipStream_t st);

// launchers (af_reduce.hip)
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st);
hipError_t launch_reduce_adam(const ReduceArgs& a, hipStream_t st);
hipError_t launch_phase_to_signal(const float* phi, float2* s, int64_t count, hipStream_t st);

// Kernel variants.  Variant v at transform size MH = 2^lg (M = 2 MH): fits
// tells whether an instance exists; its dynamic LDS is fft_lds bytes plus,
// when s_lds, s_bytes for the samples (and whatever shares their region).
struct VariantInfo {
    int lo, hi, p, split, wgs, s_lds, fits, fft_lds, nacc, s_bytes;
    int circ;  // has periodic-AF instances
};
constexpr int kNumVariants = 7;
// Variant 6 is the one-launch kernel: every size class of a plan (M = 128 to
// 8192, one lag kind) in one persistent launch over a single longest-first
// work queue, each work group taking the next item with an atomic ticket.
constexpr int kUnionVariant = 6;
VariantInfo variant_info(int v, int lg);
int variant_max_resident(int mode, int variant, int lg, int circ, int dyn_lds_bytes);
hipError_t launch_af(int mode, int variant, int lg, int circ, const AfArgs& a, int grid, int dyn_lds_bytes,
                     hipStream_t st);
// zero the one-launch kernel's ticket counter (a kernel, so that graph
// capture records no memset node)
hipError_t launch_queue_reset(int* queue, hipStream_t st);

}  // namespace graf
