/*
 * graf_af.h -- C ABI of the MI355X differentiable ambiguity-function library
 * (libgraf_af.so).
 *
 * What is computed (paper "Differentiable Radar Ambiguity Functions", Sec. 4.1,
 * Eqs. 7-12, with aperiodic lags and the library FFT sign):
 *
 *   chi[tau, k] = sum_n s[n] conj(s[n - tau]) exp(-j 2 pi k n / M)
 *
 * for a complex waveform s of N samples (s[n] = 0 outside [0, N)), lags
 * tau in [-T, T] and Doppler bins k in [0, M).  The energy E = sum |s|^2 is the
 * value of chi at the origin and its maximum, so it is the normaliser of
 * Sec. 4.3 (Eq. 17).  The library returns the eps-stabilised magnitude
 *
 *   a[tau, k] = sqrt(|chi[tau, k]|^2 / E^2 + eps)
 *
 * and the conjugate Wirtinger gradient dL/d conj(s) (Sec. 3.3 Eq. 6, Sec. 4.2
 * Eqs. 13-15) of either a user loss given through dL/da, or the built-in loss
 *
 *   L = w_isl * ISL + w_psl * softPSL
 *   ISL     = sum over Omega_s of W[tau, k] |chi|^2 / E^2        (Eq. 19)
 *   softPSL = T_psl * log sum over Omega_s of exp(a / T_psl)     (smooth Eq. 18)
 *
 * where Omega_s is every cell outside the mainlobe |tau| <= h_tau, |k_c| <= h_k
 * (k_c = ((k + M/2) mod M) - M/2) and W is 1, or the separable shaping weight
 * u[floor(31 |tau| / N)] * v[floor(31 |k_c| / (M/2 + 1))] from 62 floats per
 * waveform (u = first 31, v = last 31).
 *
 * Conventions
 *  - Every pointer argument named "device" is device memory owned by the
 *    caller; the library never frees it.  Host structs are read during the
 *    call only.
 *  - complex64 = interleaved (re, im) float32.  A batch packs its waveforms
 *    into one complex64 array; waveform b starts at element waves[b].s_off.
 *  - Grids are row-major [2T+1][M] float32 (or complex64) starting at element
 *    waves[b].grid_off; row i holds tau = i - T, bins in natural DFT order
 *    (the centring of Algorithm 1, step 5, is left to the caller).
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream).  The status reports host-side validation and launch errors only.
 *  - Compute calls allocate nothing and never synchronise, so they can be
 *    captured in a HIP graph.  They use the caller's workspace; calls on one
 *    plan must not overlap in time (they share the plan's work-queue counters).
 *  - No exception crosses the ABI.  Zero energy gives NaN results, as 0/0.
 */
#ifndef GRAF_AF_H
#define GRAF_AF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AF_OK = 0,
    AF_ERR_INVALID_ARG = -1, /* null pointer, bad size, bad offset */
    AF_ERR_UNSUPPORTED = -2, /* M not a power of two, M < 2N, M > 32768, N too long for M; GEMM shape */
    AF_ERR_BUDGET = -3,      /* workspace cannot fit the budget even with recomputation */
    AF_ERR_HIP = -4,         /* a HIP runtime call failed */
    AF_ERR_WORKSPACE = -5,   /* workspace smaller than af_plan_workspace_size */
    AF_ERR_NO_DEVICE = -6    /* no usable gfx950 device */
} af_status;

/* af_wave.flags: the periodic (circular) AF of Sec. 3 Eq. 2 and Sec. 4.1
 * Eq. 7 / Algorithm 1 instead of the aperiodic one:
 *   chi[tau, k] = sum_{n<N} s[n] conj(s[(n - tau) mod N]) e^{-j 2 pi k n / N}
 * for tau, k in [0, N): requires m = n, max_lag = -1 or n - 1 and n a power
 * of two in [64, 4096] (AF_ERR_UNSUPPORTED otherwise); the grids are
 * [N][N] with row tau (no centring), the mainlobe is min(tau, N - tau) <=
 * h_tau, |k_c| <= h_k with k_c centred over N bins (h_tau, h_k <= N/2), and
 * the shaping weights use min(tau, N - tau) and N/2 + 1 in place of |tau| and
 * M/2 + 1.  Every call supports both kinds, also mixed in one batch. */
#define AF_WAVE_PERIODIC 1

/* One waveform of a batch. */
typedef struct {
    int32_t n;        /* samples, >= 1 */
    int32_t m;        /* Doppler bins: power of two with 2n <= m, 128 <= m <= 32768 (periodic: m = n) */
    int32_t max_lag;  /* T: lags -T..T with 0 <= T <= n - 1; -1 means n - 1 */
    int32_t h_tau;    /* mainlobe half-width in lags (built-in loss only) */
    int32_t h_k;      /* mainlobe half-width in Doppler bins (built-in loss only) */
    int32_t flags;    /* 0, or AF_WAVE_PERIODIC */
    int64_t s_off;    /* first complex64 sample of this waveform in the packed input */
    int64_t grid_off; /* first element of this waveform's grids ([2T+1][M], periodic [N][N]) */
} af_wave;

/* Plan options (zero-initialise, then set what you need). */
typedef struct {
    float eps;                 /* eps in a = sqrt(p + eps); e.g. 1e-12 */
    int32_t store_mode;        /* 0: decide by budget, 1: store spectra, 2: recompute */
    int64_t budget_bytes;      /* workspace budget; <= 0 means unlimited */
    int32_t variant;           /* -1: library default; >= 0 forces a kernel variant (6:
                                  the one-launch kernel, for every size class) */
    int32_t segment_iters;     /* lag iterations per work item; 0: planner's choice */
    int32_t loss_passes;       /* 0: af_loss / af_optim_step use one fused pass where the
                                  loss allows it; 1: always a forward then a backward pass */
    int32_t launch_mode;       /* 0: waveforms of several sizes (Doppler size classes,
                                  M <= 8192, one lag kind) run in one persistent launch
                                  over one longest-first work queue (variant 6); 1: one
                                  persistent launch per size class, the classes
                                  concurrent on library-owned streams (Sec. 4.3, batch
                                  processing) */
} af_plan_opts;

typedef struct af_plan af_plan;

/* Built-in loss parameters (Sec. 5.1).  band_w: device float[batch][62] or NULL.
 * psl_hard = 1 replaces the soft PSL by the hard PSL of Eq. 18 as a power
 * ratio, max over Omega_s of |chi|^2 / E^2, whose subgradient sits on one
 * maximising cell (the smallest cell index tau * row length + k on the
 * tau >= 0 row among equal powers; both cells of a (tau, k), (-tau, -k) pair
 * give the same gradient), weighted by w_psl.  w_spec weights the spectral
 * variance of Sec. 7.1.1, var_j(P_j / sum P) with P = |DFT_N(s)|^2 (the
 * N-point spectrum, population variance; N <= 4096).  The experiment loss
 * PSL + lambda * alpha * SpectralVariance is w_psl = 1, psl_hard = 1,
 * w_spec = lambda * alpha.  w_match weights L_match of the composite loss
 * (Sec. 5.2), the squared Frobenius distance between the AF in power,
 * p = |chi|^2 / E^2, and match_target over every cell of the grid; it
 * combines with ISL and the hard PSL, not with the soft PSL
 * (AF_ERR_UNSUPPORTED).  w_width weights the soft mainlobe width of
 * Eq. 21 on the AF in power, sum over the lag rows of |tau| sigma(gamma
 * (p(tau, 0) - 1/2)) (p(0, 0) = 1 for every waveform, so half of it is the
 * -3 dB level of Eq. 20; |tau| is min(tau, N - tau) on the periodic AF);
 * gamma >= 0 sets the sharpness; like L_match it does not combine with the
 * soft PSL.  The hard PSL, L_match, the width and the cell weights run on
 * every size class (M up to 32768).  w_const weights var(|s|) (L_const of
 * Sec. 5.2, population variance; its gradient is taken as 0 at s[n] = 0),
 * w_smooth a phase-continuity term (Sec. 6.2), sum_{n < N-1} |s[n+1] -
 * s[n]|^2 / E, which for a unit-modulus code is (2/N) sum (1 - cos of the
 * phase steps); both combine with every other term.  w_cell weights
 * sum over every cell of cell_w * p, with cell_w a device float grid of
 * per-cell weights laid out like the a grid (a target profile; the
 * multi-scenario loss of Eq. 24 over such profiles is one pass with the
 * combined grid, see af_scenario_combine); like L_match it needs split
 * classes and does not combine with the soft PSL.  Zero-initialise the
 * struct: psl_hard = 0 and zero weights for the terms after it give the
 * soft-PSL losses above. */
typedef struct {
    float w_isl;
    float w_psl;
    float psl_temp; /* > 0 */
    const float* band_w;
    int32_t psl_hard; /* 0 or 1 */
    float w_spec;
    const float* match_target; /* device float grid of target powers p_t, laid out like the a grid */
    float w_match;             /* weight of L_match = sum over every cell of (p - p_t)^2 */
    float w_width;             /* weight of the soft mainlobe width (Eq. 21) */
    float gamma;               /* its sharpness, >= 0 */
    float w_const;             /* weight of var(|s|) */
    float w_smooth;            /* weight of sum |s[n+1] - s[n]|^2 / E */
    const float* cell_w;       /* device float per-cell weight grid, laid out like the a grid */
    float w_cell;              /* weight of sum cell_w * p */
} af_loss_params;

/* Adam settings for af_optim_step (Kingma & Ba; eps outside the square root). */
typedef struct {
    float lr, beta1, beta2, eps;
} af_adam_params;

/* Plan summary for callers and benchmarks. */
typedef struct {
    int64_t cells;          /* sum over waveforms of (2T+1) * M */
    int64_t store_bytes;    /* bytes of stored spectra when storing */
    int64_t workspace_bytes;
    int32_t segments;       /* work items */
    int32_t grid;           /* persistent work groups launched */
    int32_t variant;        /* kernel variant in use */
    int32_t stores;         /* 1 when the backward reads stored spectra */
} af_plan_summary;

/* Create a plan for `batch` waveforms (host array `waves`).  Validates every
 * waveform, chooses a kernel variant and a work split, decides store versus
 * recompute against the budget, and uploads small device tables (twiddles,
 * work list).  May call hipMalloc; not capturable.  On error *out is NULL. */
af_status af_plan_create(int32_t batch, const af_wave* waves, const af_plan_opts* opts, af_plan** out);
void af_plan_destroy(af_plan* plan);

/* Bytes of caller-allocated device workspace the compute calls need. */
af_status af_plan_workspace_size(const af_plan* plan, size_t* bytes);
af_status af_plan_get_summary(const af_plan* plan, af_plan_summary* out);

/* Re-pick the schedule by timing candidates on this plan's shapes (forward +
 * fused ISL loss) with the given device inputs: every kernel variant that fits
 * each size class, the tuned classes together at one, two or four work items
 * per resident work group, and (several classes) one launch of all of them at
 * three, six or twelve items per group; the fastest is kept.  Synchronises
 * `stream`.  ws must hold af_plan_workspace_size bytes for a candidate to be
 * timed (larger ones are skipped).  Results are cached per device
 * architecture and plan shapes for the process, and, when the environment
 * variable GRAF_AF_TUNE_CACHE names a file, read from and appended to it; a
 * cached schedule is applied without timing (chosen_variant and best_ms then
 * report the cached choice).  Not capturable. */
af_status af_plan_autotune(af_plan* plan, const void* s, void* ws, size_t ws_bytes, void* stream,
                           int32_t* chosen_variant, float* best_ms);

/* Forward (Sec. 4.1).  s: device complex64 input.  mag: device float32 grids
 * of a (nullable).  chi: device complex64 grids of chi (nullable).  energy:
 * device float[batch] of E (nullable).  When the plan stores spectra, the
 * forward also leaves them in ws for af_backward. */
af_status af_forward(const af_plan* plan, const void* s, float* mag, void* chi, float* energy, void* ws,
                     size_t ws_bytes, void* stream);

/* Backward for a user loss (Sec. 4.2): grad_mag holds dL/da on the grids
 * (device float32); grad_s receives dL/d conj(s) (device complex64, packed like
 * s).  In store mode it reads the spectra the last af_forward on this plan
 * left in the same ws; otherwise it recomputes them from s. */
af_status af_backward(const af_plan* plan, const void* s, const float* grad_mag, void* grad_s, void* ws,
                      size_t ws_bytes, void* stream);

/* Built-in loss forward and backward.  terms: device float[batch][4] receiving
 * (L, ISL, softPSL, E) per waveform (nullable).  mag (nullable): the a grids.
 * grad_s (nullable: loss only): dL/d conj(s).  With w_psl == 0 one fused pass
 * does everything.  With w_psl != 0, one fused pass also does when band_w is
 * NULL, every waveform has the full lag window (or w_isl == 0), psl_temp >=
 * sqrt(1 + eps) log2(e) / 100 and the kernel variant splits the two half
 * transforms: the soft-PSL gradient leaves that pass without its global
 * normaliser, which the reduction applies.  Otherwise a forward pass finds the
 * normaliser first and a backward pass follows. */
af_status af_loss(const af_plan* plan, const void* s, const af_loss_params* loss, float* terms, float* mag,
                  void* grad_s, void* ws, size_t ws_bytes, void* stream);

/* af_loss for callers that cannot allocate device memory or take a
 * workspace argument (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same passes and results as af_loss,
 * with the workspace taken from a library-owned device array of 64 MiB per
 * GPU (held by each device that loads the library until the process ends).
 * Calls no hipMalloc or hipFree.  The plan must come from af_plan_create on
 * the same device; plans whose af_plan_workspace_size exceeds 64 MiB get
 * AF_ERR_WORKSPACE, and AF_ERR_HIP means the array could not be resolved on
 * that device.  Every call on one GPU shares that GPU's array and leaves its
 * contents behind (no call needs it zeroed: each pass writes what it later
 * reads), so calls that overlap on one GPU (other streams, other threads)
 * race and must be serialised by the caller. */
af_status af_loss_no_alloc(const af_plan* plan, const void* s, const af_loss_params* loss, float* terms, float* mag,
                           void* grad_s, void* stream);

/* One stage of af_loss on its own, for timing and profiling.  stage 0: the
 * forward pass (a grids and loss partials; with grad_s set and a loss that
 * allows it, the single fused pass instead); stage 1: the backward pass (only
 * when stage 0 was not fused; reads the partials of stage 0 from ws); stage
 * 2: the reduction into terms and grad_s.  Running stages 0, 1, 2 in order
 * equals one af_loss call. */
af_status af_loss_stage(const af_plan* plan, int32_t stage, const void* s, const af_loss_params* loss,
                        float* terms, float* mag, void* grad_s, void* ws, size_t ws_bytes, void* stream);

/* The spectral variance of Sec. 7.1.1 per waveform (see af_loss_params):
 * value: device float[batch]; grad_s (nullable): dV/d conj(s), packed like
 * s (overwritten).  Every waveform must have N <= 4096 (AF_ERR_UNSUPPORTED). */
af_status af_spectral_variance(const af_plan* plan, const void* s, float* value, void* grad_s, void* ws,
                               size_t ws_bytes, void* stream);

/* Projection step of projected descent (Sec. 6.2), per waveform of the plan:
 * with mask (device float, one real weight per bin of the N-point DFT, packed
 * like s) out = IDFT_N(mask * DFT_N(s)) (inverse with 1/N), which needs
 * N <= 4096 (AF_ERR_UNSUPPORTED otherwise); then, with unit = 1, out /= |out|
 * onto the unit circle (1 where out is 0).  mask NULL: only the unit-circle
 * projection (any N).  s, out: device complex64 packed like the plan's input;
 * out may equal s (in place).  unit must be 0 or 1; mask NULL with unit 0 copies. */
af_status af_project(const af_plan* plan, const void* s, const float* mask, int32_t unit, void* out, void* stream);

/* Multi-scenario weights (Eq. 24): out = sum_s lambdas[s] * grids[s], in
 * scenario order, over the plan's grid cells.  grids: device float
 * [n_scen][cells] (each laid out like the a grids); lambdas: device
 * float[n_scen]; out: device float[cells].  A loss that is linear in the
 * power grid per scenario (cell-weighted ISL, target profiles) then runs as
 * one pass with cell_w = out, whatever n_scen. */
af_status af_scenario_combine(const af_plan* plan, int32_t n_scen, const float* grids, const float* lambdas,
                              float* out, void* stream);

/* Cross-ambiguity of two waveforms (the cross-AF / MIMO extension that the
 * limitations section names): per waveform b of the plan, s and u are
 * device complex64 arrays packed like the plan's input (u[b] has the same N
 * as s[b]) and
 *   chi_su[tau, k] = sum_n s[n] conj(u[n - tau]) exp(-j 2 pi k n / M),
 * on the plan's grids ([2T+1][M], row tau + T), with a = sqrt(|chi_su|^2 /
 * (E_s E_u) + eps) (|chi_su|^2 <= E_s E_u; chi_su = chi when u = s).
 * Periodic waveforms (AF_WAVE_PERIODIC, Eq. 2's circular lags) take
 *   chi_su[tau, k] = sum_n s[n] conj(u[(n - tau) mod N]) exp(-j 2 pi k n / N)
 * on their [N][N] grids (row tau in [0, N)).  Aperiodic M up to 32768,
 * periodic N up to 4096 (every size a plan takes).  Grid offsets must be even and mag 8-byte
 * aligned (the aperiodic forward writes the a grids as pairs of bins);
 * AF_ERR_INVALID_ARG otherwise.
 * af_cross_forward: mag (a grids), chi (chi_su grids) and energy (device
 * float[batch][2] = E_s, E_u) are each nullable; no workspace.
 * af_cross_backward: grad_mag holds dL/da on the grids; grad_s and grad_u
 * receive dL/d conj(s) and dL/d conj(u) (overwritten, packed like s); ws is
 * device memory of af_cross_workspace_size bytes, 256-byte aligned
 * (AF_ERR_WORKSPACE when smaller).  Deterministic: no atomics. */
af_status af_cross_workspace_size(const af_plan* plan, size_t* bytes);
af_status af_cross_forward(const af_plan* plan, const void* s, const void* u, float* mag, void* chi, float* energy,
                           void* stream);
af_status af_cross_backward(const af_plan* plan, const void* s, const void* u, const float* grad_mag, void* grad_s,
                            void* grad_u, void* ws, size_t ws_bytes, void* stream);

/* s[i] = exp(j phi[i]) for i < count (device arrays). */
af_status af_phase_to_signal(const float* phi, void* s, int64_t count, void* stream);

/* One optimiser step on phases (Sec. 6.2 update, Sec. 7.1.2 optimiser):
 * loss and dL/d conj(s) at s, dL/dphi = 2 Im(conj(s) dL/d conj(s)), one Adam
 * step on phi (with m, v and the device int step counter, incremented on the
 * device), and s <- exp(j phi) in place.  s must equal exp(j phi) on entry
 * (af_phase_to_signal once before the first step).  terms: device
 * float[batch][4] (nullable) gets the loss terms at the entry point. */
af_status af_optim_step(const af_plan* plan, float* phi, float* adam_m, float* adam_v, void* s, int32_t* step,
                        const af_loss_params* loss, const af_adam_params* adam, float* terms, void* ws,
                        size_t ws_bytes, void* stream);

/* ---- proposal network (paper Sec. 6.1, Fig. 1: design parameters ->
 * network -> waveform -> ambiguity function -> loss) ----------------------
 * Dense layers run as BF16 MFMA GEMMs with FP32 accumulation.  All arrays are
 * device memory, row-major, contiguous; bf16 arrays hold IEEE bfloat16.
 *
 * af_gemm_bf16: C[m][n] = sum_k A~[m][k] B~[n][k] with
 *   layout 0 (X W^T): A [m][k] bf16, B [n][k] bf16
 *   layout 1 (dZ W):  A [m][k] bf16, B [k][n] bf16
 *   layout 2 (dZ^T A): A [k][m] bf16, B [k][n] bf16
 * and epilogue
 *   0: out_f32 = C
 *   1: out_f32 = C + bias[n]
 *   2: out_f32 = Z = C + bias[n]; out_bf16 = GELU(Z)   (exact erf GELU)
 *   3: out_f32 = dZ = C * GELU'(aux) ; out_bf16 = dZ     (aux = Z of the layer)
 * m and n must be multiples of 64, k a multiple of 64 (AF_ERR_UNSUPPORTED
 * otherwise); a, b and ws 16-byte aligned.
 * tile: 0 automatic, else BM x BN x BK of one work group's output tile and k
 * step: 1: 128x128x64, 2: 128x64x64, 3: 64x128x64, 4: 64x64x64, 5-8: the
 * same tiles with BK 128 (BM must divide m, BN n, BK k).  split_k: 0
 * automatic, or s in [1, 16] with k a multiple of BK s: the k range is cut
 * into s parts whose float32 partial sums (s * m * n floats in ws) are added
 * in part order by a second kernel that applies the epilogue, so results are
 * reproducible for a given (tile, split_k).  af_gemm_config resolves the
 * automatic choices for the current device and reports the workspace bytes
 * (0 without a split; ws may then be NULL). */
af_status af_gemm_config(int32_t m, int32_t n, int32_t k, int32_t tile, int32_t split_k, int32_t* tile_out,
                         int32_t* split_out, size_t* ws_bytes);
af_status af_gemm_bf16(int32_t layout, int32_t epilogue, int32_t m, int32_t n, int32_t k, const void* a,
                       const void* b, const float* bias, const float* aux, float* out_f32, void* out_bf16,
                       int32_t tile, int32_t split_k, void* ws, size_t ws_bytes, void* stream);

/* out[c] = sum over r of in[r][c] (float32): row chunks summed into ws, then
 * the chunk sums added in chunk order.  ws must hold
 * af_colsum_workspace_size bytes (device memory). */
af_status af_colsum_workspace_size(int32_t rows, int32_t cols, size_t* bytes);
af_status af_colsum(int32_t rows, int32_t cols, const float* in, float* out, void* ws, size_t ws_bytes,
                    void* stream);

/* One bias-corrected Adam step (step >= 1 is the 1-based step number) on
 * count float32 parameters; param_bf16 (nullable) receives their bfloat16
 * copy. */
af_status af_adam_update(int64_t count, float* param, const float* grad, float* m, float* v, int32_t step,
                         const af_adam_params* adam, void* param_bf16, void* stream);

/* out[i] = bfloat16(in[i]), round to nearest even. */
af_status af_to_bf16(int64_t count, const float* in, void* out, void* stream);

/* out[i] = dL/dphi_i = 2 Im(conj(s_i) grad_s_i) for s = exp(j phi) (complex64
 * s and grad_s = dL/d conj(s)); out_bf16 (nullable) gets its bfloat16 copy. */
af_status af_phase_grad(int64_t count, const void* s, const void* grad_s, float* out, void* out_bf16,
                        void* stream);

const char* af_status_string(af_status status);
int32_t af_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GRAF_AF_H */
