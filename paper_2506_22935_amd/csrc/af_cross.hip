// Cross-ambiguity of two waveforms s and u of one length N:
//   chi_su[tau, k] = sum_n s[n] conj(u[n - tau]) e^{-j 2 pi k n / M},
// the cross-AF / MIMO extension that the paper's limitations section names
// (chi_su = chi when u = s), with the magnitude
//   a = sqrt(|chi_su|^2 / (E_s E_u) + eps)   (|chi_su|^2 <= E_s E_u)
// and the backward from an upstream dL/da for both inputs.
//
// One 256-thread work group per segment of the plan's lag list (lags
// [tau_begin, tau_end), tau >= 0); each lag gives rows +tau and -tau.  Unlike
// the auto-AF, the two rows are not conjugate mirrors, so every row is the
// M-point DFT of its own lag product x[n] = s[n] conj(u[n - tau]) (n is the
// absolute sample index: no phase correction), taken as the two MH-point
// transforms of the even and odd bins (M = 2 MH >= 2N).  Lane groups of
// MH/16 lanes take one row each per iteration, both halves in turn.
//
// Backward: per cell G = g_a chi / (2 E_s E_u a); Q[n] = sum_k G[k]
// e^{+j 2 pi k n / M} is the inverse of the even half plus w_M^{-n} times the
// inverse of the odd half, and the two halves land in the same lanes.  The
// groups leave Q in LDS, and after a barrier every thread gathers, for the
// samples it owns, dL/d conj(s[n]) += u[n - tau] Q[n] and
// dL/d conj(u[n]) += s[n + tau] conj(Q[n + tau]) over the iteration's rows
// (the gather splits into two outputs).  Per-segment slabs of both, and the
// segment's sum of g_a p / a, are added in a fixed order by xreduce_kernel,
// which applies dL/dE_s = -sum g_a p / (2 a E_s) (and E_u alike).
//
// CIRC: the periodic cross-AF of N = MH samples (sample indices modulo N, N
// Doppler bins, grid [N][N] with row tau in [0, N)): lag tau of the plan's
// list (tau in [0, N/2]) gives rows tau and N - tau, each one N-point
// transform (the even half of the M = 2N split), and the gather takes its
// indices modulo N.
#include "af_internal.h"
#include "af_device.h"

namespace graf {
namespace {

constexpr int XP = 16;     // points per lane
constexpr int XWGS = 256;  // threads per work group

__device__ float xblock_sum(float v, float* sh) {
    v = wave_allsum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

template <int LG>
struct XShape {
    static constexpr int MH = 1 << LG;
    static constexpr int L = MH / XP;    // lanes per group
    static constexpr int G = XWGS / L;   // groups (rows per iteration)
    static constexpr int BUF = LdsSize<MH>::value;
    static constexpr int NJ = (MH + XWGS - 1) / XWGS;  // samples owned per thread
    static constexpr int lds_bytes() { return (G * BUF + 2 * MH) * 8; }
};

template <int MODE, int LG, bool CIRC>
__global__ __launch_bounds__(XWGS) void xaf_kernel(CrossArgs a) {
    using S = XShape<LG>;
    constexpr int MH = S::MH, L = S::L, G = S::G, BUF = S::BUF, NJ = S::NJ;
    static_assert(L >= 1 && G >= 1 && G * L == XWGS, "lane groups must tile the work group");
    extern __shared__ float2 dyn[];
    __shared__ float shf[8];
    __shared__ double shd[4];
    float2* sv = dyn + G * BUF;  // s, zero past N
    float2* uv = sv + MH;        // u, zero past N

    const SegDesc sg = a.segs[blockIdx.x];
    const WaveDesc w = a.waves[sg.wave];
    const int N = w.n, T = w.T;
    constexpr int M = 2 * MH;
    const int tid = threadIdx.x;
    const int grp = tid / L;
    const int l = tid - grp * L;
    float2* buf = dyn + grp * BUF;
    const TwTable twl{a.tw, a.log2_mmax - w.log2m};

    float es = 0.f, eu = 0.f;
    for (int i = tid; i < MH; i += XWGS) {
        const float2 x = i < N ? a.s[w.s_off + i] : make_float2(0.f, 0.f);
        const float2 y = i < N ? a.u[w.s_off + i] : make_float2(0.f, 0.f);
        sv[i] = x;
        uv[i] = y;
        es += cabs2(x);
        eu += cabs2(y);
    }
    const float Es = xblock_sum(es, shf);
    const float Eu = xblock_sum(eu, shf + 4);
    const float invEE = 1.f / (Es * Eu);
    if (sg.tau_begin == 0 && tid == 0 && a.energy) {
        a.energy[2 * sg.wave] = Es;
        a.energy[2 * sg.wave + 1] = Eu;
    }

    float2 gs[NJ], gu[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) gs[j] = gu[j] = make_float2(0.f, 0.f);
    float qsum = 0.f;
    // a lane group within one wavefront (L divides 64) orders its own LDS
    // accesses; larger groups synchronise the work group
    auto sync = []() {
        if constexpr (L <= 64) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __syncthreads();
        }
    };
    // job j of the segment: lag tau_begin + j/2, sign + (j even) or - (j odd);
    // periodic: the row N - lag for the minus sign (none for lags 0 and N/2)
    auto job_tau = [&](int job, bool& active) {
        const int lag = sg.tau_begin + (job >> 1);
        const bool neg = (job & 1) != 0;
        active = job < 2 * (sg.tau_end - sg.tau_begin) && !(neg && (lag == 0 || (CIRC && 2 * lag == N)));
        return active ? (neg ? (CIRC ? N - lag : -lag) : lag) : 0;
    };

    const int jobs = 2 * (sg.tau_end - sg.tau_begin);
    for (int j0 = 0; j0 < jobs; j0 += G) {
        bool active;
        const int tau = job_tau(j0 + grp, active);
        const int64_t row = CIRC ? w.grid_off + (int64_t)tau * MH : w.grid_off + (int64_t)(T + tau) * M;
        float2 qa[XP];
        // the forward writes bins 2(l + qL) and 2(l + qL) + 1 of the row (the
        // two halves) as one 8-byte pair, holding the even half's magnitudes
        // until the odd half's are known (the backward's upstream reads stay
        // per bin: reading pairs and holding the odd half measured slower)
        float hold[XP];
#pragma unroll
        for (int h = 0; h < (CIRC ? 1 : 2); ++h) {
            float2 v[XP];
#pragma unroll
            for (int r = 0; r < XP; ++r) {
                const int n = l + r * L;
                if constexpr (CIRC) {
                    // u[(n - tau) mod N], N = MH
                    const float2 x = cmulc(sv[n], uv[(n - tau) & (MH - 1)]);
                    v[r] = active ? x : make_float2(0.f, 0.f);
                } else {
                    const int j = n - tau;
                    const bool in = active && n < N && j >= 0 && j < N;
                    float2 x = cmulc(sv[n], uv[in ? j : 0]);
                    x = in ? x : make_float2(0.f, 0.f);
                    if (h) x = cmul(x, twl(n));
                    v[r] = x;
                }
            }
            fft_group<MH, XP, -1>(v, buf, l, twl, sync);
#pragma unroll
            for (int q = 0; q < XP; ++q) {
                const int k = CIRC ? l + q * L : 2 * (l + q * L) + h;
                const float pw = cabs2(v[q]) * invEE;
                if constexpr (MODE == 0) {
                    const float av = __builtin_amdgcn_sqrtf(pw + a.eps);
                    if (CIRC) {
                        if (active && a.mag) a.mag[row + k] = av;
                    } else if (h == 0) {
                        hold[q] = av;
                    } else if (active && a.mag) {
                        *reinterpret_cast<float2*>(a.mag + row + 2 * (l + q * L)) = make_float2(hold[q], av);
                    }
                    if (active && a.chi) a.chi[row + k] = v[q];
                } else {
                    const float g = active ? a.grad_mag[row + k] : 0.f;
                    const float ia = __builtin_amdgcn_rsqf(pw + a.eps);
                    qsum = fmaf(g * pw, ia, qsum);
                    v[q] = cscale(v[q], 0.5f * g * invEE * ia);
                }
            }
            if constexpr (MODE == 1) {
                fft_group<MH, XP, +1>(v, buf, l, twl, sync);
#pragma unroll
                for (int q = 0; q < XP; ++q) {
                    if (h) v[q] = cmulc(v[q], twl(l + q * L));
                    qa[q] = h ? cadd(qa[q], v[q]) : v[q];
                }
            }
        }
        if constexpr (MODE == 1) {
            // Q of every group's row into its buffer, natural order
            __syncthreads();
#pragma unroll
            for (int q = 0; q < XP; ++q) buf[lds_index(l + q * L)] = qa[q];
            __syncthreads();
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) {
                const int i = tid + jj * XWGS;
                if (i >= N) continue;
                for (int g = 0; g < G; ++g) {
                    bool act;
                    const int tg = job_tau(j0 + g, act);
                    if (!act) continue;
                    const float2* Q = dyn + g * BUF;
                    if constexpr (CIRC) {
                        const int jm = (i - tg) & (MH - 1), jp = (i + tg) & (MH - 1);
                        gs[jj] = cadd(gs[jj], cmul(uv[jm], Q[lds_index(i)]));
                        gu[jj] = cadd(gu[jj], cmulc(sv[jp], Q[lds_index(jp)]));
                    } else {
                        const int jm = i - tg;
                        if (jm >= 0 && jm < N) gs[jj] = cadd(gs[jj], cmul(uv[jm], Q[lds_index(i)]));
                        const int jp = i + tg;
                        if (jp >= 0 && jp < N) gu[jj] = cadd(gu[jj], cmulc(sv[jp], Q[lds_index(jp)]));
                    }
                }
            }
            __syncthreads();
        }
    }

    if constexpr (MODE == 1) {
        const int64_t base = w.slab_off + (int64_t)(sg.rec - w.seg_begin) * N;
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            const int i = tid + jj * XWGS;
            if (i < N) {
                a.slab_s[base + i] = gs[jj];
                a.slab_u[base + i] = gu[jj];
            }
        }
        const double qw = wave_allsum((double)qsum);
        if ((tid & 63) == 0) shd[tid >> 6] = qw;
        __syncthreads();
        if (tid == 0) a.part[sg.rec] = (shd[0] + shd[1]) + (shd[2] + shd[3]);
    }
}

// Fixed-order sum over the work group's waves (every thread gets the total).
template <int WGS, typename T>
__device__ T xblock_sum_w(T v, T* sh) {
    v = wave_allsum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    T t = sh[0];
#pragma unroll
    for (int i = 1; i < WGS / 64; ++i) t += sh[i];
    return t;
}

// Transform sizes M = 16384 and 32768 (aperiodic): a row's lane group spans
// the whole work group (MH / 16 lanes), so a work group takes one row per
// iteration, both halves in turn.  The samples come from global memory
// through buffer resources over [0, N) (zero outside, which also zeroes the
// lag product beyond the overlap), the twiddles from the plan's table, and
// the backward accumulates each segment's two gradients in its slabs in
// global memory (each thread reads, adds and writes its own samples per row)
// instead of registers.
template <int MODE, int LG>
__global__ __launch_bounds__((1 << LG) / XP) void xaf_big_kernel(CrossArgs a) {
    constexpr int MH = 1 << LG, L = MH / XP, WGS = L, M = 2 * MH;
    constexpr int NJ = MH / WGS;  // samples owned per thread
    extern __shared__ float2 dyn[];
    __shared__ float shf[WGS / 64];
    __shared__ double shd[WGS / 64];
    const SegDesc sg = a.segs[blockIdx.x];
    const WaveDesc w = a.waves[sg.wave];
    const int N = w.n, T = w.T;
    const int tid = threadIdx.x;
    const int l = tid;
    float2* buf = dyn;
    const TwTable twl{a.tw, a.log2_mmax - w.log2m};
    const Rsrc s_rs = make_rsrc(a.s + w.s_off, (unsigned)N * 8u);
    const Rsrc u_rs = make_rsrc(a.u + w.s_off, (unsigned)N * 8u);

    float es = 0.f, eu = 0.f;
    for (int i = tid; i < N; i += WGS) {
        es += cabs2(buf_load2(s_rs, i * 8));
        eu += cabs2(buf_load2(u_rs, i * 8));
    }
    const float Es = xblock_sum_w<WGS>(es, shf);
    const float Eu = xblock_sum_w<WGS>(eu, shf);
    const float invEE = 1.f / (Es * Eu);
    if (sg.tau_begin == 0 && tid == 0 && a.energy) {
        a.energy[2 * sg.wave] = Es;
        a.energy[2 * sg.wave + 1] = Eu;
    }
    float2* const gs_sl = MODE == 1 ? a.slab_s + w.slab_off + (int64_t)(sg.rec - w.seg_begin) * N : nullptr;
    float2* const gu_sl = MODE == 1 ? a.slab_u + w.slab_off + (int64_t)(sg.rec - w.seg_begin) * N : nullptr;
    if constexpr (MODE == 1) {
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            const int i = tid + jj * WGS;
            if (i < N) {
                gs_sl[i] = make_float2(0.f, 0.f);
                gu_sl[i] = make_float2(0.f, 0.f);
            }
        }
    }
    float qsum = 0.f;
    auto sync = []() { __syncthreads(); };
    const int jobs = 2 * (sg.tau_end - sg.tau_begin);
    for (int job = 0; job < jobs; ++job) {
        const int lag = sg.tau_begin + (job >> 1);
        const bool neg = (job & 1) != 0;
        if (neg && lag == 0) continue;  // the same for the whole work group
        const int tau = neg ? -lag : lag;
        const int64_t row = w.grid_off + (int64_t)(T + tau) * M;
        float2 qa[XP];
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            float2 v[XP];
#pragma unroll
            for (int r = 0; r < XP; ++r) {
                const int n = l + r * L;
                // u[n - tau] is zero outside [0, N) (the range check), as is s[n]
                float2 x = cmulc(buf_load2(s_rs, n * 8), buf_load2(u_rs, (n - tau) * 8));
                if (h) x = cmul(x, twl(n));
                v[r] = x;
                if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
            }
            fft_group<MH, XP, -1, true>(v, buf, l, twl, sync);
#pragma unroll
            for (int q = 0; q < XP; ++q) {
                const int k = 2 * (l + q * L) + h;
                const float pw = cabs2(v[q]) * invEE;
                if constexpr (MODE == 0) {
                    if (a.mag) a.mag[row + k] = __builtin_amdgcn_sqrtf(pw + a.eps);
                    if (a.chi) a.chi[row + k] = v[q];
                } else {
                    const float g = a.grad_mag[row + k];
                    const float ia = __builtin_amdgcn_rsqf(pw + a.eps);
                    qsum = fmaf(g * pw, ia, qsum);
                    v[q] = cscale(v[q], 0.5f * g * invEE * ia);
                }
            }
            if constexpr (MODE == 1) {
                fft_group<MH, XP, +1, true>(v, buf, l, twl, sync);
#pragma unroll
                for (int q = 0; q < XP; ++q) {
                    if (h) v[q] = cmulc(v[q], twl(l + q * L));
                    qa[q] = h ? cadd(qa[q], v[q]) : v[q];
                }
            }
        }
        if constexpr (MODE == 1) {
            // Q of the row into the buffer, natural order, then the gather
            // into this thread's samples of the two slabs
            __syncthreads();
#pragma unroll
            for (int q = 0; q < XP; ++q) buf[lds_index(l + q * L)] = qa[q];
            __syncthreads();
#pragma unroll 4
            for (int jj = 0; jj < NJ; ++jj) {
                const int i = tid + jj * WGS;
                if (i >= N) break;
                float2 gsv = gs_sl[i], guv = gu_sl[i];
                // u[i - tau] is zero outside [0, N) (the range check)
                gsv = cadd(gsv, cmul(buf_load2(u_rs, (i - tau) * 8), buf[lds_index(i)]));
                const int jp = i + tau;
                if (jp >= 0 && jp < N) guv = cadd(guv, cmulc(buf_load2(s_rs, jp * 8), buf[lds_index(jp)]));
                gs_sl[i] = gsv;
                gu_sl[i] = guv;
            }
            __syncthreads();
        }
    }
    if constexpr (MODE == 1) {
        const double qw = xblock_sum_w<WGS>((double)qsum, shd);
        if (tid == 0) a.part[sg.rec] = qw;
    }
}

// dL/d conj(s) and dL/d conj(u): the waveform's slabs in segment order plus
// the energy terms; one thread per sample, blockIdx.y the waveform.
__global__ __launch_bounds__(256) void xreduce_kernel(CrossArgs a) {
    const int b = blockIdx.y;
    const WaveDesc w = a.waves[b];
    __shared__ double qs;
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int j = 0; j < w.seg_count; ++j) t += a.part[w.seg_begin + j];
        qs = t;
    }
    __syncthreads();
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= w.n) return;
    const float Es = a.energy[2 * b], Eu = a.energy[2 * b + 1];
    float2 gs = make_float2(0.f, 0.f), gu = make_float2(0.f, 0.f);
    for (int j = 0; j < w.seg_count; ++j) {
        const int64_t o = w.slab_off + (int64_t)j * w.n + i;
        gs = cadd(gs, a.slab_s[o]);
        gu = cadd(gu, a.slab_u[o]);
    }
    const float q = (float)qs;
    const float2 s = a.s[w.s_off + i], u = a.u[w.s_off + i];
    a.grad_s[w.s_off + i] = cadd(gs, cscale(s, -q / (2.f * Es)));
    a.grad_u[w.s_off + i] = cadd(gu, cscale(u, -q / (2.f * Eu)));
}

template <int MODE, int LG, bool CIRC>
hipError_t launch_lg(const CrossArgs& a, int grid, hipStream_t st) {
    static bool attr = false;
    const void* k = (const void*)xaf_kernel<MODE, LG, CIRC>;
    constexpr int lds = XShape<LG>::lds_bytes();
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((xaf_kernel<MODE, LG, CIRC>), dim3(grid), dim3(XWGS), (size_t)lds, st, a);
    return hipGetLastError();
}

template <int MODE, bool CIRC>
hipError_t launch_mode(int lg, const CrossArgs& a, int grid, hipStream_t st) {
    switch (lg) {
        case 6: return launch_lg<MODE, 6, CIRC>(a, grid, st);
        case 7: return launch_lg<MODE, 7, CIRC>(a, grid, st);
        case 8: return launch_lg<MODE, 8, CIRC>(a, grid, st);
        case 9: return launch_lg<MODE, 9, CIRC>(a, grid, st);
        case 10: return launch_lg<MODE, 10, CIRC>(a, grid, st);
        case 11: return launch_lg<MODE, 11, CIRC>(a, grid, st);
        case 12: return launch_lg<MODE, 12, CIRC>(a, grid, st);
    }
    return hipErrorInvalidValue;
}

template <int MODE, int LG>
hipError_t launch_big(const CrossArgs& a, int grid, hipStream_t st) {
    static bool attr = false;
    const void* k = (const void*)xaf_big_kernel<MODE, LG>;
    constexpr int lds = LdsSize<(1 << LG)>::value * 8;
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((xaf_big_kernel<MODE, LG>), dim3(grid), dim3((1 << LG) / XP), (size_t)lds, st, a);
    return hipGetLastError();
}

}  // namespace

bool cross_lg_supported(int lg, int circ) { return lg >= 6 && lg <= (circ ? 12 : 14); }

hipError_t launch_cross(int mode, int lg, int circ, const CrossArgs& a, int grid, hipStream_t st) {
    if (grid <= 0) return hipSuccess;
    if (!circ && lg == 13) return mode == 0 ? launch_big<0, 13>(a, grid, st) : launch_big<1, 13>(a, grid, st);
    if (!circ && lg == 14) return mode == 0 ? launch_big<0, 14>(a, grid, st) : launch_big<1, 14>(a, grid, st);
    if (circ) return mode == 0 ? launch_mode<0, true>(lg, a, grid, st) : launch_mode<1, true>(lg, a, grid, st);
    return mode == 0 ? launch_mode<0, false>(lg, a, grid, st) : launch_mode<1, false>(lg, a, grid, st);
}

hipError_t launch_cross_reduce(const CrossArgs& a, int batch, int max_n, hipStream_t st) {
    if (batch <= 0 || max_n <= 0) return hipSuccess;
    hipLaunchKernelGGL(xreduce_kernel, dim3((unsigned)((max_n + 255) / 256), (unsigned)batch), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace graf
