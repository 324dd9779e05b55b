// Gradient reduction, fused Adam on phases and small elementwise kernels,
// plus the launch helpers for every kernel of the library.
#include <algorithm>

#include "af_reduce.h"

namespace graf {

__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a) {
    __shared__ double sh[20];
    __shared__ float2 sh2[256];
    reduce_chunk<false>(a, (int)blockIdx.x, 0, sh, sh2);
}

// Reduce, then one Adam step with step number *step + 1; the counter itself
// is advanced by step_advance_kernel afterwards (a completion counter that
// every block bumps would serialise thousands of device-scope atomics and
// cache write-backs on one address).
__global__ __launch_bounds__(256) void reduce_adam_kernel(ReduceArgs a) {
    __shared__ double sh[20];
    __shared__ float2 sh2[256];
    reduce_chunk<true>(a, (int)blockIdx.x, *a.step, sh, sh2);
}

__global__ void step_advance_kernel(int* step) { *step += 1; }

__global__ __launch_bounds__(256) void phase_to_signal_kernel(const float* phi, float2* s, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) {
        float sn, cs;
        sincosf(phi[i], &sn, &cs);
        s[i] = make_float2(cs, sn);
    }
}

// Sum over a 256-thread block in a fixed order (wavefront sums, then the four
// waves in order); every thread gets the result.
__device__ float block_sum256(float v, float* sh) {
    v = wave_allsum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// The experiment loss's per-waveform terms (Sec. 7.1.1, Eq. 18 as a power
// ratio): the hard-PSL maximum over the segment records (larger power, then
// the smaller cell index), chi at that cell by its defining sum, and the
// subgradient there, dp/d conj(chi) = chi / E^2 with dPSL/dE = -2 PSL / E,
// through the single-cell lag-product adjoint; and the spectral variance
// V = var(P / sum P) of the N-point spectrum X of s with
// dV/d conj(s[n]) = sum_j c_j X_j e^{+j 2 pi j n / N},
// c_j = 2 (x_j - sum x^2) / (N S).  The waveform-only terms of the
// composite loss (Sec. 5.2): var(|s|) with gradient (|s[n]| - mu) s[n] /
// (N |s[n]|), and the smoothness sum |s[n+1] - s[n]|^2 / E with gradient
// (d[n-1] - d[n]) / E - (smoothness) s[n] / E, d[n] = s[n+1] - s[n]; they
// read s from global memory.  Dynamic LDS: the samples for the hard PSL and
// the spectral part, the N twiddles and c_j X_j for the spectral part
// (up to 3 N complex64).
__global__ __launch_bounds__(256) void extra_kernel(ExtraArgs a) {
    extern __shared__ float2 xs[];
    __shared__ float sh[4];
    __shared__ float shp[4];
    __shared__ int shi[4];
    const int b = blockIdx.x, t = threadIdx.x;
    const WaveDesc w = a.waves[b];
    const int N = w.n;
    const float2* __restrict__ s = a.s + w.s_off;
    float2* sv = xs;
    float2* twn = xs + N;
    float2* cx = xs + 2 * N;
    if (a.psl || a.spec)
        for (int p = t; p < N; p += 256) sv[p] = s[p];
    if (a.spec) {
        for (int r = t; r < N; r += 256) {
            float sn, cs;
            sincospif(2.f * (float)r / (float)N, &sn, &cs);
            twn[r] = make_float2(cs, -sn);  // exp(-j 2 pi r / N)
        }
    }
    __syncthreads();

    // ---- hard PSL: the maximising cell and chi there
    float pmax = -1.f;
    int tau = 0, kst = 0;
    float2 G = make_float2(0.f, 0.f);
    float E = 1.f;
    const int M = w.m;
    const int RL = w.circ ? N : M;
    const int tsh = a.log2_mmax - w.log2m;
    if (a.psl) {
        float bp = -1.f;
        int bi = 0x7fffffff;
        for (int j = t; j < w.seg_count; j += 256) {
            const Part pr = a.parts[w.seg_begin + j];
            if (pr.psl_p > bp || (pr.psl_p == bp && pr.psl_i < bi)) {
                bp = pr.psl_p;
                bi = pr.psl_i;
            }
        }
        const float wm = wave_allmax(bp);
        bi = wave_allmin_int(bp == wm ? bi : 0x7fffffff);
        __syncthreads();
        if ((t & 63) == 0) {
            shp[t >> 6] = wm;
            shi[t >> 6] = bi;
        }
        __syncthreads();
        int ci = shi[0];
        pmax = shp[0];
        for (int i = 1; i < 4; ++i)
            if (shp[i] > pmax || (shp[i] == pmax && shi[i] < ci)) {
                pmax = shp[i];
                ci = shi[i];
            }
        tau = ci / RL;
        kst = ci - tau * RL;
        // chi(tau, k*) = sum_n s[n] conj(s[n - tau]) w^{k* n}: aperiodic over
        // n in [tau, N) with w = w_M; periodic over every n with the partner
        // index modulo N and w = w_N = w_M^2
        float2 c = make_float2(0.f, 0.f);
        for (int n = t; n < N; n += 256) {
            int m;
            if (w.circ) {
                m = n >= tau ? n - tau : n - tau + N;
            } else {
                if (n < tau) continue;
                m = n - tau;
            }
            const int ti = (int)(((int64_t)kst * n * (w.circ ? 2 : 1)) & (M - 1));
            c = cadd(c, cmul(cmulc(sv[n], sv[m]), a.tw[ti << tsh]));
        }
        c.x = block_sum256(c.x, sh);
        c.y = block_sum256(c.y, sh);
        E = a.energy[b];
        const float invE2 = 1.f / (E * E);
        G = make_float2(c.x * invE2, c.y * invE2);
    }

    // ---- spectral variance of the N-point spectrum
    float V = 0.f;
    if (a.spec) {
        float ps = 0.f;
        for (int j = t; j < N; j += 256) {
            // X_j = sum_n s[n] w_N^{j n}: the twiddle index j n mod N advances by j
            float2 x = make_float2(0.f, 0.f);
            int r = 0;
            for (int n = 0; n < N; ++n) {
                x = cadd(x, cmul(sv[n], twn[r]));
                r += j;
                r = r >= N ? r - N : r;
            }
            cx[j] = x;
            ps += cabs2(x);
        }
        const float S = block_sum256(ps, sh);
        const float invS = 1.f / S, invN = 1.f / (float)N;
        float q2 = 0.f, dv = 0.f;
        for (int j = t; j < N; j += 256) {
            const float x = cabs2(cx[j]) * invS;
            q2 = fmaf(x, x, q2);
            dv = fmaf(x - invN, x - invN, dv);
        }
        const float sx2 = block_sum256(q2, sh);
        V = block_sum256(dv, sh) * invN;
        const float cs = 2.f * invN * invS;
        for (int j = t; j < N; j += 256) {
            const float x = cabs2(cx[j]) * invS;
            cx[j] = cscale(cx[j], cs * (x - sx2));
        }
        __syncthreads();
    }

    // ---- var(|s|) and the smoothness term: mean modulus, energy and the
    // sum of squared steps, then the squared deviations from the mean
    float mu = 0.f, Es = 1.f, varc = 0.f, smooth = 0.f;
    if (a.wterms) {
        float r1 = 0.f, e1 = 0.f, d1 = 0.f;
        for (int p = t; p < N; p += 256) {
            const float2 x = s[p];
            const float q = cabs2(x);
            r1 += __builtin_amdgcn_sqrtf(q);
            e1 += q;
            if (p + 1 < N) d1 += cabs2(csub(s[p + 1], x));
        }
        mu = block_sum256(r1, sh) / (float)N;
        Es = block_sum256(e1, sh);
        smooth = block_sum256(d1, sh) / Es;
        float v1 = 0.f;
        for (int p = t; p < N; p += 256) {
            const float d = __builtin_amdgcn_sqrtf(cabs2(s[p])) - mu;
            v1 = fmaf(d, d, v1);
        }
        varc = block_sum256(v1, sh) / (float)N;
    }

    // ---- gradient: w_psl (single-cell adjoint + energy term) + w_spec dV/d conj(s)
    // + w_const dvar/d conj(s) + w_smooth dSmooth/d conj(s)
    if (a.g_extra) {
        for (int p = t; p < N; p += 256) {
            float2 g = make_float2(0.f, 0.f);
            if (a.psl) {
                // Q(n) = G e^{+j 2 pi k* n / RL}
                auto Q = [&](int n) {
                    const int ti = (int)(((int64_t)kst * n * (w.circ ? 2 : 1)) & (M - 1));
                    return cmulc(G, a.tw[ti << tsh]);
                };
                float2 gp = make_float2(0.f, 0.f);
                if (w.circ) {
                    const int lo = p >= tau ? p - tau : p - tau + N;
                    const int hi = p + tau < N ? p + tau : p + tau - N;
                    gp = cadd(cmul(Q(p), sv[lo]), cmul(cconj(Q(hi)), sv[hi]));
                } else {
                    if (p >= tau) gp = cmul(Q(p), sv[p - tau]);
                    if (p + tau < N) gp = cadd(gp, cmul(cconj(Q(p + tau)), sv[p + tau]));
                }
                const float de = -2.f * pmax / E;
                gp.x = fmaf(de, sv[p].x, gp.x);
                gp.y = fmaf(de, sv[p].y, gp.y);
                g = cscale(gp, a.w_psl);
            }
            if (a.spec) {
                float2 x = make_float2(0.f, 0.f);
                int r = 0;  // j p mod N
                for (int j = 0; j < N; ++j) {
                    x = cadd(x, cmulc(cx[j], twn[r]));
                    r += p;
                    r = r >= N ? r - N : r;
                }
                g = cadd(g, cscale(x, a.w_spec));
            }
            if (a.wterms) {
                const float2 x = s[p];
                const float r = __builtin_amdgcn_sqrtf(cabs2(x));
                const float cc = r > 0.f ? a.w_const * (r - mu) / ((float)N * r) : 0.f;
                const float invE = 1.f / Es;
                float2 ds = cscale(x, -smooth * invE);
                if (p > 0) ds = cadd(ds, cscale(csub(x, s[p - 1]), invE));
                if (p + 1 < N) ds = csub(ds, cscale(csub(s[p + 1], x), invE));
                g = cadd(g, cadd(cscale(x, cc), cscale(ds, a.w_smooth)));
            }
            a.g_extra[w.s_off + p] = g;
        }
    }
    if (t == 0) {
        if (a.vals) {
            a.vals[4 * b] = a.psl ? pmax : 0.f;
            a.vals[4 * b + 1] = V;
            a.vals[4 * b + 2] = varc;
            a.vals[4 * b + 3] = smooth;
        }
        if (a.spec_out) a.spec_out[b] = V;
    }
}

// Spectral-mask projection of projected descent (Sec. 6.2): X = DFT_N(s)
// by its definition (the twiddle index j n mod N advances by j), Y = mask X,
// out = IDFT_N(Y) / N; with unit, out / |out| (1 where it is 0).  Without a
// mask only the unit-circle projection runs.  Dynamic LDS: samples, the N
// twiddles and Y (3 N complex64).  Every sample is read into LDS before the
// first store, so out may alias s.
__global__ __launch_bounds__(256) void project_kernel(ProjectArgs a) {
    extern __shared__ float2 xs[];
    const int b = blockIdx.x, t = threadIdx.x;
    const WaveDesc w = a.waves[b];
    const int N = w.n;
    const float2* s = a.s + w.s_off;  // may alias out
    float2* out = a.out + w.s_off;
    auto unit = [&](float2 y) {
        const float r2 = cabs2(y);
        return r2 > 0.f ? cscale(y, __builtin_amdgcn_rsqf(r2)) : make_float2(1.f, 0.f);
    };
    if (!a.mask) {
        for (int p = t; p < N; p += 256) out[p] = a.unit ? unit(s[p]) : s[p];
        return;
    }
    const float* __restrict__ mask = a.mask + w.s_off;
    float2* sv = xs;
    float2* twn = xs + N;
    float2* yv = xs + 2 * N;
    for (int p = t; p < N; p += 256) {
        sv[p] = s[p];
        float sn, cs;
        sincospif(2.f * (float)p / (float)N, &sn, &cs);
        twn[p] = make_float2(cs, -sn);  // exp(-j 2 pi p / N)
    }
    __syncthreads();
    for (int j = t; j < N; j += 256) {
        float2 x = make_float2(0.f, 0.f);
        int r = 0;
        for (int n = 0; n < N; ++n) {
            x = cadd(x, cmul(sv[n], twn[r]));
            r += j;
            r = r >= N ? r - N : r;
        }
        yv[j] = cscale(x, mask[j] / (float)N);
    }
    __syncthreads();
    for (int p = t; p < N; p += 256) {
        float2 y = make_float2(0.f, 0.f);
        int r = 0;  // j p mod N
        for (int j = 0; j < N; ++j) {
            y = cadd(y, cmulc(yv[j], twn[r]));
            r += p;
            r = r >= N ? r - N : r;
        }
        out[p] = a.unit ? unit(y) : y;
    }
}

// ------------------------------------------------------------ launchers --
void* variant_kernel_0(int mode, int lg, int circ);
void* variant_kernel_1(int mode, int lg, int circ);
void* variant_kernel_2(int mode, int lg, int circ);
void* variant_kernel_3(int mode, int lg, int circ);
void* variant_kernel_4(int mode, int lg, int circ);
void* variant_kernel_5(int mode, int lg, int circ);
void* variant_kernel_6(int mode, int lg, int circ);
VariantInfo variant_info_0(int lg);
VariantInfo variant_info_1(int lg);
VariantInfo variant_info_2(int lg);
VariantInfo variant_info_3(int lg);
VariantInfo variant_info_4(int lg);
VariantInfo variant_info_5(int lg);
VariantInfo variant_info_6(int lg);

VariantInfo variant_info(int v, int lg) {
    switch (v) {
        case 0: return variant_info_0(lg);
        case 1: return variant_info_1(lg);
        case 2: return variant_info_2(lg);
        case 3: return variant_info_3(lg);
        case 4: return variant_info_4(lg);
        case 5: return variant_info_5(lg);
        case 6: return variant_info_6(lg);
    }
    return VariantInfo{};
}

static void* kernel_for(int mode, int variant, int lg, int circ) {
    switch (variant) {
        case 0: return variant_kernel_0(mode, lg, circ);
        case 1: return variant_kernel_1(mode, lg, circ);
        case 2: return variant_kernel_2(mode, lg, circ);
        case 3: return variant_kernel_3(mode, lg, circ);
        case 4: return variant_kernel_4(mode, lg, circ);
        case 5: return variant_kernel_5(mode, lg, circ);
        case 6: return variant_kernel_6(mode, lg, circ);
    }
    return nullptr;
}

int variant_max_resident(int mode, int variant, int lg, int circ, int dyn_lds_bytes) {
    const VariantInfo vi = variant_info(variant, lg);
    void* k = (vi.fits && (!circ || vi.circ)) ? kernel_for(mode, variant, lg, circ) : nullptr;
    if (!k) return 0;
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_lds_bytes) != hipSuccess) return 0;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, vi.wgs, dyn_lds_bytes) != hipSuccess) return 0;
    return blocks;
}

hipError_t launch_af(int mode, int variant, int lg, int circ, const AfArgs& a, int grid, int dyn_lds_bytes,
                     hipStream_t st) {
    const VariantInfo vi = variant_info(variant, lg);
    void* k = (vi.fits && (!circ || vi.circ)) ? kernel_for(mode, variant, lg, circ) : nullptr;
    if (!k || grid <= 0) return hipErrorInvalidValue;
    void* args[] = {(void*)&a};
    return hipLaunchKernel(k, dim3(grid), dim3(vi.wgs), args, (size_t)dyn_lds_bytes, st);
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st) {
    if (a.n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_kernel, dim3(a.n_blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_reduce_adam(const ReduceArgs& a, hipStream_t st) {
    if (a.n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_adam_kernel, dim3(a.n_blocks), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(step_advance_kernel, dim3(1), dim3(1), 0, st, a.step);
    return hipGetLastError();
}

hipError_t launch_extra(const ExtraArgs& a, int batch, int max_n, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    const int lds = (a.spec ? 3 : (a.psl ? 1 : 0)) * max_n * (int)sizeof(float2);
    static bool attr = false;
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute((const void*)extra_kernel,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 3 * 4096 * 8);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(extra_kernel, dim3(batch), dim3(256), (size_t)lds, st, a);
    return hipGetLastError();
}

hipError_t launch_project(const ProjectArgs& a, int batch, int max_n, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    const int lds = a.mask ? 3 * max_n * (int)sizeof(float2) : 0;
    static bool attr = false;
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute((const void*)project_kernel,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 3 * 4096 * 8);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(project_kernel, dim3(batch), dim3(256), (size_t)lds, st, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void combine_kernel(const float* __restrict__ grids,
                                                     const float* __restrict__ lambdas, int n_scen, int64_t cells,
                                                     float* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < cells; i += (int64_t)gridDim.x * 256) {
        float acc = 0.f;
        for (int s = 0; s < n_scen; ++s) acc = fmaf(lambdas[s], grids[(int64_t)s * cells + i], acc);
        out[i] = acc;
    }
}

hipError_t launch_combine(const float* grids, const float* lambdas, int n_scen, int64_t cells, float* out,
                          hipStream_t st) {
    if (cells <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((cells + 255) / 256, 8192);
    hipLaunchKernelGGL(combine_kernel, dim3((unsigned)blocks), dim3(256), 0, st, grids, lambdas, n_scen, cells, out);
    return hipGetLastError();
}

hipError_t launch_phase_to_signal(const float* phi, float2* s, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(phase_to_signal_kernel, dim3((unsigned)blocks), dim3(256), 0, st, phi, s, count);
    return hipGetLastError();
}

}  // namespace graf
