// Gradient reduction, fused Adam on phases and small elementwise kernels,
// plus the launch helpers for every kernel of the library.
#include "af_device.h"
#include "af_internal.h"

#include <math.h>

namespace graf {

constexpr float kLog2eR = 1.4426950408889634f;

__device__ __forceinline__ void lse_merge_r(float& m, double& s, float m2, double s2, float inv_t2) {
    float mn = fmaxf(m, m2);
    if (mn == -INFINITY) return;
    s = s * (double)exp2f((m - mn) * inv_t2) + s2 * (double)exp2f((m2 - mn) * inv_t2);
    m = mn;
}

// --------------------------------------------------------------- reduce --
// One block per (waveform, 256-sample chunk): sums the waveform's slabs in
// segment order, adds dL/dE * s, optionally writes the loss terms.
__device__ __forceinline__ void reduce_common(const ReduceArgs& a, int& wv, int& p, float2& g, float2& sp,
                                              float& loss, float& isl, float& soft, float& E) {
    const int2 ch = a.chunks[blockIdx.x];
    wv = ch.x;
    const WaveDesc w = a.waves[wv];
    p = ch.y + (int)threadIdx.x;
    const float inv_t2 = kLog2eR / a.temp;
    double isl_raw = 0.0, s = 0.0, dle = 0.0;
    float m = -INFINITY;
    for (int j = 0; j < w.seg_count; ++j) {
        const Part pr = a.parts[w.seg_begin + j];
        isl_raw += pr.isl;
        lse_merge_r(m, s, pr.lse_m, pr.lse_s, inv_t2);
        dle += pr.dle;
    }
    E = a.energy[wv];
    // complement waveforms carry ISL - M (Moyal: the full grid holds M E^2)
    const double isl_d = isl_raw + ((a.uniform_w && w.full_window) ? (double)w.m : 0.0);
    isl = (float)isl_d;
    soft = (s > 0.0) ? (float)((double)m + (double)a.temp * log(s)) : 0.f;
    loss = (float)((double)a.w_isl * isl_d + (a.w_psl != 0.f ? (double)a.w_psl * (double)soft : 0.0));
    // dL/dE of the ISL part is -2 w_isl (collected sum) / E in both forms
    const float dLdE = (float)(-2.0 * (double)a.w_isl * isl_raw / (double)E + dle);
    g = make_float2(0.f, 0.f);
    sp = make_float2(0.f, 0.f);
    if (p < w.n && !a.skip_slabs) {
        const float2* sl = a.slabs + w.slab_off + p;
        for (int j = 0; j < w.seg_count; ++j) g = cadd(g, sl[(int64_t)j * w.n]);
        sp = a.s[w.s_off + p];
        g.x = fmaf(dLdE, sp.x, g.x);
        g.y = fmaf(dLdE, sp.y, g.y);
    }
}

__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a) {
    int wv, p;
    float2 g, sp;
    float loss, isl, soft, E;
    reduce_common(a, wv, p, g, sp, loss, isl, soft, E);
    const WaveDesc& w = a.waves[wv];
    if (p < w.n && a.grad) a.grad[w.s_off + p] = g;
    if (a.chunks[blockIdx.x].y == 0 && threadIdx.x == 0 && a.terms) {
        a.terms[4 * wv + 0] = loss;
        a.terms[4 * wv + 1] = isl;
        a.terms[4 * wv + 2] = soft;
        a.terms[4 * wv + 3] = E;
    }
}

// Reduce, then one Adam step on the phases of s = exp(j phi) (Sec. 6.2's
// update with the Sec. 7.1.2 optimiser): dL/dphi = 2 Im(conj(s) g).
__global__ __launch_bounds__(256) void reduce_adam_kernel(ReduceArgs a) {
    const int t_prev = *a.step;  // read before this block signals completion
    int wv, p;
    float2 g, sp;
    float loss, isl, soft, E;
    reduce_common(a, wv, p, g, sp, loss, isl, soft, E);
    const WaveDesc& w = a.waves[wv];
    if (p < w.n) {
        const int64_t i = w.s_off + p;
        const float dphi = 2.f * (sp.x * g.y - sp.y * g.x);
        const float t = (float)(t_prev + 1);
        float m = a.adam_m[i], v = a.adam_v[i];
        m = fmaf(a.beta1, m, (1.f - a.beta1) * dphi);
        v = fmaf(a.beta2, v, (1.f - a.beta2) * dphi * dphi);
        const float mh = m / (1.f - powf(a.beta1, t));
        const float vh = v / (1.f - powf(a.beta2, t));
        const float ph = a.phi[i] - a.lr * mh / (sqrtf(vh) + a.adam_eps);
        a.adam_m[i] = m;
        a.adam_v[i] = v;
        a.phi[i] = ph;
        float sn, cs;
        sincosf(ph, &sn, &cs);
        a.s_next[i] = make_float2(cs, sn);
    }
    if (a.chunks[blockIdx.x].y == 0 && threadIdx.x == 0 && a.terms) {
        a.terms[4 * wv + 0] = loss;
        a.terms[4 * wv + 1] = isl;
        a.terms[4 * wv + 2] = soft;
        a.terms[4 * wv + 3] = E;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned done = atomicAdd(&a.ctrl[0], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(a.step, t_prev + 1);
            atomicExch(&a.ctrl[0], 0u);
        }
    }
}

__global__ __launch_bounds__(256) void phase_to_signal_kernel(const float* phi, float2* s, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) {
        float sn, cs;
        sincosf(phi[i], &sn, &cs);
        s[i] = make_float2(cs, sn);
    }
}

// ------------------------------------------------------------ launchers --
void* variant_kernel_0(int mode, int lg);
void* variant_kernel_1(int mode, int lg);
void* variant_kernel_2(int mode, int lg);
void* variant_kernel_3(int mode, int lg);
void* variant_kernel_4(int mode, int lg);
VariantInfo variant_info_0(int lg);
VariantInfo variant_info_1(int lg);
VariantInfo variant_info_2(int lg);
VariantInfo variant_info_3(int lg);
VariantInfo variant_info_4(int lg);

VariantInfo variant_info(int v, int lg) {
    switch (v) {
        case 0: return variant_info_0(lg);
        case 1: return variant_info_1(lg);
        case 2: return variant_info_2(lg);
        case 3: return variant_info_3(lg);
        case 4: return variant_info_4(lg);
    }
    return VariantInfo{};
}

static void* kernel_for(int mode, int variant, int lg) {
    switch (variant) {
        case 0: return variant_kernel_0(mode, lg);
        case 1: return variant_kernel_1(mode, lg);
        case 2: return variant_kernel_2(mode, lg);
        case 3: return variant_kernel_3(mode, lg);
        case 4: return variant_kernel_4(mode, lg);
    }
    return nullptr;
}

int variant_max_resident(int mode, int variant, int lg, int dyn_lds_bytes) {
    const VariantInfo vi = variant_info(variant, lg);
    void* k = vi.fits ? kernel_for(mode, variant, lg) : nullptr;
    if (!k) return 0;
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_lds_bytes) != hipSuccess) return 0;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, vi.wgs, dyn_lds_bytes) != hipSuccess) return 0;
    return blocks;
}

hipError_t launch_af(int mode, int variant, int lg, const AfArgs& a, int grid, int dyn_lds_bytes, hipStream_t st) {
    const VariantInfo vi = variant_info(variant, lg);
    void* k = vi.fits ? kernel_for(mode, variant, lg) : nullptr;
    if (!k || grid <= 0) return hipErrorInvalidValue;
    void* args[] = {(void*)&a};
    return hipLaunchKernel(k, dim3(grid), dim3(vi.wgs), args, (size_t)dyn_lds_bytes, st);
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st) {
    if (a.n_chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_kernel, dim3(a.n_chunks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_reduce_adam(const ReduceArgs& a, hipStream_t st) {
    if (a.n_chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_adam_kernel, dim3(a.n_chunks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_phase_to_signal(const float* phi, float2* s, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(phase_to_signal_kernel, dim3((unsigned)blocks), dim3(256), 0, st, phi, s, count);
    return hipGetLastError();
}

}  // namespace graf
