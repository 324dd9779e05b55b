// Gradient reduction, fused Adam on phases and small elementwise kernels,
// plus the launch helpers for every kernel of the library.
#include "af_reduce.h"

namespace graf {

__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a) {
    __shared__ double sh[16];
    __shared__ float2 sh2[256];
    reduce_chunk<false>(a, (int)blockIdx.x, 0, sh, sh2);
}

// Reduce, then one Adam step with step number *step + 1; the counter itself
// is advanced by step_advance_kernel afterwards (a completion counter that
// every block bumps would serialise thousands of device-scope atomics and
// cache write-backs on one address).
__global__ __launch_bounds__(256) void reduce_adam_kernel(ReduceArgs a) {
    __shared__ double sh[16];
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

// ------------------------------------------------------------ launchers --
void* variant_kernel_0(int mode, int lg, int circ);
void* variant_kernel_1(int mode, int lg, int circ);
void* variant_kernel_2(int mode, int lg, int circ);
void* variant_kernel_3(int mode, int lg, int circ);
void* variant_kernel_4(int mode, int lg, int circ);
void* variant_kernel_5(int mode, int lg, int circ);
VariantInfo variant_info_0(int lg);
VariantInfo variant_info_1(int lg);
VariantInfo variant_info_2(int lg);
VariantInfo variant_info_3(int lg);
VariantInfo variant_info_4(int lg);
VariantInfo variant_info_5(int lg);

VariantInfo variant_info(int v, int lg) {
    switch (v) {
        case 0: return variant_info_0(lg);
        case 1: return variant_info_1(lg);
        case 2: return variant_info_2(lg);
        case 3: return variant_info_3(lg);
        case 4: return variant_info_4(lg);
        case 5: return variant_info_5(lg);
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

hipError_t launch_phase_to_signal(const float* phi, float2* s, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(phase_to_signal_kernel, dim3((unsigned)blocks), dim3(256), 0, st, phi, s, count);
    return hipGetLastError();
}

}  // namespace graf
