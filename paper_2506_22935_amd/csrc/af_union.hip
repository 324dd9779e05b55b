// Instances of the one-launch kernel (variant 6): every mode, both lag kinds.
#include "af_segment.h"

namespace graf {

template <bool CIRC>
static void* union_mode(int mode) {
    switch (mode) {
        case MODE_FWD: return (void*)af_union_kernel<MODE_FWD, CIRC>;
        case MODE_BWD_MAG: return (void*)af_union_kernel<MODE_BWD_MAG, CIRC>;
        case MODE_BWD_LOSS: return (void*)af_union_kernel<MODE_BWD_LOSS, CIRC>;
        case MODE_FUSED_ISL: return (void*)af_union_kernel<MODE_FUSED_ISL, CIRC>;
        case MODE_LOSS: return (void*)af_union_kernel<MODE_LOSS, CIRC>;
        case MODE_FUSED_EXT: return (void*)af_union_kernel<MODE_FUSED_ISL, CIRC, true>;
        case MODE_FWD_EXT: return (void*)af_union_kernel<MODE_FWD, CIRC, true>;
        case MODE_FWD_MAG: return (void*)af_union_kernel<MODE_FWD, CIRC>;
        case MODE_FWD_HARD: return (void*)af_union_kernel<MODE_FWD, CIRC, true>;
    }
    return nullptr;
}

void* variant_kernel_6(int mode, int lg, int circ) {
    if (!VU::fits(lg)) return nullptr;
    return circ ? union_mode<true>(mode) : union_mode<false>(mode);
}

// Sizes as the planner sees them: the transform buffers and short tables of
// the largest class whatever lg, then the region of the pass-2 table and the
// samples (or the periodic samples staged twice) for the plan's largest lg.
VariantInfo variant_info_6(int lg) {
    VariantInfo vi{};
    vi.lo = VU::LO;
    vi.hi = VU::HI;
    vi.p = VU::P;
    vi.split = VU::SPLIT;
    vi.wgs = VU::WGS;
    vi.s_lds = VU::S_LDS;
    vi.circ = 1;
    vi.fits = 0;
    if (VU::fits(lg)) {
        vi.fits = 1;
        vi.fft_lds = VU::fft_lds_bytes(VU::HI);
        vi.nacc = VU::nacc(lg);
        vi.s_bytes = union_region_bytes(lg);
    }
    return vi;
}

__global__ void queue_reset_kernel(int* q) { *q = 0; }

hipError_t launch_queue_reset(int* queue, hipStream_t st) {
    hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(1), 0, st, queue);
    return hipGetLastError();
}

}  // namespace graf
