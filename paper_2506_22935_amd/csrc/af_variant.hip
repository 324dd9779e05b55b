// One kernel variant's instantiations, one per transform size it covers
// (compiled once per GRAF_VARIANT so the variants build in parallel).
#include "af_segment.h"

#ifndef GRAF_VARIANT
#error "GRAF_VARIANT must be defined"
#endif

namespace graf {

#define GRAF_CAT2(a, b) a##b
#define GRAF_CAT(a, b) GRAF_CAT2(a, b)
using VSel = GRAF_CAT(V, GRAF_VARIANT);

template <int MODE, int LG, bool CIRC, bool EXTK = false, bool MAGONLY = false, bool HARDONLY = false>
static void* pick_lg(int lg) {
    if constexpr (LG > 15) {
        return nullptr;
    } else {
        if (lg == LG) {
            if constexpr (VSel::fits(LG) && (!CIRC || (VSel::SPLIT && VSel::S_LDS)))
                return (void*)af_kernel<MODE, VSel, LG, CIRC, EXTK, MAGONLY, HARDONLY>;
            return nullptr;
        }
        return pick_lg<MODE, LG + 1, CIRC, EXTK, MAGONLY, HARDONLY>(lg);
    }
}

template <bool CIRC>
static void* pick_mode(int mode, int lg) {
    switch (mode) {
        case MODE_FWD: return pick_lg<MODE_FWD, 1, CIRC>(lg);
        case MODE_BWD_MAG: return pick_lg<MODE_BWD_MAG, 1, CIRC>(lg);
        case MODE_BWD_LOSS: return pick_lg<MODE_BWD_LOSS, 1, CIRC>(lg);
        case MODE_FUSED_ISL: return pick_lg<MODE_FUSED_ISL, 1, CIRC>(lg);
        case MODE_LOSS: return pick_lg<MODE_LOSS, 1, CIRC>(lg);
        case MODE_FUSED_EXT: return pick_lg<MODE_FUSED_ISL, 1, CIRC, true>(lg);
        case MODE_FWD_EXT: return pick_lg<MODE_FWD, 1, CIRC, true>(lg);
        case MODE_FWD_HARD: return pick_lg<MODE_FWD, 1, CIRC, true, false, true>(lg);
        case MODE_FWD_MAG:
            if constexpr (VSel::SPLIT) return pick_lg<MODE_FWD, 1, CIRC>(lg);
            return pick_lg<MODE_FWD, 1, CIRC, false, true>(lg);
    }
    return nullptr;
}

void* GRAF_CAT(variant_kernel_, GRAF_VARIANT)(int mode, int lg, int circ) {
    return circ ? pick_mode<true>(mode, lg) : pick_mode<false>(mode, lg);
}

VariantInfo GRAF_CAT(variant_info_, GRAF_VARIANT)(int lg) {
    VariantInfo vi{};
    vi.lo = VSel::LO;
    vi.hi = VSel::HI;
    vi.p = VSel::P;
    vi.split = VSel::SPLIT;
    vi.wgs = VSel::WGS;
    vi.s_lds = VSel::S_LDS;
    vi.circ = VSel::SPLIT && VSel::S_LDS;
    vi.fits = 0;
    vi.fft_lds = 0;
    vi.nacc = 0;
    vi.s_bytes = 0;
    if (lg >= 1 && lg <= 15 && VSel::fits(lg)) {
        vi.fits = 1;
        vi.fft_lds = VSel::fft_lds_bytes(lg);
        vi.nacc = VSel::nacc(lg);
        vi.s_bytes = VSel::S_LDS ? 8 * (2 << lg) : 0;  // samples zero-padded to M
    }
    return vi;
}

}  // namespace graf
