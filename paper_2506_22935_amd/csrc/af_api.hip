// Host side of libgraf_af.so: argument validation, the work planner
// (segments, longest-first order, store-versus-recompute under a budget),
// the variant autotuner and the launch sequences behind the C ABI declared
// in include/graf_af.h.
#include "../../include/graf_af.h"
#include "af_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using graf::AfArgs;
using graf::ReduceArgs;
using graf::SegDesc;
using graf::VariantInfo;
using graf::WaveDesc;

namespace {

constexpr int kMaxLds = 160 * 1024;
constexpr int kMinM = 128;
constexpr int kMaxM = 32768;
constexpr int kMinCircN = 64;   // periodic AF: N = M, the split variants' sizes
constexpr int kMaxCircN = 4096;
constexpr int kMaxSpecN = 4096;  // spectral variance: three N-vectors in LDS
constexpr int kMaxQueues = 64;   // ticket counters: at most one per class (2 kinds x 9 sizes)

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
int ilog2(int64_t x) {
    int r = 0;
    while ((int64_t(1) << r) < x) ++r;
    return r;
}
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// Workspace of af_loss_no_alloc: a file-scope device array, one copy per GPU
// (each device that loads the library holds it until the process ends).
// Its name in host code is a stand-in, not a device address, so no host
// code passes it to a kernel: af_plan_create resolves the array's address
// on the plan's device once (hipGetSymbolAddress, with that device current)
// and every later use goes through that pointer.
constexpr size_t kNoAllocWsBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoAllocWsBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
int g_scratch_state[kMaxDevices] = {};  // 0 not resolved yet, 1 resolved, -1 failed

// Resolve device dev's copy of `scratch`; dev must be the current device.
void resolve_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_state[dev] != 0) return;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess && ptr != nullptr && ((uintptr_t)ptr & 255) == 0) {
        g_scratch_ptr[dev] = ptr;
        g_scratch_state[dev] = 1;
    } else {
        (void)hipGetLastError();  // leave no error behind for the next call
        g_scratch_state[dev] = -1;
    }
}

void* scratch_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_state[dev] == 1 ? g_scratch_ptr[dev] : nullptr;
}

}  // namespace

struct af_plan {
    int device = -1;
    int cus = 0;
    int batch = 0;
    std::vector<af_wave> waves;
    float eps = 0.f;
    int store_mode = 0;
    int64_t budget = 0;
    int seg_iters_opt = 0;
    double items_per_slot = 0.0;  // work items per resident work group (0: the planner's default)
    int loss_passes_opt = 0;

    // schedule: one class per distinct M, each with its own kernel variant,
    // slice of the execution order, grid and work-queue counters
    struct Class {
        int lg = 0;          // log2(M/2) (the kernel's M: 2N for a periodic class)
        int circ = 0;        // periodic waveforms
        int variant = -1;
        int begin = 0, count = 0;  // slice of the execution order
        int grid[graf::kNumModes] = {};
        int dyn_lds = 0;
        int max_n = 0;
        int single_wave = -1;  // the waveform index when the class has one
        double cost = 0.0;
    };
    std::vector<Class> classes;
    std::vector<int> forced;  // per natural class: variant forced by the autotuner (-1: default)
    int natural_classes = 0;  // distinct (transform size, lag kind) pairs
    bool one_launch = true;   // run several classes as one launch of the one-launch kernel when they fit it
    bool one_active = false;  // the current schedule is that one launch
    // cross-AF launches: one per natural class over its slice of d_segs_x
    struct XClass {
        int lg = 0, circ = 0, begin = 0, count = 0;
    };
    std::vector<XClass> xclasses;
    std::vector<WaveDesc> wave_desc;  // host copy of the device descriptors
    int opt_variant = -1;
    bool stores = false;
    int n_segs = 0, n_chunks = 0, sg_log = 2;
    int log2_mmax = 0;
    int max_n = 0;
    int64_t cells = 0, store_bytes = 0;
    size_t off_parts = 0, off_energy = 0, off_slabs = 0, off_slabs2 = 0, off_extra = 0, off_vals = 0, off_store = 0,
           ws_total = 0;
    int64_t slab_elems = 0;  // complex64 per slab set ([segs][N] per waveform)

    // plan-owned device tables
    WaveDesc* d_waves = nullptr;
    SegDesc* d_segs = nullptr;
    SegDesc* d_segs_x = nullptr;       // the segments in natural-class order (one-launch plans)
    graf::RBlock* d_chunks = nullptr;  // reduce blocks
    float2* d_tw = nullptr;
    int* d_queue = nullptr;            // ticket counters of the one-launch kernel, one per class
    size_t cap_segs = 0, cap_chunks = 0, cap_segs_x = 0;

    // Plans with several size classes run them concurrently: class 0 (the
    // largest) on the caller's stream, class c > 0 on side[c - 1], forked
    // from and joined back into the caller's stream with events, so that a
    // class's tail overlaps the next classes' work instead of draining the
    // GPU between launches.  Default-priority streams; capturable.
    std::vector<hipStream_t> side;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
};

namespace {

void free_streams(af_plan* p) {
    for (hipStream_t s : p->side) (void)hipStreamDestroy(s);
    for (hipEvent_t e : p->join) (void)hipEventDestroy(e);
    if (p->fork) (void)hipEventDestroy(p->fork);
    p->side.clear();
    p->join.clear();
    p->fork = nullptr;
}

// side streams and events for C concurrent classes
af_status make_streams(af_plan* p, int C) {
    if (C <= 1) return AF_OK;
    if (hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) != hipSuccess) return AF_ERR_HIP;
    for (int c = 1; c < C; ++c) {
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return AF_ERR_HIP;
        p->side.push_back(s);
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return AF_ERR_HIP;
        p->join.push_back(e);
    }
    return AF_OK;
}

void free_tables(af_plan* p) {
    free_streams(p);
    if (p->d_waves) (void)hipFree(p->d_waves);
    if (p->d_segs) (void)hipFree(p->d_segs);
    if (p->d_segs_x) (void)hipFree(p->d_segs_x);
    if (p->d_chunks) (void)hipFree(p->d_chunks);
    if (p->d_tw) (void)hipFree(p->d_tw);
    if (p->d_queue) (void)hipFree(p->d_queue);
    p->d_waves = nullptr;
    p->d_segs = nullptr;
    p->d_segs_x = nullptr;
    p->d_chunks = nullptr;
    p->d_tw = nullptr;
    p->d_queue = nullptr;
}

// Periodic (circular) waveforms: N = M bins, run as the even half of the
// kernel's M = 2N split with lag pairs tau, N - tau for tau in [0, N/2].
bool is_circ(const af_wave& w) { return (w.flags & AF_WAVE_PERIODIC) != 0; }
int kernel_m(const af_wave& w) { return is_circ(w) ? 2 * w.n : w.m; }
int pair_lags(const af_wave& w) { return is_circ(w) ? w.n / 2 : w.max_lag; }
int64_t grid_cells(const af_wave& w) {
    return is_circ(w) ? (int64_t)w.n * w.n : (int64_t)(2 * w.max_lag + 1) * w.m;
}

// Can variant v run transform size 2^lg (periodic or not) for waveforms up
// to max_n samples?
bool variant_fits(int v, int lg, int max_n, int circ) {
    const VariantInfo vi = graf::variant_info(v, lg);
    if (!vi.fits || (circ && !vi.circ)) return false;
    const int lds = vi.fft_lds + vi.s_bytes;
    return lds <= kMaxLds;
}

int default_variant(int lg, int max_n, int circ) {
    // small transforms run faster with 8 points per lane (with 16 the lane
    // groups are 4-16 lanes): periodic N <= 256, aperiodic M = 128 (measured
    // fused passes of 4096 waveforms: periodic N = 64 / 128 / 256 0.09 / 0.15
    // / 0.46 ms against 0.16 / 0.28 / 0.54; aperiodic M = 128 0.13 against
    // 0.21; from aperiodic M = 256 and periodic N = 512 on, 16 points win)
    if ((circ ? lg <= 8 : lg <= 6) && variant_fits(3, lg, max_n, circ)) return 3;
    const int order[] = {0, 1, 2};
    for (int v : order)
        if (variant_fits(v, lg, max_n, circ)) return v;
    return -1;
}

// lags per iteration of a work group: one per lane-group pair (split
// halves), one per lane group (halves in turn, or periodic)
int lags_per_iter(const VariantInfo& vi, int m, int circ) {
    const int L = (m / 2) / vi.p;
    const int groups = vi.wgs / L;
    return (vi.split && !circ) ? groups / 2 : groups;
}

af_status hip_fail() { return AF_ERR_HIP; }

// Build classes, segments, order, chunks and the workspace layout, and
// upload the device tables.  Variant per class: forced[c] if set, else
// opt_variant if it fits, else the default for that size.
af_status build_schedule(af_plan* p) {
    const int B = p->batch;
    // classes by (transform size, periodic), largest first; key 2 lg + circ
    std::vector<int> keys;
    for (const af_wave& w : p->waves) keys.push_back(2 * (ilog2(kernel_m(w)) - 1) + (is_circ(w) ? 1 : 0));
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    std::reverse(keys.begin(), keys.end());
    const int NC = (int)keys.size();
    p->natural_classes = NC;
    if ((int)p->forced.size() != NC) p->forced.assign(NC, -1);
    // one launch for every class: the classes share a lag kind and each fits
    // the one-launch kernel; by default for plans with several classes,
    // always when that variant is asked for, never once the autotuner has
    // forced variants per class
    bool union_ok = true, forced_any = false;
    for (int key : keys)
        if ((key & 1) != (keys[0] & 1) || !graf::variant_info(graf::kUnionVariant, key >> 1).fits) union_ok = false;
    for (int f : p->forced) forced_any = forced_any || f >= 0;
    if (p->opt_variant == graf::kUnionVariant && !union_ok) return AF_ERR_UNSUPPORTED;
    const bool one = union_ok && !forced_any &&
                     (p->opt_variant == graf::kUnionVariant || (p->opt_variant < 0 && p->one_launch && NC > 1));
    const int C = one ? 1 : NC;
    std::vector<af_plan::Class> cls(C);
    std::vector<int> cls_of_wave(B), nat_of_wave(B);
    for (int b = 0; b < B; ++b) {
        const int key = 2 * (ilog2(kernel_m(p->waves[b])) - 1) + (is_circ(p->waves[b]) ? 1 : 0);
        const int nat = (int)(std::find(keys.begin(), keys.end(), key) - keys.begin());
        const int c = one ? 0 : nat;
        nat_of_wave[b] = nat;
        cls_of_wave[b] = c;
        cls[c].lg = std::max(cls[c].lg, key >> 1);
        cls[c].circ = key & 1;
        cls[c].max_n = std::max(cls[c].max_n, p->waves[b].n);
    }
    int total_slots = 0;
    for (int c = 0; c < C; ++c) {
        af_plan::Class& k = cls[c];
        int v = one ? graf::kUnionVariant : p->forced[c];
        if (v < 0 && p->opt_variant >= 0 && p->opt_variant != graf::kUnionVariant &&
            variant_fits(p->opt_variant, k.lg, k.max_n, k.circ))
            v = p->opt_variant;
        if (v < 0) v = default_variant(k.lg, k.max_n, k.circ);
        if (v < 0 || !variant_fits(v, k.lg, k.max_n, k.circ)) return AF_ERR_UNSUPPORTED;
        k.variant = v;
        const VariantInfo vi = graf::variant_info(v, k.lg);
        k.dyn_lds = vi.fft_lds + vi.s_bytes;
        for (int mode = 0; mode < graf::kNumModes; ++mode) {
            const int r = graf::variant_max_resident(mode, v, k.lg, k.circ, k.dyn_lds);
            if (r <= 0 && graf::is_ext_mode(mode) && !vi.split) {
                k.grid[mode] = 0;  // no extended instance: those terms are refused
                continue;
            }
            if (r <= 0) return AF_ERR_UNSUPPORTED;
            k.grid[mode] = r * p->cus;  // capped by the segment count below
        }
        total_slots = std::max(total_slots, k.grid[graf::MODE_FUSED_ISL]);
    }

    // per-waveform iteration counts and costs
    std::vector<int> lpi(B), iters(B);
    std::vector<double> cost_iter(B);
    double total = 0.0;
    for (int b = 0; b < B; ++b) {
        const af_wave& w = p->waves[b];
        const af_plan::Class& k = cls[cls_of_wave[b]];
        const VariantInfo vi = graf::variant_info(k.variant, k.lg);
        const int mk = kernel_m(w);
        lpi[b] = lags_per_iter(vi, mk, k.circ);
        iters[b] = (pair_lags(w) + 1 + lpi[b] - 1) / lpi[b];
        // a periodic lag runs one half-size transform, an aperiodic pair two
        cost_iter[b] = (double)lpi[b] * (k.circ ? mk / 2 : mk) * ilog2(mk);
        total += iters[b] * cost_iter[b];
    }
    // about two items per resident work group; six for the one-launch
    // kernel, whose work groups take items from one queue by ticket, so that
    // the queue's last items are short
    const double ips = p->items_per_slot > 0.0 ? p->items_per_slot : (one ? 6.0 : 2.0);
    const double target = total / (ips * std::max(1, total_slots));

    std::vector<WaveDesc> wd(B);
    std::vector<SegDesc> segs;
    std::vector<double> seg_cost;
    std::vector<int2> rpos;  // reduce blocks: (wave, first sample)
    int64_t slab_elems = 0, slab2_elems = 0, store_elems = 0;
    for (int b = 0; b < B; ++b) {
        const af_wave& w = p->waves[b];
        int per = p->seg_iters_opt > 0 ? p->seg_iters_opt
                                       : std::max(1, (int)std::lround(target / std::max(cost_iter[b], 1.0)));
        per = std::min(per, iters[b]);
        WaveDesc& d = wd[b];
        const int mk = kernel_m(w);
        d.n = w.n;
        d.m = mk;
        d.T = pair_lags(w);
        d.log2m = ilog2(mk);
        d.circ = is_circ(w) ? 1 : 0;
        d.moyal = is_circ(w) ? w.n : mk;
        d.s_off = w.s_off;
        d.grid_off = w.grid_off;
        d.store_off = store_elems;
        d.slab_off = slab_elems;
        d.seg_begin = (int)segs.size();
        d.h_tau = w.h_tau;
        d.h_k = w.h_k;
        d.band_off = 62 * b;
        d.full_window = (is_circ(w) || w.max_lag == w.n - 1) ? 1 : 0;
        for (int it = 0; it < iters[b]; it += per) {
            SegDesc sd;
            sd.wave = b;
            sd.tau_begin = it * lpi[b];
            sd.tau_end = std::min(pair_lags(w) + 1, (it + per) * lpi[b]);
            sd.rec = (int)segs.size();
            segs.push_back(sd);
            seg_cost.push_back(std::min(per, iters[b] - it) * cost_iter[b]);
        }
        d.seg_count = (int)segs.size() - d.seg_begin;
        slab_elems += (int64_t)d.seg_count * w.n;
        // segments holding mainlobe lags (second slabs of the fused loss pass)
        d.isl_segs = 0;
        for (int i = d.seg_begin; i < (int)segs.size(); ++i)
            if (segs[i].tau_begin <= w.h_tau) ++d.isl_segs;
        d.slab2_off = slab2_elems;
        slab2_elems += (int64_t)d.isl_segs * w.n;
        // spectra per lag pair: M (two halves), or N for a periodic lag
        store_elems += (int64_t)(pair_lags(w) + 1) * (is_circ(w) ? w.n : w.m);
        (void)0;
    }
    // reduce blocks: 16 slab subgroups per block when waveforms have many
    // segments, 4 for a few dozen, and one (256 samples per block, every
    // slab load of a thread in flight at once) for at most 32: the many
    // short waveforms of a large batch then need a quarter of the blocks
    int max_segs = 0;
    for (int b = 0; b < B; ++b) max_segs = std::max(max_segs, wd[b].seg_count);
    const int sg_log = max_segs >= 64 ? 4 : (max_segs > 32 ? 2 : 0);
    for (int b = 0; b < B; ++b)
        for (int c = 0; c < wd[b].n; c += (256 >> sg_log)) rpos.push_back(make_int2(b, c));

    // execution order: by class, longest segment first within a class
    std::vector<int> order;
    order.reserve(segs.size());
    for (int c = 0; c < C; ++c) {
        cls[c].begin = (int)order.size();
        for (size_t i = 0; i < segs.size(); ++i)
            if (cls_of_wave[segs[i].wave] == c) order.push_back((int)i);
        std::stable_sort(order.begin() + cls[c].begin, order.end(),
                         [&](int a, int b) { return seg_cost[a] > seg_cost[b]; });
        cls[c].count = (int)order.size() - cls[c].begin;
        for (int i = cls[c].begin; i < (int)order.size(); ++i) cls[c].cost += seg_cost[order[i]];
        for (int mode = 0; mode < graf::kNumModes; ++mode) cls[c].grid[mode] = std::min(cls[c].grid[mode], cls[c].count);
    }

    std::vector<SegDesc> exec(order.size());
    for (size_t i = 0; i < order.size(); ++i) exec[i] = segs[order[i]];

    // cross-AF launches: one per natural class; with one launch they run
    // over a second copy of the segments in natural-class order
    std::vector<af_plan::XClass> xcls(NC);
    std::vector<SegDesc> exec_x;
    for (int c = 0; c < NC; ++c) {
        xcls[c].lg = keys[c] >> 1;
        xcls[c].circ = keys[c] & 1;
        if (one) {
            xcls[c].begin = (int)exec_x.size();
            for (const SegDesc& sd : segs)
                if (nat_of_wave[sd.wave] == c) exec_x.push_back(sd);
            xcls[c].count = (int)exec_x.size() - xcls[c].begin;
        } else {
            xcls[c].begin = cls[c].begin;
            xcls[c].count = cls[c].count;
        }
    }

    // workspace layout and the store decision
    const size_t parts_b = align256(segs.size() * sizeof(graf::Part));
    const size_t energy_b = align256((size_t)B * sizeof(float));
    const size_t slabs_b = align256((size_t)slab_elems * sizeof(float2));
    p->slab_elems = slab_elems;
    const size_t slabs2_b = align256((size_t)slab2_elems * sizeof(float2));
    const size_t store_b = align256((size_t)store_elems * sizeof(float2));
    // the per-waveform terms' gradient (packed like s) and their [B][4] values
    int64_t s_extent = 0;
    for (const af_wave& w : p->waves) s_extent = std::max<int64_t>(s_extent, w.s_off + w.n);
    const size_t extra_b = align256((size_t)s_extent * sizeof(float2));
    const size_t vals_b = align256((size_t)B * 4 * sizeof(float));
    const size_t base = parts_b + energy_b + slabs_b + slabs2_b + extra_b + vals_b;
    bool stores;
    if (p->store_mode == 1)
        stores = true;
    else if (p->store_mode == 2)
        stores = false;
    else
        stores = p->budget <= 0 || (int64_t)(base + store_b) <= p->budget;
    if (p->budget > 0 && (int64_t)(base + (stores ? store_b : 0)) > p->budget) return AF_ERR_BUDGET;

    // upload
    if (segs.size() > p->cap_segs) {
        if (p->d_segs) (void)hipFree(p->d_segs);
        p->d_segs = nullptr;
        if (hipMalloc(&p->d_segs, segs.size() * sizeof(SegDesc)) != hipSuccess) return hip_fail();
        p->cap_segs = segs.size();
    }
    // reduce blocks carry their waveform's final descriptor
    std::vector<graf::RBlock> rblocks(rpos.size());
    for (size_t i = 0; i < rpos.size(); ++i) {
        rblocks[i].w = wd[rpos[i].x];
        rblocks[i].wave = rpos[i].x;
        rblocks[i].p0 = rpos[i].y;
    }
    if (rblocks.size() > p->cap_chunks) {
        if (p->d_chunks) (void)hipFree(p->d_chunks);
        p->d_chunks = nullptr;
        if (hipMalloc(&p->d_chunks, rblocks.size() * sizeof(graf::RBlock)) != hipSuccess) return hip_fail();
        p->cap_chunks = rblocks.size();
    }
    if (one && exec_x.size() > p->cap_segs_x) {
        if (p->d_segs_x) (void)hipFree(p->d_segs_x);
        p->d_segs_x = nullptr;
        if (hipMalloc(&p->d_segs_x, exec_x.size() * sizeof(SegDesc)) != hipSuccess) return hip_fail();
        p->cap_segs_x = exec_x.size();
    }
    if (one && hipMemcpy(p->d_segs_x, exec_x.data(), exec_x.size() * sizeof(SegDesc), hipMemcpyHostToDevice) !=
                   hipSuccess)
        return hip_fail();
    if (!p->d_waves && hipMalloc(&p->d_waves, (size_t)B * sizeof(WaveDesc)) != hipSuccess) return hip_fail();
    if (hipMemcpy(p->d_waves, wd.data(), (size_t)B * sizeof(WaveDesc), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_segs, exec.data(), exec.size() * sizeof(SegDesc), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_chunks, rblocks.data(), rblocks.size() * sizeof(graf::RBlock), hipMemcpyHostToDevice) !=
            hipSuccess)
        return hip_fail();

    for (int c = 0; c < C; ++c) {
        int count = 0, last = -1;
        for (int b = 0; b < B; ++b)
            if (cls_of_wave[b] == c) {
                ++count;
                last = b;
            }
        cls[c].single_wave = count == 1 ? last : -1;
    }
    p->wave_desc = wd;
    p->classes = cls;
    p->xclasses = xcls;
    p->one_active = one;
    p->stores = stores;
    p->n_segs = (int)segs.size();
    p->n_chunks = (int)rblocks.size();
    p->sg_log = sg_log;
    p->store_bytes = (int64_t)store_elems * (int64_t)sizeof(float2);
    p->off_parts = 0;
    p->off_energy = parts_b;
    p->off_slabs = parts_b + energy_b;
    p->off_slabs2 = parts_b + energy_b + slabs_b;
    p->off_extra = parts_b + energy_b + slabs_b + slabs2_b;
    p->off_vals = p->off_extra + extra_b;
    p->off_store = base;
    p->ws_total = base + (stores ? store_b : 0);
    return AF_OK;
}

af_status validate_plan_inputs(int32_t batch, const af_wave* waves, const af_plan_opts* opts) {
    if (batch <= 0 || !waves || !opts) return AF_ERR_INVALID_ARG;
    if (!(opts->eps >= 0.f) || opts->store_mode < 0 || opts->store_mode > 2) return AF_ERR_INVALID_ARG;
    if (opts->loss_passes < 0 || opts->loss_passes > 1) return AF_ERR_INVALID_ARG;
    if (opts->launch_mode < 0 || opts->launch_mode > 1) return AF_ERR_INVALID_ARG;
    for (int b = 0; b < batch; ++b) {
        const af_wave& w = waves[b];
        if (w.n < 1 || w.s_off < 0 || w.grid_off < 0 || w.h_tau < 0 || w.h_k < 0 || (w.flags & ~AF_WAVE_PERIODIC))
            return AF_ERR_INVALID_ARG;
        if (w.grid_off % 4 != 0) return AF_ERR_INVALID_ARG;  // rows move as 16-byte vectors
        const int T = w.max_lag < 0 ? w.n - 1 : w.max_lag;
        if (w.max_lag < -1 || T > w.n - 1) return AF_ERR_INVALID_ARG;
        if (is_circ(w)) {
            // periodic: N = M bins, a power of two in [64, 4096], every lag
            if (w.m != w.n || T != w.n - 1 || w.h_tau > w.n / 2 || w.h_k > w.n / 2) return AF_ERR_INVALID_ARG;
            if (!is_pow2(w.n) || w.n < kMinCircN || w.n > kMaxCircN) return AF_ERR_UNSUPPORTED;
            continue;
        }
        if (!is_pow2(w.m) || w.m < kMinM || w.m > kMaxM || w.m < 2 * (int64_t)w.n) return AF_ERR_UNSUPPORTED;
    }
    return AF_OK;
}

struct WsView {
    graf::Part* parts;
    float* energy;
    float2* slabs;
    float2* slabs2;
    float2* extra;
    float* vals;
    float2* store;
};

WsView ws_view(const af_plan* p, void* ws) {
    char* b = (char*)ws;
    WsView v;
    v.parts = (graf::Part*)(b + p->off_parts);
    v.energy = (float*)(b + p->off_energy);
    v.slabs = (float2*)(b + p->off_slabs);
    v.slabs2 = (float2*)(b + p->off_slabs2);
    v.extra = (float2*)(b + p->off_extra);
    v.vals = (float*)(b + p->off_vals);
    v.store = p->stores ? (float2*)(b + p->off_store) : nullptr;
    return v;
}

AfArgs base_args(const af_plan* p, const void* s, const WsView& v) {
    AfArgs a;
    std::memset(&a, 0, sizeof(a));
    a.s = (const float2*)s;
    a.waves = p->d_waves;
    a.segs = p->d_segs;
    a.n_segs = 0;
    a.log2_mmax = p->log2_mmax;
    a.tw = p->d_tw;
    a.eps = p->eps;
    a.w_isl = 0.f;
    a.w_psl = 0.f;
    a.temp = 1.f;
    a.parts = v.parts;
    a.slabs = v.slabs;
    a.slabs2 = v.slabs2;
    a.energy = v.energy;
    return a;
}

ReduceArgs reduce_args(const af_plan* p, const void* s, const WsView& v) {
    ReduceArgs r;
    std::memset(&r, 0, sizeof(r));
    r.s = (const float2*)s;
    r.blocks = p->d_chunks;
    if (p->batch == 1) {
        r.single = 1;
        r.w0 = p->wave_desc[0];
    }
    r.n_blocks = p->n_chunks;
    r.sg_log = p->sg_log;
    r.parts = v.parts;
    r.slabs = v.slabs;
    r.slabs2 = v.slabs2;
    r.energy = v.energy;
    r.temp = 1.f;
    return r;
}

// one persistent launch per size class, each on its own slice of the order;
// with several classes, class c > 0 runs on its side stream between a fork
// from and a join into st
af_status launch(const af_plan* p, int mode, const AfArgs& a0, hipStream_t st, int only_class = -1) {
    const int C = (int)p->classes.size();
    const bool concurrent = only_class < 0 && C > 1 && (int)p->side.size() >= C - 1;
    if (concurrent) {
        if (hipEventRecord(p->fork, st) != hipSuccess) return AF_ERR_HIP;
        for (int c = 1; c < C; ++c)
            if (hipStreamWaitEvent(p->side[c - 1], p->fork, 0) != hipSuccess) return AF_ERR_HIP;
    }
    for (int c = 0; c < C; ++c) {
        if (only_class >= 0 && c != only_class) continue;
        const af_plan::Class& k = p->classes[c];
        hipStream_t cs = (concurrent && c > 0) ? p->side[c - 1] : st;
        AfArgs a = a0;
        a.segs = p->d_segs + k.begin;
        a.n_segs = k.count;
        a.single = k.single_wave >= 0 ? 1 : 0;
        if (a.single) {
            a.w0 = p->wave_desc[k.single_wave];
            a.w0_index = k.single_wave;
        }
        if (k.variant == graf::kUnionVariant) {
            // the one-launch kernel takes items by ticket from a zeroed counter
            a.queue = p->d_queue + c;
            if (graf::launch_queue_reset(a.queue, cs) != hipSuccess) return AF_ERR_HIP;
        }
        hipError_t e = graf::launch_af(mode, k.variant, k.lg, k.circ, a, k.grid[mode], k.dyn_lds, cs);
        if (e != hipSuccess) return AF_ERR_HIP;
    }
    if (concurrent) {
        for (int c = 1; c < C; ++c) {
            if (hipEventRecord(p->join[c - 1], p->side[c - 1]) != hipSuccess) return AF_ERR_HIP;
            if (hipStreamWaitEvent(st, p->join[c - 1], 0) != hipSuccess) return AF_ERR_HIP;
        }
    }
    return AF_OK;
}

bool aligned(const void* x, uintptr_t a) { return ((uintptr_t)x & (a - 1)) == 0; }

af_status check_common(const af_plan* p, const void* s, void* ws, size_t ws_bytes) {
    if (!p || !s) return AF_ERR_INVALID_ARG;
    if (!aligned(s, 8) || (ws && !aligned(ws, 256))) return AF_ERR_INVALID_ARG;
    if (p->ws_total > 0 && (!ws || ws_bytes < p->ws_total)) return AF_ERR_WORKSPACE;
    return AF_OK;
}

// terms of the extended epilogue copy (split variants, forward and fused
// ISL passes): the hard PSL, L_match, the soft mainlobe width, cell weights
bool extended_terms(const af_loss_params* lp) {
    return (lp->psl_hard != 0 && lp->w_psl != 0.f) || lp->w_match != 0.f || lp->w_width != 0.f ||
           lp->w_cell != 0.f;
}
// The forward pass of a loss: the extended instance when a term needs it,
// the hard-PSL-only one when the maximum is the only such term
int forward_mode(const af_loss_params* lp) {
    if (!extended_terms(lp)) return graf::MODE_FWD;
    return (lp->w_match != 0.f || lp->w_width != 0.f || lp->w_cell != 0.f) ? graf::MODE_FWD_EXT
                                                                            : graf::MODE_FWD_HARD;
}

af_status check_loss(const af_plan* p, const af_loss_params* lp) {
    if (!lp) return AF_ERR_INVALID_ARG;
    if (!(lp->psl_temp > 0.f) || !std::isfinite(lp->w_isl) || !std::isfinite(lp->w_psl) || !std::isfinite(lp->w_spec))
        return AF_ERR_INVALID_ARG;
    if (lp->psl_hard != 0 && lp->psl_hard != 1) return AF_ERR_INVALID_ARG;
    if (!std::isfinite(lp->w_match) || (lp->w_match != 0.f && !lp->match_target)) return AF_ERR_INVALID_ARG;
    if (!std::isfinite(lp->w_width) || !std::isfinite(lp->gamma) || !(lp->gamma >= 0.f) ||
        !std::isfinite(lp->w_const) || !std::isfinite(lp->w_smooth) || !std::isfinite(lp->w_cell) ||
        (lp->w_cell != 0.f && !lp->cell_w) || !aligned(lp->cell_w, 4) || !aligned(lp->match_target, 4))
        return AF_ERR_INVALID_ARG;
    // L_match, the width and the cell weights run in the forward and fused
    // ISL passes: not with the soft PSL
    if ((lp->w_match != 0.f || lp->w_width != 0.f || lp->w_cell != 0.f) && lp->w_psl != 0.f && !lp->psl_hard)
        return AF_ERR_UNSUPPORTED;
    // the hard PSL, L_match, the width and the cell weights need every
    // class's extended instances
    if (extended_terms(lp))
        for (const af_plan::Class& k : p->classes)
            if (k.grid[graf::MODE_FUSED_EXT] <= 0 || k.grid[graf::MODE_FWD_EXT] <= 0 ||
                k.grid[graf::MODE_FWD_HARD] <= 0)
                return AF_ERR_UNSUPPORTED;
    if (lp->w_spec != 0.f && p->max_n > kMaxSpecN) return AF_ERR_UNSUPPORTED;
    return AF_OK;
}

// Does the loss take a per-waveform term (the hard PSL, the spectral
// variance, var(|s|), the smoothness term: the per-waveform kernel)?
bool hard_psl(const af_loss_params* lp) { return lp->psl_hard != 0 && lp->w_psl != 0.f; }
bool needs_extra(const af_loss_params* lp) {
    return hard_psl(lp) || lp->w_spec != 0.f || lp->w_const != 0.f || lp->w_smooth != 0.f;
}

// loss forward/backward into slabs and parts (no reduce)
// Can ISL + soft-PSL forward and backward run as one pass (MODE_LOSS)?  The
// soft-PSL gradient then leaves the pass without its normaliser 1/S: this
// needs the fixed shift of the soft-PSL sums (the same rule the kernels use),
// uniform ISL weights with full lag windows (the ISL gradient then lives on
// the mainlobe cells) and variants that split the two half transforms.
bool fused_loss_ok(const af_plan* p, const af_loss_params* lp) {
    if (p->loss_passes_opt == 1 || lp->w_psl == 0.f || lp->psl_hard || lp->band_w != nullptr || lp->w_match != 0.f ||
        lp->w_width != 0.f || lp->w_cell != 0.f)
        return false;
    const float inv_t2 = 1.4426950408889634f / lp->psl_temp;
    if (!(std::sqrt(1.f + p->eps) * inv_t2 < 100.f)) return false;
    for (const af_plan::Class& k : p->classes)
        if (!graf::variant_info(k.variant, k.lg).split) return false;
    if (lp->w_isl != 0.f)
        for (const WaveDesc& d : p->wave_desc)
            if (!d.full_window) return false;
    return true;
}

// Arguments of the loss passes: the hard PSL takes no soft-PSL sums in the
// kernels (its maximum is recorded instead)
AfArgs loss_args(const af_plan* p, const void* s, const af_loss_params* lp, float* mag, const WsView& v) {
    AfArgs a = base_args(p, s, v);
    a.w_isl = lp->w_isl;
    a.w_psl = lp->psl_hard ? 0.f : lp->w_psl;
    a.temp = lp->psl_temp;
    a.band_w = lp->band_w;
    a.mag = mag;
    a.psl_hard = hard_psl(lp) ? 1 : 0;
    if (lp->w_match != 0.f) {
        a.match_t = lp->match_target;
        a.w_match = lp->w_match;
    }
    a.w_width = lp->w_width;
    a.gamma = lp->gamma;
    if (lp->w_cell != 0.f) {
        a.cell_w = lp->cell_w;
        a.w_cell = lp->w_cell;
    }
    return a;
}

// Does a term take a gradient over the cells of the grid?  Else the forward
// pass alone serves: the hard PSL's gradient lives on one cell, and the
// waveform-only terms take none through the AF.
bool grid_gradient(const af_loss_params* lp) {
    return lp->w_isl != 0.f || (lp->w_psl != 0.f && !lp->psl_hard) || lp->w_match != 0.f || lp->w_width != 0.f ||
           lp->w_cell != 0.f;
}
// Do the passes of this loss leave gradient slabs (else the reduction reads none)?
bool loss_writes_slabs(const af_loss_params* lp, bool want_grad) { return want_grad && grid_gradient(lp); }
// Is the forward pass alone enough for this loss?
bool forward_only(const af_loss_params* lp, bool want_grad) { return !want_grad || !grid_gradient(lp); }

// The per-waveform kernel: the hard PSL, the spectral variance, var(|s|) and
// the smoothness term (after the AF pass: it reads the segment records and E)
af_status launch_extra(const af_plan* p, const void* s, const af_loss_params* lp, bool want_grad, const WsView& v,
                       hipStream_t st) {
    if (!needs_extra(lp)) return AF_OK;
    graf::ExtraArgs e;
    std::memset(&e, 0, sizeof(e));
    e.s = (const float2*)s;
    e.waves = p->d_waves;
    e.parts = v.parts;
    e.energy = v.energy;
    e.tw = p->d_tw;
    e.log2_mmax = p->log2_mmax;
    e.psl = hard_psl(lp) ? 1 : 0;
    e.w_psl = lp->w_psl;
    e.spec = lp->w_spec != 0.f ? 1 : 0;
    e.w_spec = lp->w_spec;
    e.wterms = (lp->w_const != 0.f || lp->w_smooth != 0.f) ? 1 : 0;
    e.w_const = lp->w_const;
    e.w_smooth = lp->w_smooth;
    e.g_extra = want_grad ? v.extra : nullptr;
    e.vals = v.vals;
    return graf::launch_extra(e, p->batch, p->max_n, st) == hipSuccess ? AF_OK : AF_ERR_HIP;
}

af_status loss_passes(const af_plan* p, const void* s, const af_loss_params* lp, float* mag, bool want_grad,
                      const WsView& v, hipStream_t st, int only_class = -1) {
    AfArgs a = loss_args(p, s, lp, mag, v);
    af_status rc;
    if (forward_only(lp, want_grad)) {
        rc = launch(p, forward_mode(lp), a, st, only_class);
    } else if (a.w_psl == 0.f) {
        rc = launch(p, extended_terms(lp) ? graf::MODE_FUSED_EXT : graf::MODE_FUSED_ISL, a, st, only_class);
    } else if (fused_loss_ok(p, lp)) {
        rc = launch(p, graf::MODE_LOSS, a, st, only_class);
    } else {
        a.ystore = v.store;
        rc = launch(p, graf::MODE_FWD, a, st, only_class);
        if (rc != AF_OK) return rc;
        a.mag = nullptr;
        a.load_store = v.store != nullptr;
        rc = launch(p, graf::MODE_BWD_LOSS, a, st, only_class);
    }
    if (rc != AF_OK || only_class >= 0) return rc;
    return launch_extra(p, s, lp, want_grad, v, st);
}

// Reduction arguments of a loss call
ReduceArgs loss_reduce_args(const af_plan* p, const void* s, const af_loss_params* lp, bool want_grad,
                            const WsView& v) {
    ReduceArgs r = reduce_args(p, s, v);
    r.w_isl = lp->w_isl;
    r.w_psl = lp->w_psl;
    r.temp = lp->psl_temp;
    r.uniform_w = lp->band_w == nullptr;
    r.skip_slabs = loss_writes_slabs(lp, want_grad) ? 0 : 1;
    r.psl_scaled = want_grad && fused_loss_ok(p, lp);
    r.psl_hard = hard_psl(lp) ? 1 : 0;
    r.w_spec = lp->w_spec;
    r.w_const = lp->w_const;
    r.w_smooth = lp->w_smooth;
    r.ext_cells = ((lp->match_target && lp->w_match != 0.f) || lp->w_width != 0.f || lp->w_cell != 0.f) ? 1 : 0;
    r.vals = v.vals;
    r.g_extra = (want_grad && needs_extra(lp)) ? v.extra : nullptr;
    return r;
}

// ---------------------------------------------------------- tuning cache --
// Autotuned schedules keyed by the device architecture and the plan's shapes
// (every waveform's N, M, lag window, kind, and the plan options that change
// the schedule).  Held in memory for the process; with the environment
// variable GRAF_AF_TUNE_CACHE naming a file, entries are also read from and
// appended to it, one line per entry:
//   <key> <one_launch> <items_per_slot> <ms> <classes> <variant per class...>
struct TuneEntry {
    bool one_launch = true;
    std::vector<int> forced;
    double items_per_slot = 0.0;
    float ms = 0.f;
};
std::mutex g_tune_mu;
std::vector<std::pair<std::string, TuneEntry>> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const af_plan* p) {
    hipDeviceProp_t prop;
    std::string arch = hipGetDeviceProperties(&prop, p->device) == hipSuccess ? prop.gcnArchName : "unknown";
    for (char& c : arch)
        if (c == ' ' || c == ':') c = '_';
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the shapes
    auto mix = [&](int64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (uint64_t)((v >> (8 * i)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    mix(p->batch);
    for (const af_wave& w : p->waves) {
        mix(w.n);
        mix(w.m);
        mix(w.max_lag);
        mix(w.flags);
    }
    mix(p->store_mode);
    mix(p->seg_iters_opt);
    mix(p->loss_passes_opt);
    char buf[64];
    std::snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
    return arch + "/" + buf;
}

void tune_load_file() {
    g_tune_loaded = true;
    const char* path = std::getenv("GRAF_AF_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char key[256];
    int one = 0, nc = 0;
    double ips = 0.0;
    float ms = 0.f;
    while (std::fscanf(f, "%255s %d %lf %f %d", key, &one, &ips, &ms, &nc) == 5) {
        if (nc < 0 || nc > 64) break;
        TuneEntry e;
        e.one_launch = one != 0;
        e.items_per_slot = ips;
        e.ms = ms;
        e.forced.resize(nc);
        bool ok = true;
        for (int i = 0; i < nc && ok; ++i) ok = std::fscanf(f, "%d", &e.forced[i]) == 1;
        if (!ok) break;
        g_tune.emplace_back(key, e);
    }
    std::fclose(f);
}

bool tune_lookup(const std::string& key, TuneEntry* out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) tune_load_file();
    for (auto it = g_tune.rbegin(); it != g_tune.rend(); ++it)
        if (it->first == key) {
            *out = it->second;
            return true;
        }
    return false;
}

void tune_store(const std::string& key, const TuneEntry& e) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) tune_load_file();
    g_tune.emplace_back(key, e);
    const char* path = std::getenv("GRAF_AF_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %.3f %.5f %d", key.c_str(), e.one_launch ? 1 : 0, e.items_per_slot, e.ms,
                 (int)e.forced.size());
    for (int v : e.forced) std::fprintf(f, " %d", v);
    std::fprintf(f, "\n");
    std::fclose(f);
}

// af_loss on a given workspace (the caller's, or af_loss_no_alloc's array)
af_status loss_call(const af_plan* p, const void* s, const af_loss_params* lp, float* terms, float* mag, void* grad_s,
                    void* ws, size_t ws_bytes, hipStream_t st) {
    af_status rc = check_common(p, s, ws, ws_bytes);
    if (rc != AF_OK) return rc;
    if ((rc = check_loss(p, lp)) != AF_OK) return rc;
    if (!aligned(mag, 16) || !aligned(grad_s, 8) || !aligned(terms, 4) || !aligned(lp->band_w, 4))
        return AF_ERR_INVALID_ARG;
    const WsView v = ws_view(p, ws);
    rc = loss_passes(p, s, lp, mag, grad_s != nullptr, v, st);
    if (rc != AF_OK) return rc;
    if (!terms && !grad_s) return AF_OK;
    ReduceArgs r = loss_reduce_args(p, s, lp, grad_s != nullptr, v);
    r.grad = (float2*)grad_s;
    r.terms = terms;
    return graf::launch_reduce(r, st) == hipSuccess ? AF_OK : AF_ERR_HIP;
}

}  // namespace

extern "C" {

const char* af_status_string(af_status s) {
    switch (s) {
        case AF_OK: return "ok";
        case AF_ERR_INVALID_ARG: return "invalid argument";
        case AF_ERR_UNSUPPORTED: return "unsupported shape (AF: M a power of two in [128, 32768], M >= 2N; GEMM: m, n multiples of 64 and of the tile, k of 32 x split)";
        case AF_ERR_BUDGET: return "workspace does not fit the budget";
        case AF_ERR_HIP: return "HIP runtime error";
        case AF_ERR_WORKSPACE: return "workspace too small";
        case AF_ERR_NO_DEVICE: return "no gfx950 device";
    }
    return "unknown status";
}

int32_t af_version(void) { return 100; }

af_status af_plan_create(int32_t batch, const af_wave* waves, const af_plan_opts* opts, af_plan** out) {
    if (!out) return AF_ERR_INVALID_ARG;
    *out = nullptr;
    af_status rc = validate_plan_inputs(batch, waves, opts);
    if (rc != AF_OK) return rc;

    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return AF_ERR_NO_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return AF_ERR_NO_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return AF_ERR_NO_DEVICE;

    af_plan* p = new (std::nothrow) af_plan();
    if (!p) return AF_ERR_HIP;
    p->device = dev;
    p->cus = prop.multiProcessorCount;
    p->batch = batch;
    p->waves.assign(waves, waves + batch);
    int64_t mmax = 0;
    for (af_wave& w : p->waves) {
        if (w.max_lag < 0) w.max_lag = w.n - 1;
        mmax = std::max<int64_t>(mmax, kernel_m(w));
        p->max_n = std::max(p->max_n, w.n);
        p->cells += grid_cells(w);
    }
    p->eps = opts->eps;
    p->store_mode = opts->store_mode;
    p->budget = opts->budget_bytes;
    p->seg_iters_opt = opts->segment_iters;
    p->loss_passes_opt = opts->loss_passes;
    p->one_launch = opts->launch_mode == 0;
    p->log2_mmax = ilog2(mmax);

    // twiddles exp(-j 2 pi i / MMAX), computed in double, rounded once
    std::vector<float2> tw((size_t)mmax);
    for (int64_t i = 0; i < mmax; ++i) {
        const double ang = -2.0 * M_PI * (double)i / (double)mmax;
        tw[(size_t)i] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    if (hipMalloc(&p->d_tw, tw.size() * sizeof(float2)) != hipSuccess ||
        hipMemcpy(p->d_tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) {
        free_tables(p);
        delete p;
        return AF_ERR_HIP;
    }

    p->opt_variant = opts->variant;
    if (opts->variant >= graf::kNumVariants) rc = AF_ERR_INVALID_ARG;
    else rc = build_schedule(p);
    if (rc != AF_OK) {
        free_tables(p);
        delete p;
        return rc;
    }
    if (hipMalloc(&p->d_queue, kMaxQueues * sizeof(int)) != hipSuccess ||
        make_streams(p, p->natural_classes) != AF_OK) {
        free_tables(p);
        delete p;
        return AF_ERR_HIP;
    }
    // this device's copy of af_loss_no_alloc's workspace, once per device; a
    // failure only disables that entry point
    resolve_scratch(dev);
    *out = p;
    return AF_OK;
}

void af_plan_destroy(af_plan* p) {
    if (!p) return;
    free_tables(p);
    delete p;
}

af_status af_plan_workspace_size(const af_plan* p, size_t* bytes) {
    if (!p || !bytes) return AF_ERR_INVALID_ARG;
    *bytes = p->ws_total;
    return AF_OK;
}

af_status af_plan_get_summary(const af_plan* p, af_plan_summary* o) {
    if (!p || !o) return AF_ERR_INVALID_ARG;
    o->cells = p->cells;
    o->store_bytes = p->store_bytes;
    o->workspace_bytes = (int64_t)p->ws_total;
    o->segments = p->n_segs;
    o->grid = p->classes.empty() ? 0 : p->classes[0].grid[graf::MODE_FUSED_ISL];
    o->variant = p->classes.empty() ? -1 : p->classes[0].variant;
    o->stores = p->stores ? 1 : 0;
    return AF_OK;
}

af_status af_forward(const af_plan* p, const void* s, float* mag, void* chi, float* energy, void* ws,
                     size_t ws_bytes, void* stream) {
    af_status rc = check_common(p, s, ws, ws_bytes);
    if (rc != AF_OK) return rc;
    if (!aligned(mag, 16) || !aligned(chi, 8) || !aligned(energy, 4)) return AF_ERR_INVALID_ARG;
    const WsView v = ws_view(p, ws);
    AfArgs a = base_args(p, s, v);
    a.mag = mag;
    a.chi = (float2*)chi;
    a.ystore = v.store;
    if (energy) a.energy = energy;
    return launch(p, chi ? graf::MODE_FWD : graf::MODE_FWD_MAG, a, (hipStream_t)stream);
}

af_status af_backward(const af_plan* p, const void* s, const float* grad_mag, void* grad_s, void* ws,
                      size_t ws_bytes, void* stream) {
    af_status rc = check_common(p, s, ws, ws_bytes);
    if (rc != AF_OK) return rc;
    if (!grad_mag || !grad_s) return AF_ERR_INVALID_ARG;
    if (!aligned(grad_mag, 16) || !aligned(grad_s, 8)) return AF_ERR_INVALID_ARG;
    const WsView v = ws_view(p, ws);
    AfArgs a = base_args(p, s, v);
    a.grad_mag = grad_mag;
    a.ystore = v.store;
    a.load_store = v.store != nullptr;
    rc = launch(p, graf::MODE_BWD_MAG, a, (hipStream_t)stream);
    if (rc != AF_OK) return rc;
    ReduceArgs r = reduce_args(p, s, v);
    r.grad = (float2*)grad_s;
    return graf::launch_reduce(r, (hipStream_t)stream) == hipSuccess ? AF_OK : AF_ERR_HIP;
}

af_status af_loss(const af_plan* p, const void* s, const af_loss_params* lp, float* terms, float* mag, void* grad_s,
                  void* ws, size_t ws_bytes, void* stream) {
    return loss_call(p, s, lp, terms, mag, grad_s, ws, ws_bytes, (hipStream_t)stream);
}

af_status af_loss_no_alloc(const af_plan* p, const void* s, const af_loss_params* lp, float* terms, float* mag,
                           void* grad_s, void* stream) {
    if (!p) return AF_ERR_INVALID_ARG;
    if (p->ws_total > kNoAllocWsBytes) return AF_ERR_WORKSPACE;
    void* ws = scratch_ptr(p->device);
    if (!ws) return AF_ERR_HIP;
    return loss_call(p, s, lp, terms, mag, grad_s, ws, kNoAllocWsBytes, (hipStream_t)stream);
}

af_status af_loss_stage(const af_plan* p, int32_t stage, const void* s, const af_loss_params* lp, float* terms,
                        float* mag, void* grad_s, void* ws, size_t ws_bytes, void* stream) {
    af_status rc = check_common(p, s, ws, ws_bytes);
    if (rc != AF_OK) return rc;
    if ((rc = check_loss(p, lp)) != AF_OK) return rc;
    if (!aligned(mag, 16) || !aligned(grad_s, 8) || !aligned(terms, 4) || !aligned(lp->band_w, 4))
        return AF_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const WsView v = ws_view(p, ws);
    AfArgs a = loss_args(p, s, lp, mag, v);
    const bool grad = grad_s != nullptr;
    const bool fwd_only = forward_only(lp, grad);
    const bool fused = !fwd_only && a.w_psl == 0.f;
    const bool fused_loss = !fwd_only && !fused && fused_loss_ok(p, lp);
    switch (stage) {
        case 0:
            if (fused) return launch(p, extended_terms(lp) ? graf::MODE_FUSED_EXT : graf::MODE_FUSED_ISL, a, st);
            if (fused_loss) return launch(p, graf::MODE_LOSS, a, st);
            a.ystore = fwd_only ? nullptr : v.store;
            return launch(p, fwd_only ? forward_mode(lp) : graf::MODE_FWD, a, st);
        case 1:
            if (!(fwd_only || fused || fused_loss)) {
                a.mag = nullptr;
                a.ystore = v.store;
                a.load_store = v.store != nullptr;
                rc = launch(p, graf::MODE_BWD_LOSS, a, st);
                if (rc != AF_OK) return rc;
            }
            return launch_extra(p, s, lp, grad, v, st);
        case 2: {
            if (!terms && !grad_s) return AF_OK;
            ReduceArgs r = loss_reduce_args(p, s, lp, grad, v);
            r.grad = (float2*)grad_s;
            r.terms = terms;
            return graf::launch_reduce(r, st) == hipSuccess ? AF_OK : AF_ERR_HIP;
        }
    }
    return AF_ERR_INVALID_ARG;
}

af_status af_spectral_variance(const af_plan* p, const void* s, float* value, void* grad_s, void* ws, size_t ws_bytes,
                               void* stream) {
    af_status rc = check_common(p, s, ws, ws_bytes);
    if (rc != AF_OK) return rc;
    if (!value || !aligned(value, 4) || !aligned(grad_s, 8)) return AF_ERR_INVALID_ARG;
    if (p->max_n > kMaxSpecN) return AF_ERR_UNSUPPORTED;
    const WsView v = ws_view(p, ws);
    graf::ExtraArgs e;
    std::memset(&e, 0, sizeof(e));
    e.s = (const float2*)s;
    e.waves = p->d_waves;
    e.tw = p->d_tw;
    e.log2_mmax = p->log2_mmax;
    e.spec = 1;
    e.w_spec = 1.f;
    e.g_extra = (float2*)grad_s;
    e.vals = v.vals;
    e.spec_out = value;
    return graf::launch_extra(e, p->batch, p->max_n, (hipStream_t)stream) == hipSuccess ? AF_OK : AF_ERR_HIP;
}

af_status af_project(const af_plan* p, const void* s, const float* mask, int32_t unit, void* out, void* stream) {
    if (!p || !s || !out || (unit != 0 && unit != 1)) return AF_ERR_INVALID_ARG;
    if (!aligned(s, 8) || !aligned(out, 8) || !aligned(mask, 4)) return AF_ERR_INVALID_ARG;
    if (mask && p->max_n > kMaxSpecN) return AF_ERR_UNSUPPORTED;
    graf::ProjectArgs a;
    a.s = (const float2*)s;
    a.waves = p->d_waves;
    a.mask = mask;
    a.unit = unit;
    a.out = (float2*)out;
    return graf::launch_project(a, p->batch, p->max_n, (hipStream_t)stream) == hipSuccess ? AF_OK : AF_ERR_HIP;
}

af_status af_scenario_combine(const af_plan* p, int32_t n_scen, const float* grids, const float* lambdas, float* out,
                              void* stream) {
    if (!p || n_scen < 1 || !grids || !lambdas || !out || !aligned(grids, 4) || !aligned(lambdas, 4) ||
        !aligned(out, 4))
        return AF_ERR_INVALID_ARG;
    return graf::launch_combine(grids, lambdas, n_scen, p->cells, out, (hipStream_t)stream) == hipSuccess
               ? AF_OK
               : AF_ERR_HIP;
}

// ------------------------------------------------------- cross-AF --
namespace {
af_status check_cross(const af_plan* p, const void* s, const void* u) {
    if (!p || !s || !u || !aligned(s, 8) || !aligned(u, 8)) return AF_ERR_INVALID_ARG;
    for (const af_plan::XClass& k : p->xclasses)
        if (!graf::cross_lg_supported(k.lg, k.circ)) return AF_ERR_UNSUPPORTED;
    // the kernels move the a and dL/da grids as 8-byte bin pairs
    for (const af_wave& w : p->waves)
        if (w.grid_off & 1) return AF_ERR_INVALID_ARG;
    return AF_OK;
}
size_t cross_slab_bytes(const af_plan* p) { return align256((size_t)p->slab_elems * sizeof(float2)); }
size_t cross_ws_bytes(const af_plan* p) {
    return 2 * cross_slab_bytes(p) + align256((size_t)p->n_segs * sizeof(double)) +
           align256((size_t)p->batch * 2 * sizeof(float));
}
graf::CrossArgs cross_args(const af_plan* p, const void* s, const void* u) {
    graf::CrossArgs a;
    std::memset(&a, 0, sizeof(a));
    a.s = (const float2*)s;
    a.u = (const float2*)u;
    a.waves = p->d_waves;
    a.tw = p->d_tw;
    a.log2_mmax = p->log2_mmax;
    a.eps = p->eps;
    return a;
}
af_status launch_cross_classes(const af_plan* p, int mode, graf::CrossArgs a, hipStream_t st) {
    const SegDesc* segs = p->one_active ? p->d_segs_x : p->d_segs;
    for (const af_plan::XClass& k : p->xclasses) {
        a.segs = segs + k.begin;
        if (graf::launch_cross(mode, k.lg, k.circ, a, k.count, st) != hipSuccess) return AF_ERR_HIP;
    }
    return AF_OK;
}
}  // namespace

af_status af_cross_workspace_size(const af_plan* p, size_t* bytes) {
    if (!p || !bytes) return AF_ERR_INVALID_ARG;
    *bytes = cross_ws_bytes(p);
    return AF_OK;
}

af_status af_cross_forward(const af_plan* p, const void* s, const void* u, float* mag, void* chi, float* energy,
                           void* stream) {
    af_status rc = check_cross(p, s, u);
    if (rc != AF_OK) return rc;
    if (!aligned(mag, 8) || !aligned(chi, 8) || !aligned(energy, 4)) return AF_ERR_INVALID_ARG;
    graf::CrossArgs a = cross_args(p, s, u);
    a.mag = mag;
    a.chi = (float2*)chi;
    a.energy = energy;
    return launch_cross_classes(p, 0, a, (hipStream_t)stream);
}

af_status af_cross_backward(const af_plan* p, const void* s, const void* u, const float* grad_mag, void* grad_s,
                            void* grad_u, void* ws, size_t ws_bytes, void* stream) {
    af_status rc = check_cross(p, s, u);
    if (rc != AF_OK) return rc;
    if (!grad_mag || !grad_s || !grad_u || !ws || !aligned(grad_mag, 4) || !aligned(grad_s, 8) ||
        !aligned(grad_u, 8) || !aligned(ws, 256))
        return AF_ERR_INVALID_ARG;
    if (ws_bytes < cross_ws_bytes(p)) return AF_ERR_WORKSPACE;
    char* b = (char*)ws;
    const size_t sb = cross_slab_bytes(p);
    graf::CrossArgs a = cross_args(p, s, u);
    a.grad_mag = grad_mag;
    a.slab_s = (float2*)b;
    a.slab_u = (float2*)(b + sb);
    a.part = (double*)(b + 2 * sb);
    a.energy = (float*)(b + 2 * sb + align256((size_t)p->n_segs * sizeof(double)));
    a.grad_s = (float2*)grad_s;
    a.grad_u = (float2*)grad_u;
    hipStream_t st = (hipStream_t)stream;
    rc = launch_cross_classes(p, 1, a, st);
    if (rc != AF_OK) return rc;
    return graf::launch_cross_reduce(a, p->batch, p->max_n, st) == hipSuccess ? AF_OK : AF_ERR_HIP;
}

af_status af_phase_to_signal(const float* phi, void* s, int64_t count, void* stream) {
    if (count < 0 || (count > 0 && (!phi || !s))) return AF_ERR_INVALID_ARG;
    return graf::launch_phase_to_signal(phi, (float2*)s, count, (hipStream_t)stream) == hipSuccess ? AF_OK
                                                                                                 : AF_ERR_HIP;
}

af_status af_optim_step(const af_plan* p, float* phi, float* adam_m, float* adam_v, void* s, int32_t* step,
                        const af_loss_params* lp, const af_adam_params* ad, float* terms, void* ws, size_t ws_bytes,
                        void* stream) {
    af_status rc = check_common(p, s, ws, ws_bytes);
    if (rc != AF_OK) return rc;
    if ((rc = check_loss(p, lp)) != AF_OK) return rc;
    if (!phi || !adam_m || !adam_v || !step || !ad) return AF_ERR_INVALID_ARG;
    if (!(ad->lr > 0.f) || !(ad->beta1 >= 0.f && ad->beta1 < 1.f) || !(ad->beta2 >= 0.f && ad->beta2 < 1.f) ||
        !(ad->eps >= 0.f))
        return AF_ERR_INVALID_ARG;
    const WsView v = ws_view(p, ws);
    rc = loss_passes(p, s, lp, nullptr, true, v, (hipStream_t)stream);
    if (rc != AF_OK) return rc;
    ReduceArgs r = loss_reduce_args(p, s, lp, true, v);
    r.terms = terms;
    r.phi = phi;
    r.adam_m = adam_m;
    r.adam_v = adam_v;
    r.s_next = (float2*)s;
    r.step = step;
    r.lr = ad->lr;
    r.beta1 = ad->beta1;
    r.beta2 = ad->beta2;
    r.adam_eps = ad->eps;
    return graf::launch_reduce_adam(r, (hipStream_t)stream) == hipSuccess ? AF_OK : AF_ERR_HIP;
}

af_status af_plan_autotune(af_plan* p, const void* s, void* ws, size_t ws_bytes, void* stream, int32_t* chosen,
                           float* best_ms) {
    if (!p || !s || !ws) return AF_ERR_INVALID_ARG;
    // a schedule tuned before for the same device architecture and plan
    // shapes (in this process, or in the file GRAF_AF_TUNE_CACHE names)
    const std::string key = tune_key(p);
    TuneEntry hit;
    if (tune_lookup(key, &hit) && (int)hit.forced.size() == p->natural_classes) {
        p->one_launch = hit.one_launch;
        p->forced = hit.forced;
        p->items_per_slot = hit.items_per_slot;
        af_status rc = build_schedule(p);
        if (rc == AF_OK && p->ws_total <= ws_bytes) {
            if (chosen) *chosen = p->classes.empty() ? -1 : p->classes[0].variant;
            if (best_ms) *best_ms = hit.ms;
            return AF_OK;
        }
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return AF_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return AF_ERR_HIP;
    }
    af_loss_params lp;
    std::memset(&lp, 0, sizeof(lp));
    lp.w_isl = 1.f;
    lp.psl_temp = 0.05f;
    // ms per forward + fused loss pass of one class (c >= 0) or of the whole
    // plan (c < 0, classes concurrent), or < 0 when the schedule does not run
    auto time_schedule = [&](int c) -> float {
        if (build_schedule(p) != AF_OK || p->ws_total > ws_bytes) return -1.f;
        const WsView view = ws_view(p, ws);
        bool ok = true;
        for (int it = 0; it < 2 && ok; ++it) ok = loss_passes(p, s, &lp, nullptr, true, view, st, c) == AF_OK;
        if (!ok || hipStreamSynchronize(st) != hipSuccess) return -1.f;
        const int reps = 5;
        (void)hipEventRecord(e0, st);
        for (int it = 0; it < reps && ok; ++it) {
            AfArgs a = base_args(p, s, view);
            ok = launch(p, graf::MODE_FWD, a, st, c) == AF_OK && loss_passes(p, s, &lp, nullptr, true, view, st, c) == AF_OK;
        }
        (void)hipEventRecord(e1, st);
        if (!ok || hipEventSynchronize(e1) != hipSuccess) return -1.f;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        return ms / reps;
    };
    const bool one_before = p->one_launch;
    const std::vector<int> forced_before = p->forced;
    const double ips_before = p->items_per_slot;
    p->items_per_slot = 0.0;
    af_status rc = AF_OK;
    // 1. per class: every variant that fits the class, the class timed alone
    p->one_launch = false;
    p->forced.assign(p->natural_classes, -1);
    if (build_schedule(p) != AF_OK) rc = AF_ERR_UNSUPPORTED;
    const int NC = p->natural_classes;
    std::vector<af_plan::Class> nat = p->classes;
    std::vector<int> best(NC, -1);
    for (int c = 0; c < NC && rc == AF_OK; ++c) {
        float best_t = 0.f;
        for (int v = 0; v < graf::kNumVariants; ++v) {
            if (v == graf::kUnionVariant || !variant_fits(v, nat[c].lg, nat[c].max_n, nat[c].circ)) continue;
            p->forced[c] = v;
            const float ms = time_schedule(c);
            if (ms >= 0.f && (best[c] < 0 || ms < best_t)) {
                best[c] = v;
                best_t = ms;
            }
        }
        if (best[c] < 0) rc = AF_ERR_UNSUPPORTED;
        p->forced[c] = best[c];
    }
    // 2. the tuned classes together, with one, two or four work items per
    // resident work group; then one launch of all of them, with three, six
    // or twelve items per group (shorter last items against more staging)
    float t_per = -1.f, t_one = -1.f;
    double ips_per = 0.0, ips_one = 0.0;
    if (rc == AF_OK) {
        for (double ips : {1.0, 2.0, 4.0}) {
            p->items_per_slot = ips;
            const float t = time_schedule(-1);
            if (t >= 0.f && (t_per < 0.f || t < t_per)) {
                t_per = t;
                ips_per = ips;
            }
        }
    }
    if (rc == AF_OK && NC > 1) {
        const std::vector<int> tuned = p->forced;
        p->forced.assign(NC, -1);
        p->one_launch = true;
        for (double ips : {3.0, 6.0, 12.0}) {
            p->items_per_slot = ips;
            if (build_schedule(p) != AF_OK || p->classes.size() != 1 || p->classes[0].variant != graf::kUnionVariant)
                break;
            const float t = time_schedule(-1);
            if (t >= 0.f && (t_one < 0.f || t < t_one)) {
                t_one = t;
                ips_one = ips;
            }
        }
        if (!(t_one >= 0.f && (t_per < 0.f || t_one < t_per))) {
            p->one_launch = false;
            p->forced = tuned;
            t_one = -1.f;
        }
    }
    p->items_per_slot = t_one >= 0.f ? ips_one : ips_per;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == AF_OK && t_per < 0.f && t_one < 0.f) rc = AF_ERR_UNSUPPORTED;
    if (rc != AF_OK) {
        p->one_launch = one_before;
        p->forced = forced_before;
        p->items_per_slot = ips_before;
        (void)build_schedule(p);
        return rc;
    }
    rc = build_schedule(p);
    if (rc != AF_OK) return rc;
    const float t_best = t_one >= 0.f ? t_one : t_per;
    tune_store(key, TuneEntry{p->one_launch, p->forced, p->items_per_slot, t_best});
    if (chosen) *chosen = p->classes.empty() ? -1 : p->classes[0].variant;
    if (best_ms) *best_ms = t_best;
    return AF_OK;
}

}  // extern "C"
