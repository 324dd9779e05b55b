// Kernels of the proposal network (paper Sec. 6.1, Fig. 1: design
// parameters -> network -> waveform -> ambiguity function -> loss): a BF16
// MFMA GEMM with fused epilogues and deterministic split-k, column sums,
// Adam, conversions and the phase-gradient map.  gfx950:
// v_mfma_f32_32x32x16_bf16, FP32 accumulation.
#include "../../include/graf_af.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

namespace graf_mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

enum Layout { L_NT = 0, L_NN = 1, L_TN = 2 };
enum Epi { E_F32 = 0, E_BIAS_F32 = 1, E_BIAS_GELU = 2, E_GELU_BWD = 3, E_PARTIAL = 4 };

// LDS row pitch for k depth BK (64 or 128): BK + 8 bf16, i.e. 36 or 68
// banks, so the 16 rows that one quarter-wave's 16-byte fragment reads touch
// start banks 36 r or 68 r mod 64, all distinct groups of four.  k must be a
// multiple of kMinK.
constexpr int kMinK = 64;

struct GemmArgs {
    int m, n, k;
    int k_split;          // k range of one blockIdx.z (the whole k without split)
    const __bf16* a;
    const __bf16* b;
    const float* bias;    // [n]
    const float* aux;     // [m][n] pre-activation (E_GELU_BWD)
    float* out_f32;       // [m][n]
    __bf16* out_bf16;     // [m][n]
    float* part;          // [splits][m][n] partial sums (E_PARTIAL)
};

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// The epilogue of one output element C[row][col] = v (idx = row * n + col).
template <int EPI>
__device__ __forceinline__ void epilogue_store(const GemmArgs& g, int64_t idx, int col, float v) {
    if (EPI == E_F32) {
        g.out_f32[idx] = v;
    } else if (EPI == E_BIAS_F32) {
        g.out_f32[idx] = v + g.bias[col];
    } else if (EPI == E_BIAS_GELU) {
        const float z = v + g.bias[col];
        g.out_f32[idx] = z;
        g.out_bf16[idx] = (__bf16)gelu(z);
    } else {  // E_GELU_BWD: dZ = dA * GELU'(Z)
        const float dz = v * gelu_grad(g.aux[idx]);
        g.out_f32[idx] = dz;
        g.out_bf16[idx] = (__bf16)dz;
    }
}

// Operand tile of BR rows x BK k, from a k-contiguous array (element (r, k)
// at p[r * ld + k]): 16-byte chunks of 8 k, BR BK / 2048 per thread, stored
// as they come.
template <int BR, int BK>
struct LoadKContig {
    static constexpr int LDK = BK + 8, CPR = BK / 8, CH = BR * BK / 2048;
    u32x4 v[CH];
    __device__ __forceinline__ void load(const __bf16* p, int ld, int r0, int k0) {
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int c = (int)threadIdx.x + 256 * i;
            v[i] = *reinterpret_cast<const u32x4*>(p + (int64_t)(r0 + c / CPR) * ld + k0 + (c % CPR) * 8);
        }
    }
    __device__ __forceinline__ void store(__bf16* lds) const {
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int c = (int)threadIdx.x + 256 * i;
            *reinterpret_cast<u32x4*>(lds + (c / CPR) * LDK + (c % CPR) * 8) = v[i];
        }
    }
};

// Operand tile of BR rows x BK k, from a row-contiguous array (element
// (r, k) at p[k * ld + r]), transposed on the way into the k-contiguous LDS
// tile.  Thread unit: rows 2q, 2q + 1 at 8 consecutive k, read as one 4-byte
// pair per k (a wavefront reads whole rows of the array, 128 or 256 bytes)
// and repacked into one 16-byte LDS write per row; BR BK / 4096 units per
// thread.
template <int BR, int BK>
struct LoadRContig {
    static constexpr int LDK = BK + 8, Q = BR / 2, U = BR * BK / 4096;
    unsigned v[U][8];
    __device__ __forceinline__ void load(const __bf16* p, int ld, int r0, int k0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = (int)threadIdx.x + 256 * u;
            const int q = c % Q, kq = c / Q;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                v[u][j] = *reinterpret_cast<const unsigned*>(p + (int64_t)(k0 + kq * 8 + j) * ld + r0 + 2 * q);
        }
    }
    __device__ __forceinline__ void store(__bf16* lds) const {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = (int)threadIdx.x + 256 * u;
            const int q = c % Q, kq = c / Q;
            unsigned lo[4], hi[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                // low halves: row 2q at k = 2j, 2j + 1; high halves: row 2q + 1
                lo[j] = (v[u][2 * j] & 0xffffu) | (v[u][2 * j + 1] << 16);
                hi[j] = (v[u][2 * j] >> 16) | (v[u][2 * j + 1] & 0xffff0000u);
            }
            __bf16* row = lds + (2 * q) * LDK + kq * 8;
            *reinterpret_cast<u32x4*>(row) = u32x4{lo[0], lo[1], lo[2], lo[3]};
            *reinterpret_cast<u32x4*>(row + LDK) = u32x4{hi[0], hi[1], hi[2], hi[3]};
        }
    }
};

// C[m][n] = sum_k A~[m][k] B~[n][k] over this block's k range, with
//   L_NT: A~ = A [m][k],   B~ = B [n][k]      (X W^T)
//   L_NN: A~ = A [m][k],   B~ = B^T, B [k][n] (dZ W)
//   L_TN: A~ = A^T, A [k][m], B~ = B^T, B [k][n] (dZ^T A)
// Block tile BM x BN, 256 threads as 2 x 2 wavefronts, each owning
// (BM/2) x (BN/2) as 32 x 32 MFMA tiles, k in tiles of BK.  Operand tiles
// go through registers into a double-buffered LDS pair in dynamic shared
// memory (the next tile's global loads are in flight while the current one
// feeds the MFMAs; one barrier per tile).  E_PARTIAL writes the raw sums of
// split blockIdx.z to part.
template <int BM, int BN, int BK>
constexpr int gemm_lds_bytes() {
    return 2 * (BM + BN) * (BK + 8) * 2;
}

template <int LAYOUT, int EPI, int BM, int BN, int BK>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
    constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 32, TN = WN / 32;
    constexpr int LDK = BK + 8, TILE = (BM + BN) * LDK;
    extern __shared__ __attribute__((aligned(16))) __bf16 lds[];
    using LA = typename std::conditional<LAYOUT == L_TN, LoadRContig<BM, BK>, LoadKContig<BM, BK>>::type;
    using LB = typename std::conditional<LAYOUT == L_NT, LoadKContig<BN, BK>, LoadRContig<BN, BK>>::type;
    const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
    const int wm = w >> 1, wn = w & 1;
    // XCD-aware tile order: work groups are dealt to the eight XCDs in turn
    // by linear index, so hardware group h runs on XCD h mod 8; give XCD c
    // the c-th contiguous eighth of the row-major tile order (a band of
    // output rows: its A rows and the B it needs stay in that XCD's L2)
    const int nx = (int)gridDim.x, tiles = nx * (int)gridDim.y;
    const int hw = (int)blockIdx.y * nx + (int)blockIdx.x;
    const int lid = (tiles & 7) == 0 ? (hw & 7) * (tiles >> 3) + (hw >> 3) : hw;
    const int m0 = (lid / nx) * BM, n0 = (lid % nx) * BN;
    const int kb = (int)blockIdx.z * g.k_split;
    const int nk = g.k_split / BK;
    const int lda = LAYOUT == L_TN ? g.m : g.k;
    const int ldb = LAYOUT == L_NT ? g.k : g.n;
    LA la;
    LB lb;
    f32x16 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x16{};

    la.load(g.a, lda, m0, kb);
    lb.load(g.b, ldb, n0, kb);
    la.store(lds);
    lb.store(lds + BM * LDK);
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
        const __bf16* cur = lds + (it & 1) * TILE;
        if (it + 1 < nk) {
            la.load(g.a, lda, m0, kb + (it + 1) * BK);
            lb.load(g.b, ldb, n0, kb + (it + 1) * BK);
        }
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            bf16x8 af[TM], bf[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i)
                af[i] = *reinterpret_cast<const bf16x8*>(cur + (wm * WM + 32 * i + (lane & 31)) * LDK + kk +
                                                         8 * (lane >> 5));
#pragma unroll
            for (int j = 0; j < TN; ++j)
                bf[j] = *reinterpret_cast<const bf16x8*>(cur + (BM + wn * WN + 32 * j + (lane & 31)) * LDK + kk +
                                                         8 * (lane >> 5));
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        if (it + 1 < nk) {
            __bf16* nxt = lds + ((it + 1) & 1) * TILE;
            la.store(nxt);
            lb.store(nxt + BM * LDK);
        }
        __syncthreads();
    }

    // D layout: register r of lane l holds row 8 (r/4) + 4 (l/32) + r%4, column l%32
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int col = n0 + wn * WN + 32 * j + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm * WM + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int64_t idx = (int64_t)row * g.n + col;
                if (EPI == E_PARTIAL)
                    g.part[(int64_t)blockIdx.z * g.m * g.n + idx] = acc[i][j][r];
                else
                    epilogue_store<EPI>(g, idx, col, acc[i][j][r]);
            }
        }
}

// Sum of the split partials in split order, then the epilogue: four
// consecutive elements per thread.
template <int EPI>
__global__ __launch_bounds__(256) void split_reduce_kernel(GemmArgs g, int splits) {
    const int64_t mn = (int64_t)g.m * g.n;
    const int64_t i4 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (i4 >= mn) return;
    float4 s = *reinterpret_cast<const float4*>(g.part + i4);
    for (int z = 1; z < splits; ++z) {
        const float4 p = *reinterpret_cast<const float4*>(g.part + z * mn + i4);
        s.x += p.x;
        s.y += p.y;
        s.z += p.z;
        s.w += p.w;
    }
    const int col = (int)(i4 % g.n);
    epilogue_store<EPI>(g, i4 + 0, col + 0, s.x);
    epilogue_store<EPI>(g, i4 + 1, col + 1, s.y);
    epilogue_store<EPI>(g, i4 + 2, col + 2, s.z);
    epilogue_store<EPI>(g, i4 + 3, col + 3, s.w);
}

// Column sums in two fixed-order stages: block (x, y) sums rows
// [y * rows_per, (y + 1) * rows_per) of columns 256 x + t into part[y][c],
// then colsum_final adds the row-chunk partials in chunk order.
__global__ __launch_bounds__(256) void colsum_partial_kernel(int rows, int cols, int rows_per, const float* in,
                                                             float* part) {
    const int c = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (c >= cols) return;
    const int r0 = (int)blockIdx.y * rows_per;
    const int r1 = min(rows, r0 + rows_per);
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int r = r0;
    for (; r + 4 <= r1; r += 4) {
        s0 += in[(int64_t)r * cols + c];
        s1 += in[(int64_t)(r + 1) * cols + c];
        s2 += in[(int64_t)(r + 2) * cols + c];
        s3 += in[(int64_t)(r + 3) * cols + c];
    }
    for (; r < r1; ++r) s0 += in[(int64_t)r * cols + c];
    part[(int64_t)blockIdx.y * cols + c] = (s0 + s1) + (s2 + s3);
}

__global__ __launch_bounds__(256) void colsum_final_kernel(int cols, int chunks, const float* part, float* out) {
    const int c = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
#pragma unroll 8
    for (int y = 0; y < chunks; ++y) s += part[(int64_t)y * cols + c];
    out[c] = s;
}

__global__ __launch_bounds__(256) void adam_kernel(int64_t count, float* p, const float* g, float* m, float* v,
                                                   float bc1, float bc2, float lr, float b1, float b2, float eps,
                                                   __bf16* p16) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
    if (p16) p16[i] = (__bf16)pi;
}

__global__ __launch_bounds__(256) void to_bf16_kernel(int64_t count, const float* in, __bf16* out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) out[i] = (__bf16)in[i];
}

// dL/dphi = 2 Im(conj(s) dL/d conj(s)) for s = exp(j phi)
__global__ __launch_bounds__(256) void phase_grad_kernel(int64_t count, const float2* s, const float2* g, float* out,
                                                         __bf16* out16) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const float2 a = s[i], b = g[i];
    const float d = 2.f * (a.x * b.y - a.y * b.x);
    out[i] = d;
    if (out16) out16[i] = (__bf16)d;
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// Compute units of the current device (cached per device).
static int device_cus() {
    static int cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] <= 0) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
        cus[dev] = c;
    }
    return cus[dev];
}

// Tile ids 1-8: BM x BN x BK = 128x128, 128x64, 64x128, 64x64 with BK 64
// (1-4), then the same with BK 128 (5-8).
constexpr int kTiles = 8;
constexpr int kTileM[kTiles + 1] = {0, 128, 128, 64, 64, 128, 128, 64, 64};
constexpr int kTileN[kTiles + 1] = {0, 128, 64, 128, 64, 128, 64, 128, 64};
constexpr int kTileK[kTiles + 1] = {0, 64, 64, 64, 64, 128, 128, 128, 128};
constexpr int kMaxSplit = 16;

static bool split_ok(int k, int bk, int s) { return s >= 1 && s <= kMaxSplit && k % (s * bk) == 0; }
static bool tile_ok(int m, int n, int k, int c) { return m % kTileM[c] == 0 && n % kTileN[c] == 0 && k % kTileK[c] == 0; }

// Resolve tile and split: explicit values are checked; the automatic choice
// takes the 64 x 64 x 64 tile (four work groups per compute unit hide the
// operand round trips better than one large tile, measured over the
// proposal network's shapes) and splits k (powers of two, at least 4 k
// tiles per split) until the grid covers every compute unit twice.
static af_status resolve(int m, int n, int k, int tile, int split, int* tile_out, int* split_out) {
    if (m <= 0 || n <= 0 || k <= 0 || m % 64 || n % 64 || k % kMinK) return AF_ERR_UNSUPPORTED;
    if (tile < 0 || tile > kTiles || split < 0) return AF_ERR_INVALID_ARG;
    if (tile > 0 && !tile_ok(m, n, k, tile)) return AF_ERR_UNSUPPORTED;
    if (tile == 0) tile = 4;
    const int bk = kTileK[tile];
    if (split > 0 && !split_ok(k, bk, split)) return AF_ERR_UNSUPPORTED;
    if (split == 0) {
        const int cus = device_cus();
        const int64_t blocks = (int64_t)(m / kTileM[tile]) * (n / kTileN[tile]);
        split = 1;
        while (blocks * split < 2 * cus && split_ok(k, bk, 2 * split) && k / (2 * split) >= 4 * bk) split *= 2;
    }
    *tile_out = tile;
    *split_out = split;
    return AF_OK;
}

template <int LAYOUT, int EPI, int BM, int BN, int BK>
static hipError_t launch_one(const dim3& grid, const GemmArgs& g, hipStream_t st) {
    constexpr int lds = gemm_lds_bytes<BM, BN, BK>();
    static bool attr = false;  // raise the dynamic LDS limit once per instance
    if (!attr) {
        const hipError_t e =
            hipFuncSetAttribute((const void*)gemm_kernel<LAYOUT, EPI, BM, BN, BK>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((gemm_kernel<LAYOUT, EPI, BM, BN, BK>), grid, dim3(256), lds, st, g);
    return hipGetLastError();
}

template <int LAYOUT, int BM, int BN, int BK>
static hipError_t launch_tile(int epi, const GemmArgs& g, int splits, hipStream_t st) {
    const dim3 grid(g.n / BN, g.m / BM, splits);
    switch (splits > 1 ? (int)E_PARTIAL : epi) {
        case E_F32: return launch_one<LAYOUT, E_F32, BM, BN, BK>(grid, g, st);
        case E_BIAS_F32: return launch_one<LAYOUT, E_BIAS_F32, BM, BN, BK>(grid, g, st);
        case E_BIAS_GELU: return launch_one<LAYOUT, E_BIAS_GELU, BM, BN, BK>(grid, g, st);
        case E_GELU_BWD: return launch_one<LAYOUT, E_GELU_BWD, BM, BN, BK>(grid, g, st);
        case E_PARTIAL: return launch_one<LAYOUT, E_PARTIAL, BM, BN, BK>(grid, g, st);
    }
    return hipErrorInvalidValue;
}

template <int LAYOUT>
static hipError_t launch_layout(int tile, int epi, const GemmArgs& g, int splits, hipStream_t st) {
    switch (tile) {
        case 1: return launch_tile<LAYOUT, 128, 128, 64>(epi, g, splits, st);
        case 2: return launch_tile<LAYOUT, 128, 64, 64>(epi, g, splits, st);
        case 3: return launch_tile<LAYOUT, 64, 128, 64>(epi, g, splits, st);
        case 4: return launch_tile<LAYOUT, 64, 64, 64>(epi, g, splits, st);
        case 5: return launch_tile<LAYOUT, 128, 128, 128>(epi, g, splits, st);
        case 6: return launch_tile<LAYOUT, 128, 64, 128>(epi, g, splits, st);
        case 7: return launch_tile<LAYOUT, 64, 128, 128>(epi, g, splits, st);
        case 8: return launch_tile<LAYOUT, 64, 64, 128>(epi, g, splits, st);
    }
    return hipErrorInvalidValue;
}

static hipError_t launch_split_reduce(int epi, const GemmArgs& g, int splits, hipStream_t st) {
    const int64_t quads = (int64_t)g.m * g.n / 4;
    const dim3 grid((unsigned)((quads + 255) / 256)), block(256);
    switch (epi) {
        case E_F32: hipLaunchKernelGGL(split_reduce_kernel<E_F32>, grid, block, 0, st, g, splits); break;
        case E_BIAS_F32: hipLaunchKernelGGL(split_reduce_kernel<E_BIAS_F32>, grid, block, 0, st, g, splits); break;
        case E_BIAS_GELU: hipLaunchKernelGGL(split_reduce_kernel<E_BIAS_GELU>, grid, block, 0, st, g, splits); break;
        case E_GELU_BWD: hipLaunchKernelGGL(split_reduce_kernel<E_GELU_BWD>, grid, block, 0, st, g, splits); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Row chunks of the two-stage column sum: about two blocks per compute unit.
static void colsum_chunks(int rows, int cols, int* chunks, int* rows_per) {
    const int cb = (cols + 255) / 256;
    const int want = (2 * device_cus() + cb - 1) / cb;
    const int rp = std::max(8, (rows + want - 1) / want);
    *rows_per = rp;
    *chunks = (rows + rp - 1) / rp;
}

}  // namespace graf_mlp

using namespace graf_mlp;

extern "C" {

af_status af_gemm_config(int32_t m, int32_t n, int32_t k, int32_t tile, int32_t split_k, int32_t* tile_out,
                         int32_t* split_out, size_t* ws_bytes) {
    int tl = 0, sp = 0;
    const af_status rc = resolve(m, n, k, tile, split_k, &tl, &sp);
    if (rc != AF_OK) return rc;
    if (tile_out) *tile_out = tl;
    if (split_out) *split_out = sp;
    if (ws_bytes) *ws_bytes = sp > 1 ? (size_t)sp * (size_t)m * (size_t)n * sizeof(float) : 0;
    return AF_OK;
}

af_status af_gemm_bf16(int32_t layout, int32_t epilogue, int32_t m, int32_t n, int32_t k, const void* a,
                       const void* b, const float* bias, const float* aux, float* out_f32, void* out_bf16,
                       int32_t tile, int32_t split_k, void* ws, size_t ws_bytes, void* stream) {
    if (layout < 0 || layout > 2 || epilogue < 0 || epilogue > 3) return AF_ERR_INVALID_ARG;
    if (!a || !b || !out_f32) return AF_ERR_INVALID_ARG;
    int tl = 0, sp = 0;
    const af_status rc = resolve(m, n, k, tile, split_k, &tl, &sp);
    if (rc != AF_OK) return rc;
    if (!aligned16(a) || !aligned16(b)) return AF_ERR_INVALID_ARG;
    if ((epilogue == E_BIAS_F32 || epilogue == E_BIAS_GELU) && !bias) return AF_ERR_INVALID_ARG;
    if ((epilogue == E_BIAS_GELU || epilogue == E_GELU_BWD) && !out_bf16) return AF_ERR_INVALID_ARG;
    if (epilogue == E_GELU_BWD && !aux) return AF_ERR_INVALID_ARG;
    const size_t need = sp > 1 ? (size_t)sp * (size_t)m * (size_t)n * sizeof(float) : 0;
    if (need && (!ws || ws_bytes < need)) return AF_ERR_WORKSPACE;
    if (need && !aligned16(ws)) return AF_ERR_INVALID_ARG;
    GemmArgs g{m, n, k, k / sp, (const __bf16*)a, (const __bf16*)b, bias, aux, out_f32, (__bf16*)out_bf16,
               (float*)ws};
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = layout == L_NT   ? launch_layout<L_NT>(tl, epilogue, g, sp, st)
                   : layout == L_NN ? launch_layout<L_NN>(tl, epilogue, g, sp, st)
                                    : launch_layout<L_TN>(tl, epilogue, g, sp, st);
    if (e == hipSuccess && sp > 1) e = launch_split_reduce(epilogue, g, sp, st);
    return e == hipSuccess ? AF_OK : AF_ERR_HIP;
}

af_status af_colsum_workspace_size(int32_t rows, int32_t cols, size_t* bytes) {
    if (rows <= 0 || cols <= 0 || !bytes) return AF_ERR_INVALID_ARG;
    int chunks = 0, rows_per = 0;
    colsum_chunks(rows, cols, &chunks, &rows_per);
    *bytes = (size_t)chunks * (size_t)cols * sizeof(float);
    return AF_OK;
}

af_status af_colsum(int32_t rows, int32_t cols, const float* in, float* out, void* ws, size_t ws_bytes,
                    void* stream) {
    if (rows <= 0 || cols <= 0 || !in || !out) return AF_ERR_INVALID_ARG;
    int chunks = 0, rows_per = 0;
    colsum_chunks(rows, cols, &chunks, &rows_per);
    if (!ws || ws_bytes < (size_t)chunks * (size_t)cols * sizeof(float)) return AF_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const unsigned cb = (unsigned)((cols + 255) / 256);
    hipLaunchKernelGGL(colsum_partial_kernel, dim3(cb, (unsigned)chunks), dim3(256), 0, st, rows, cols, rows_per, in,
                       (float*)ws);
    if (hipGetLastError() != hipSuccess) return AF_ERR_HIP;
    hipLaunchKernelGGL(colsum_final_kernel, dim3(cb), dim3(256), 0, st, cols, chunks, (const float*)ws, out);
    return hipGetLastError() == hipSuccess ? AF_OK : AF_ERR_HIP;
}

af_status af_adam_update(int64_t count, float* param, const float* grad, float* m, float* v, int32_t step,
                         const af_adam_params* ad, void* param_bf16, void* stream) {
    if (count < 0 || (count > 0 && (!param || !grad || !m || !v)) || !ad || step < 1) return AF_ERR_INVALID_ARG;
    if (count == 0) return AF_OK;
    const float bc1 = 1.f - powf(ad->beta1, (float)step);
    const float bc2 = 1.f - powf(ad->beta2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, (hipStream_t)stream, count,
                       param, grad, m, v, bc1, bc2, ad->lr, ad->beta1, ad->beta2, ad->eps, (__bf16*)param_bf16);
    return hipGetLastError() == hipSuccess ? AF_OK : AF_ERR_HIP;
}

af_status af_to_bf16(int64_t count, const float* in, void* out, void* stream) {
    if (count < 0 || (count > 0 && (!in || !out))) return AF_ERR_INVALID_ARG;
    if (count == 0) return AF_OK;
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, (hipStream_t)stream, count,
                       in, (__bf16*)out);
    return hipGetLastError() == hipSuccess ? AF_OK : AF_ERR_HIP;
}

af_status af_phase_grad(int64_t count, const void* s, const void* grad_s, float* out, void* out_bf16, void* stream) {
    if (count < 0 || (count > 0 && (!s || !grad_s || !out))) return AF_ERR_INVALID_ARG;
    if (count == 0) return AF_OK;
    hipLaunchKernelGGL(phase_grad_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       count, (const float2*)s, (const float2*)grad_s, out, (__bf16*)out_bf16);
    return hipGetLastError() == hipSuccess ? AF_OK : AF_ERR_HIP;
}

}  // extern "C"
