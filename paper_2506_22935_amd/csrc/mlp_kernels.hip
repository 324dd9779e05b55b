// Kernels of the proposal network (paper Sec. 6.1, Fig. 1: design
// parameters -> network -> waveform -> ambiguity function -> loss): a BF16
// MFMA GEMM with fused epilogues, column sums, Adam, conversions and the
// phase-gradient map.  gfx950: v_mfma_f32_32x32x16_bf16, FP32 accumulation.
#include "../../include/graf_af.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace graf_mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

enum Layout { L_NT = 0, L_NN = 1, L_TN = 2 };
enum Epi { E_F32 = 0, E_BIAS_F32 = 1, E_BIAS_GELU = 2, E_GELU_BWD = 3 };

constexpr int BM = 64, BN = 64, BK = 32, PAD = 8;

struct GemmArgs {
    int m, n, k;
    const __bf16* a;
    const __bf16* b;
    const float* bias;   // [n]
    const float* aux;    // [m][n] pre-activation (E_GELU_BWD)
    float* out_f32;      // [m][n]
    __bf16* out_bf16;    // [m][n]
};

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// C[m][n] = sum_k A~[m][k] B~[n][k] with
//   L_NT: A~ = A [m][k],   B~ = B [n][k]      (X W^T)
//   L_NN: A~ = A [m][k],   B~ = B^T, B [k][n] (dZ W)
//   L_TN: A~ = A^T, A [k][m], B~ = B^T, B [k][n] (dZ^T A)
// Tiles of 64 x 64 per 256-thread block; wave w owns rows 32 (w >> 1) and
// columns 32 (w & 1) of the tile.  Both operand tiles sit in LDS with k
// contiguous, so the MFMA fragments are 16-byte LDS reads.
template <int LAYOUT, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) __bf16 As[BM][BK + PAD];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[BN][BK + PAD];
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    f32x16 acc = {};

    for (int k0 = 0; k0 < g.k; k0 += BK) {
        // A tile -> As[row][k]
        if (LAYOUT == L_TN) {
            const int kr = t >> 3, mc = (t & 7) * 8;
            const bf16x8 v = *reinterpret_cast<const bf16x8*>(g.a + (int64_t)(k0 + kr) * g.m + m0 + mc);
#pragma unroll
            for (int i = 0; i < 8; ++i) As[mc + i][kr] = v[i];
        } else {
            const int r = t >> 2, kc = (t & 3) * 8;
            *reinterpret_cast<bf16x8*>(&As[r][kc]) =
                *reinterpret_cast<const bf16x8*>(g.a + (int64_t)(m0 + r) * g.k + k0 + kc);
        }
        // B tile -> Bs[col][k]
        if (LAYOUT == L_NT) {
            const int r = t >> 2, kc = (t & 3) * 8;
            *reinterpret_cast<bf16x8*>(&Bs[r][kc]) =
                *reinterpret_cast<const bf16x8*>(g.b + (int64_t)(n0 + r) * g.k + k0 + kc);
        } else {
            const int kr = t >> 3, nc = (t & 7) * 8;
            const bf16x8 v = *reinterpret_cast<const bf16x8*>(g.b + (int64_t)(k0 + kr) * g.n + n0 + nc);
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[nc + i][kr] = v[i];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            const bf16x8 af = *reinterpret_cast<const bf16x8*>(&As[wm * 32 + (lane & 31)][kk + 8 * (lane >> 5)]);
            const bf16x8 bf = *reinterpret_cast<const bf16x8*>(&Bs[wn * 32 + (lane & 31)][kk + 8 * (lane >> 5)]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, bf, acc, 0, 0, 0);
        }
        __syncthreads();
    }

    // D layout: register r of lane l holds row 8 (r/4) + 4 (l/32) + r%4, column l%32
    const int col = n0 + wn * 32 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t idx = (int64_t)row * g.n + col;
        float v = acc[r];
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
}

// out[c] = sum over rows of in[r][c]: 16 columns x 16 row groups per block,
// the group sums added in group order (deterministic)
__global__ __launch_bounds__(256) void colsum_kernel(int rows, int cols, const float* in, float* out) {
    __shared__ float sh[256];
    const int c = blockIdx.x * 16 + (threadIdx.x & 15);
    const int rg = threadIdx.x >> 4;
    float s = 0.f;
    if (c < cols)
        for (int r = rg; r < rows; r += 16) s += in[(int64_t)r * cols + c];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (rg == 0 && c < cols) {
        float tsum = 0.f;
        for (int i = 0; i < 16; ++i) tsum += sh[16 * i + (threadIdx.x & 15)];
        out[c] = tsum;
    }
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

template <int LAYOUT>
static hipError_t launch_gemm_layout(int epi, const GemmArgs& g, hipStream_t st) {
    dim3 grid(g.n / BN, g.m / BM), block(256);
    switch (epi) {
        case E_F32: hipLaunchKernelGGL((gemm_kernel<LAYOUT, E_F32>), grid, block, 0, st, g); break;
        case E_BIAS_F32: hipLaunchKernelGGL((gemm_kernel<LAYOUT, E_BIAS_F32>), grid, block, 0, st, g); break;
        case E_BIAS_GELU: hipLaunchKernelGGL((gemm_kernel<LAYOUT, E_BIAS_GELU>), grid, block, 0, st, g); break;
        case E_GELU_BWD: hipLaunchKernelGGL((gemm_kernel<LAYOUT, E_GELU_BWD>), grid, block, 0, st, g); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace graf_mlp

using namespace graf_mlp;

extern "C" {

af_status af_gemm_bf16(int32_t layout, int32_t epilogue, int32_t m, int32_t n, int32_t k, const void* a,
                       const void* b, const float* bias, const float* aux, float* out_f32, void* out_bf16,
                       void* stream) {
    if (layout < 0 || layout > 2 || epilogue < 0 || epilogue > 3) return AF_ERR_INVALID_ARG;
    if (m <= 0 || n <= 0 || k <= 0 || !a || !b || !out_f32) return AF_ERR_INVALID_ARG;
    if (m % BM || n % BN || k % BK) return AF_ERR_UNSUPPORTED;
    if (!aligned16(a) || !aligned16(b)) return AF_ERR_INVALID_ARG;
    if ((epilogue == E_BIAS_F32 || epilogue == E_BIAS_GELU) && !bias) return AF_ERR_INVALID_ARG;
    if ((epilogue == E_BIAS_GELU || epilogue == E_GELU_BWD) && !out_bf16) return AF_ERR_INVALID_ARG;
    if (epilogue == E_GELU_BWD && !aux) return AF_ERR_INVALID_ARG;
    GemmArgs g{m, n, k, (const __bf16*)a, (const __bf16*)b, bias, aux, out_f32, (__bf16*)out_bf16};
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = layout == L_NT ? launch_gemm_layout<L_NT>(epilogue, g, st)
                   : layout == L_NN ? launch_gemm_layout<L_NN>(epilogue, g, st)
                                    : launch_gemm_layout<L_TN>(epilogue, g, st);
    return e == hipSuccess ? AF_OK : AF_ERR_HIP;
}

af_status af_colsum(int32_t rows, int32_t cols, const float* in, float* out, void* stream) {
    if (rows <= 0 || cols <= 0 || !in || !out) return AF_ERR_INVALID_ARG;
    hipLaunchKernelGGL(colsum_kernel, dim3((cols + 15) / 16), dim3(256), 0, (hipStream_t)stream, rows, cols, in, out);
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
