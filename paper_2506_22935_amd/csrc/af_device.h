// Device building blocks for the ambiguity-function kernels (gfx950).
//
// * complex64 arithmetic on float2 (re, im)
// * compile-time twiddle constants (constexpr Taylor series, double precision)
// * register DFTs of size 2..32, decimation in time, either sign
// * one Stockham autosort pass over a lane group whose lanes each hold P
//   points, exchanging through LDS with one padding slot per 32 entries
//
// Sign convention: SIGN = -1 is the forward transform sum x[n] e^{-j2pi kn/R}
// (the "FFT" of Algorithm 1, step 3), SIGN = +1 the unnormalised inverse.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace graf {

// ---------------------------------------------------------------- complex --
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float cabs2(float2 a) { return fmaf(a.x, a.x, a.y * a.y); }

// ------------------------------------------------------ buffer access --
// A buffer resource: base address and byte range in scalar registers, a
// 32-bit per-lane byte offset per access.  Loads beyond the range return zero
// and stores beyond it are dropped (the hardware checks the per-lane offset),
// so global rows and sample arrays need neither 64-bit lane addresses nor
// bounds predicates.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit access, no swizzle
__device__ __forceinline__ Rsrc make_rsrc(const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRsrcWord3);
}
__device__ __forceinline__ float2 buf_load2(Rsrc r, int byte_off) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
}
__device__ __forceinline__ void buf_store2(Rsrc r, int byte_off, float2 v) {
    using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, byte_off, 0, 0);
}
__device__ __forceinline__ float buf_load1(Rsrc r, int byte_off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}
__device__ __forceinline__ void buf_store1(Rsrc r, int byte_off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, byte_off, 0, 0);
}

// ------------------------------------------------ wavefront reductions --
// Lane exchange through DPP: quad permutations and row rotations act inside
// rows of 16 lanes; the four row sums are then read out lane by lane.  The
// additions run in a fixed order, and every lane receives the same total.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
constexpr int kDppQuadXor1 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4E;  // quad_perm [2, 3, 0, 1]
constexpr int kDppRowRor4 = 0x124;
constexpr int kDppRowRor8 = 0x128;

__device__ __forceinline__ float wave_allsum(float v) {
    v += dpp_f<kDppQuadXor1>(v);
    v += dpp_f<kDppQuadXor2>(v);
    v += dpp_f<kDppRowRor4>(v);
    v += dpp_f<kDppRowRor8>(v);
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (r0 + r1) + (r2 + r3);
}
__device__ __forceinline__ double wave_allsum(double v) {
    v += dpp_d<kDppQuadXor1>(v);
    v += dpp_d<kDppQuadXor2>(v);
    v += dpp_d<kDppRowRor4>(v);
    v += dpp_d<kDppRowRor8>(v);
    auto lane = [&](int src) {
        return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), src),
                                __builtin_amdgcn_readlane(__double2loint(v), src));
    };
    return (lane(0) + lane(16)) + (lane(32) + lane(48));
}

__device__ __forceinline__ float wave_allmax(float v) {
    v = fmaxf(v, dpp_f<kDppQuadXor1>(v));
    v = fmaxf(v, dpp_f<kDppQuadXor2>(v));
    v = fmaxf(v, dpp_f<kDppRowRor4>(v));
    v = fmaxf(v, dpp_f<kDppRowRor8>(v));
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return fmaxf(fmaxf(r0, r1), fmaxf(r2, r3));
}

// Smallest int over a wavefront (butterfly exchange; every lane gets it).
__device__ __forceinline__ int wave_allmin_int(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

// Log-sum-exp pairs (m, s) = (max, sum of exp2((x - m) k)) over a wavefront:
// the common maximum first, then one rescale per lane and a plain sum.
__device__ __forceinline__ void wave_lse_pair(float& m, double& s, float k) {
    const float mw = wave_allmax(m);
    s = (m == -INFINITY) ? 0.0 : s * (double)exp2f((m - mw) * k);
    s = wave_allsum(s);
    m = mw;
}

// ------------------------------------------------- compile-time twiddles --
// cos / sin of 2*pi*k/R in double precision, reduced to the first octant and
// evaluated with a Taylor series (error far below float rounding).
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
    double term = x, sum = x;
    for (int i = 1; i < 14; ++i) {
        term *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double taylor_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int i = 1; i < 14; ++i) {
        term *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
        sum += term;
    }
    return sum;
}
// cos(2 pi k / R) for integer k, R > 0
constexpr double ccos(long k, long R) {
    k = ((k % R) + R) % R;
    // use the quadrant symmetry to keep the Taylor argument within [0, pi/4]
    long k8 = 8 * k;  // angle in units of 2pi/(8R): octant = k8 / R
    if (k8 <= R) return taylor_cos(2.0 * kPi * k / R);
    if (k8 <= 2 * R) return taylor_sin(2.0 * kPi * (R - 4 * k) / (4.0 * R));
    if (k8 <= 3 * R) return -taylor_sin(2.0 * kPi * (4 * k - R) / (4.0 * R));
    if (k8 <= 4 * R) return -taylor_cos(2.0 * kPi * (R - 2 * k) / (2.0 * R));
    return ccos(R - k, R);
}
constexpr double csin(long k, long R) { return ccos(R - 4 * k, 4 * R); }

// v * exp(SIGN * j 2 pi K / R) for a compile-time K, with the trivial
// multiples of pi/4 spelled out so they cost no multiplications.
template <int K, int R, int SIGN>
__device__ __forceinline__ float2 twiddle_const(float2 v) {
    constexpr int k = ((K % R) + R) % R;
    constexpr int e8 = (8 * k) % R == 0 ? (8 * k) / R : -1;  // multiple of pi/4?
    if constexpr (e8 == 0) {
        return v;
    } else if constexpr (e8 == 2) {  // e^{SIGN j pi/2} = SIGN j
        return SIGN < 0 ? make_float2(v.y, -v.x) : make_float2(-v.y, v.x);
    } else if constexpr (e8 == 4) {
        return make_float2(-v.x, -v.y);
    } else if constexpr (e8 == 6) {  // e^{SIGN j 3pi/2} = -SIGN j
        return SIGN < 0 ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
    } else if constexpr (e8 == 1 || e8 == 3 || e8 == 5 || e8 == 7) {
        constexpr float h = 0.70710678118654752440f;
        // (x + jy)(c + jSs) with |c| = |s| = 1/sqrt2
        constexpr float c = (e8 == 1 || e8 == 7) ? h : -h;
        constexpr float s = (e8 == 1 || e8 == 3) ? h : -h;
        constexpr float ss = SIGN < 0 ? -s : s;
        if constexpr (c == ss) {
            return make_float2((v.x - v.y) * c, (v.x + v.y) * c);
        } else {
            return make_float2((v.x + v.y) * c, (v.y - v.x) * c);
        }
    } else {
        constexpr float c = (float)ccos(k, R);
        constexpr float s = (float)(SIGN < 0 ? -csin(k, R) : csin(k, R));
        return make_float2(fmaf(v.x, c, -v.y * s), fmaf(v.x, s, v.y * c));
    }
}

// v[K] *= exp(SIGN j 2 pi K / R) for every slot K < P (compile-time constants)
template <int R, int SIGN, int P, int K = 0>
__device__ __forceinline__ void twist_const(float2* v) {
    if constexpr (K < P) {
        v[K] = twiddle_const<K, R, SIGN>(v[K]);
        twist_const<R, SIGN, P, K + 1>(v);
    }
}

// -------------------------------------------------------- register DFTs --
// In-place DFT of R values held in registers, natural order in and out.
template <int R, int SIGN>
struct Dft {
    template <int K>
    __device__ __forceinline__ static void combine(float2* e, float2* o, float2* v) {
        if constexpr (K < R / 2) {
            float2 t = twiddle_const<K, R, SIGN>(o[K]);
            v[K] = cadd(e[K], t);
            v[K + R / 2] = csub(e[K], t);
            combine<K + 1>(e, o, v);
        }
    }
    __device__ __forceinline__ static void run(float2* v) {
        float2 e[R / 2], o[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            e[i] = v[2 * i];
            o[i] = v[2 * i + 1];
        }
        Dft<R / 2, SIGN>::run(e);
        Dft<R / 2, SIGN>::run(o);
        combine<0>(e, o, v);
    }
};
template <int SIGN>
struct Dft<1, SIGN> {
    __device__ __forceinline__ static void run(float2*) {}
};
template <int SIGN>
struct Dft<2, SIGN> {
    __device__ __forceinline__ static void run(float2* v) {
        float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};
template <int SIGN>
struct Dft<4, SIGN> {
    __device__ __forceinline__ static void run(float2* v) {
        float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        float2 t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
        // t3 * (SIGN j)
        float2 u = SIGN < 0 ? make_float2(t3.y, -t3.x) : make_float2(-t3.y, t3.x);
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, u);
        v[3] = csub(t1, u);
    }
};

// ----------------------------------------------------------- LDS layout --
// One padding slot per 32 complex entries spreads stride-R stores over banks.
__device__ __forceinline__ int lds_index(int i) { return i + (i >> 5); }
// lds_index(b + c) = lds_index(b) + lds_index(c) whenever (b mod 32) +
// (c mod 32) < 32: accesses at compile-time offsets c from one per-lane base
// then need one address register and immediate offsets.
constexpr int lds_off(int c) { return c + (c >> 5); }
template <int N>
struct LdsSize {
    static constexpr int value = N + (N >> 5);
};

// --------------------------------------------------------- Stockham FFT --
// Lane group of L lanes, P points per lane, transform size MH = L * P.
// Register layout at entry: v[r] = x[l + r*L]  (l = lane in the group).
// Register layout at exit:  v[q] = X[l + q*L].
// Passes use radix P except the last, whose radix RL divides P; each lane
// runs P/R butterflies per pass.  Twiddles exp(SIGN j 2pi i / MMAX) come from
// tw[i] (i < MMAX), the table of the largest transform in the launch.
template <int MH, int P>
struct Plan {
    static constexpr int L = MH / P;
    static constexpr int log2(int x) { return x <= 1 ? 0 : 1 + log2(x / 2); }
    static constexpr int LOG_MH = log2(MH);
    static constexpr int LOG_P = log2(P);
    static constexpr int NPASS = (LOG_MH + LOG_P - 1) / LOG_P;
    static constexpr int RLAST = 1 << (LOG_MH - (NPASS - 1) * LOG_P);
};

// ------------------------------------------------------- twiddle tables --
// w_M^i = exp(-j 2 pi i / M) for 0 <= i < M of the transform's M = 2 MH.
// TwTable reads one table (index scaled by sh when the table serves a larger
// transform); TwSplit multiplies two short tables, hi[i >> b] * lo[i mod 2^b],
// which fit in LDS beside the transform buffers of large sizes.
// Twiddle accessors.  kPassTables: per-pass tables (TwPass); kPass1: a
// table of the first twiddled pass of 16-point passes, w_256^(r k) for r in
// [1, 16), k in [0, 16) laid out [r - 1][k] (the first twiddled pass of any
// transform of 256 points or more with P = 16 needs exactly these); kPass2:
// likewise w_4096^(r k), k < 256, for the pass of stride 256, which serves
// every transform size of that pass (radix R: w_{256 R}^(r k) =
// w_4096^((16 / R) r k)).
constexpr int kPass1Entries = 15 * 16;
constexpr int kPass2Entries = 15 * 256;
struct TwTable {
    static constexpr bool kPassTables = false;
    static constexpr bool kPass1 = false;
    static constexpr bool kPass2 = false;
    const float2* t;
    int sh;
    __device__ __forceinline__ float2 operator()(int i) const { return t[i << sh]; }
    // w_M^i for i < M/2
    __device__ __forceinline__ float2 low(int i) const { return t[i << sh]; }
};
struct TwSplit {
    static constexpr bool kPassTables = false;
    static constexpr bool kPass1 = true;
    static constexpr bool kPass2 = false;
    const float2* hi;
    const float2* lo;
    int b;
    const float2* p1;
    __device__ __forceinline__ float2 operator()(int i) const { return cmul(hi[i >> b], lo[i & ((1 << b) - 1)]); }
    __device__ __forceinline__ float2 low(int i) const { return (*this)(i); }
};

// Per-pass twiddle tables of one transform size (MH points, P per lane).
// Pass p >= 1 of the Stockham transform (stride NS = P^p, radix R) needs
// w_M^(r k M / (NS R)) for r in [1, R) and k in [0, NS); its table holds them
// as [r - 1][k].  The lanes of a wavefront have consecutive (or repeating) k,
// so they read consecutive entries: no LDS bank conflicts, where reading one
// shared table at index r k M / (NS R) put up to 16 lanes on one bank.
template <int MH, int P>
struct PassTables {
    static constexpr int radix(int ns) { return ns * P >= MH ? MH / ns : P; }
    // first entry of the table of the pass with stride ns (ns = P, P^2, ...)
    static constexpr int offset(int ns) {
        int o = 0;
        for (int q = P; q < ns; q *= P) o += (radix(q) - 1) * q;
        return o;
    }
    static constexpr int total() { return offset(MH); }
};
// Index into the w_M table (M = 2 MH) of entry e of the pass tables.
template <int MH, int P, int NS = P>
__device__ __forceinline__ int pass_table_source(int e) {
    if constexpr (NS >= MH) {
        return 0;
    } else {
        constexpr int R = PassTables<MH, P>::radix(NS);
        constexpr int SZ = (R - 1) * NS;
        if (e < SZ) {
            const int r = e / NS + 1, k = e % NS;
            return (r * k * (2 * MH / (NS * R))) & (2 * MH - 1);
        }
        return pass_table_source<MH, P, NS * P>(e - SZ);
    }
}
// Half table w_M^i (i < M/2) followed by the pass tables; w_M^i for
// i in [M/2, M) is -w_M^(i - M/2).
struct TwPass {
    static constexpr bool kPassTables = true;
    static constexpr bool kPass1 = false;
    static constexpr bool kPass2 = false;
    const float2* half;
    const float2* pass;
    int mh;
    __device__ __forceinline__ float2 operator()(int i) const {
        const float2 w = half[i & (mh - 1)];
        return i < mh ? w : make_float2(-w.x, -w.y);
    }
    __device__ __forceinline__ float2 low(int i) const { return half[i]; }
};
// The short tables of the largest transform in a launch serving a smaller
// one: w_M^i = w_MMAX^(i << sh) with sh = log2(MMAX / M).
template <bool P2>
struct TwSplitSh {
    static constexpr bool kPassTables = false;
    static constexpr bool kPass1 = true;
    static constexpr bool kPass2 = P2;
    const float2* hi;
    const float2* lo;
    int b;
    int sh;
    const float2* p1;
    const float2* p2;  // staged whenever some transform has a pass of stride 256
    __device__ __forceinline__ float2 operator()(int i) const {
        const int j = i << sh;
        return cmul(hi[j >> b], lo[j & ((1 << b) - 1)]);
    }
    __device__ __forceinline__ float2 low(int i) const { return (*this)(i); }
};

// Pass number PASS (0-based) with stride NS = P^PASS and radix R.
// in: v laid out as slots [b*R + r] = x[j + r*MH/R], j = l + L*b
// out: written to LDS y[(j/NS)*NS*R + j%NS + r*NS] unless LAST, in which
//      case the values stay in registers: slot [b*R + r] = X[j + r*MH/R].
template <int MH, int P, int R, int NS, int SIGN, bool LAST, bool LEAN, typename Tw>
__device__ __forceinline__ void stockham_pass(float2* v, float2* lds, int l, const Tw& tw, int tw_shift) {
    constexpr int L = MH / P;
    constexpr int NB = P / R;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = l + L * b;
        const int k = j & (NS - 1);
        float2* u = v + b * R;
        if constexpr (NS > 1) {
            // exp(SIGN j 2pi r k / (NS R)) = w_M^(r k M/(NS R))
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w;
                if constexpr (Tw::kPassTables)
                    w = tw.pass[PassTables<MH, P>::offset(NS) + (r - 1) * NS + k];
                else if constexpr (Tw::kPass1 && P == 16 && NS == 16 && R == 16)
                    w = tw.p1[(r - 1) * 16 + k];  // w_M^(r k M / 256) = w_256^(r k)
                else if constexpr (Tw::kPass2 && P == 16 && NS == 256)
                    w = tw.p2[(r * (16 / R) - 1) * 256 + k];
                else
                    w = tw((r * k) << tw_shift);
                if (SIGN > 0) w.y = -w.y;
                u[r] = cmul(u[r], w);
                // register-lean instances: a few twiddles in flight at a time
                if (LEAN && (r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
            }
        }
        Dft<R, SIGN>::run(u);
        if constexpr (!LAST) {
            // base mod 32 + (r NS) mod 32 < 32 holds when NS = 1 (base is a
            // multiple of R), when NS R >= 32 (base mod 32 = k < NS and r NS
            // mod 32 <= 32 - NS) and when NS >= 32
            static_assert(NS == 1 || NS * R >= 32, "write offsets would carry");
            const int bi = lds_index((j / NS) * NS * R + k);
#pragma unroll
            for (int r = 0; r < R; ++r) lds[bi + lds_off(r * NS)] = u[r];
        }
    }
}

// Gather the next pass's inputs: slot [b*R + r] = y[l + L*b + r*MH/R].
template <int MH, int P, int R>
__device__ __forceinline__ void read_group(float2* v, const float2* lds, int l) {
    constexpr int L = MH / P;
#pragma unroll
    for (int b = 0; b < P / R; ++b) {
        if constexpr ((MH / R) % 32 == 0) {
            const int bi = lds_index(l + L * b);
#pragma unroll
            for (int r = 0; r < R; ++r) v[b * R + r] = lds[bi + lds_off(r * (MH / R))];
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) v[b * R + r] = lds[lds_index(l + L * b + r * (MH / R))];
        }
    }
}

// Full transform of one lane group.  Synchronisation between passes goes
// through SYNC(), which must make every lane's LDS stores visible to every
// lane of the group (a work-group barrier or a wavefront-level fence).
// tw gives w_M^i for the transform's M = 2 MH.  LEAN bounds the twiddle loads
// in flight (instances with few registers per lane).
template <int MH, int P, int SIGN, bool LEAN = false, typename Tw, typename Sync>
__device__ __forceinline__ void fft_group(float2* v, float2* lds, int l, const Tw& tw, Sync sync) {
    using PL = Plan<MH, P>;
    constexpr int L = PL::L;
    constexpr int NPASS = PL::NPASS;
    constexpr int RL = PL::RLAST;
    // tw index for pass with NS, R: (r k) * (M / (NS R)), M / (NS R) =
    // 2 MH / (NS R), a power of two -> shift
    constexpr int sh0 = 1;
    static_assert(NPASS >= 1 && NPASS <= 4, "transform size out of range");
    if constexpr (NPASS == 1) {
        stockham_pass<MH, P, RL, 1, SIGN, true, LEAN>(v, lds, l, tw, 0);
    } else {
        stockham_pass<MH, P, P, 1, SIGN, false, LEAN>(v, lds, l, tw, 0);
        sync();
        constexpr int NS1 = P;
        constexpr int R1 = NPASS == 2 ? RL : P;
        read_group<MH, P, R1>(v, lds, l);
        sync();
        stockham_pass<MH, P, R1, NS1, SIGN, NPASS == 2, LEAN>(v, lds, l, tw, sh0 + PL::LOG_MH - PL::log2(NS1 * R1));
        if constexpr (NPASS >= 3) {
            sync();
            constexpr int NS2 = P * P;
            constexpr int R2 = NPASS == 3 ? RL : P;
        read_group<MH, P, R2>(v, lds, l);
            sync();
            stockham_pass<MH, P, R2, NS2, SIGN, NPASS == 3, LEAN>(v, lds, l, tw, sh0 + PL::LOG_MH - PL::log2(NS2 * R2));
            if constexpr (NPASS >= 4) {
                sync();
                constexpr int NS3 = P * P * P;
                constexpr int R3 = RL;
                read_group<MH, P, R3>(v, lds, l);
                sync();
                stockham_pass<MH, P, R3, NS3, SIGN, true, LEAN>(v, lds, l, tw, sh0 + PL::LOG_MH - PL::log2(NS3 * R3));
            }
        }
    }
    // exit layout: slot [b*RL + r] = X[l + L*b + r*MH/RL] = X[l + L*(b + r*P/RL)]
    // reorder to slot q = b + r*(P/RL) so that v[q] = X[l + q*L]
    if constexpr (RL != P) {
        float2 t[P];
#pragma unroll
        for (int b = 0; b < P / RL; ++b)
#pragma unroll
            for (int r = 0; r < RL; ++r) t[b + r * (P / RL)] = v[b * RL + r];
#pragma unroll
        for (int q = 0; q < P; ++q) v[q] = t[q];
    }
}

}  // namespace graf
