// Device helpers shared by the forward and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hhffbp_internal.hpp"

namespace hh {
namespace dev {

// ---------------------------------------------------------------------------
// Storage of complex profiles and subimages: float32 pairs (C64), IEEE half
// pairs (F16) or bfloat16 pairs (BF16).  Arithmetic is always float32: values
// are widened on load and rounded to nearest even on store.  `C` is one
// complex value, `R` one real component (the range-compression GEMM sees the
// interleaved arrays as real matrices).
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f32_to_f16(float f)
{
    return __builtin_bit_cast(uint16_t, (_Float16)f);
}
__device__ __forceinline__ float f16_to_f32(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

template <int ST>
struct Store;
template <>
struct Store<HHFFBP_C64> {
    using C = float2;
    using R = float;
    static __device__ __forceinline__ float2 ld(C v) { return v; }
    static __device__ __forceinline__ C st(float2 v) { return v; }
    static __device__ __forceinline__ float ldr(R v) { return v; }
    static __device__ __forceinline__ R str(float v) { return v; }
};
template <>
struct Store<HHFFBP_F16> {
    using C = uint32_t;
    using R = uint16_t;
    static __device__ __forceinline__ float2 ld(C v)
    {
        return make_float2(f16_to_f32((uint16_t)(v & 0xffffu)), f16_to_f32((uint16_t)(v >> 16)));
    }
    static __device__ __forceinline__ C st(float2 v)
    {
        return (uint32_t)f32_to_f16(v.x) | ((uint32_t)f32_to_f16(v.y) << 16);
    }
    static __device__ __forceinline__ float ldr(R v) { return f16_to_f32(v); }
    static __device__ __forceinline__ R str(float v) { return f32_to_f16(v); }
};
template <>
struct Store<HHFFBP_BF16> {
    using C = uint32_t;
    using R = uint16_t;
    static __device__ __forceinline__ float2 ld(C v)
    {
        return make_float2(__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u));
    }
    static __device__ __forceinline__ C st(float2 v)
    {
        return (uint32_t)f32_to_bf16(v.x) | ((uint32_t)f32_to_bf16(v.y) << 16);
    }
    static __device__ __forceinline__ float ldr(R v) { return bf16_to_f32(v); }
    static __device__ __forceinline__ R str(float v) { return f32_to_bf16(v); }
};

constexpr int kBlock = kBlockThreads;
constexpr int kPosChunkMax = 16;
constexpr size_t kLdsBudget = 20 * 1024;  // dynamic LDS per block

// Positions staged per LDS chunk with their profiles.  Small chunks keep the
// LDS per block near 12 KB so that eight 256-lane blocks fit on a CU; the
// inner loop's dependency chain (sqrt, rcp, gather, sincos) needs that many
// waves to hide its latency.
inline int pos_chunk(int64_t Nr, size_t per_pos_header)
{
    const size_t per = per_pos_header + (size_t)Nr * sizeof(float2);
    int c = (int)(kLdsBudget / per);
    return c > kPosChunkMax ? kPosChunkMax : (c < 1 ? 1 : c);
}

// XCD-aware block order.  The dispatcher hands workgroup b to XCD b mod 8, each
// XCD with its own L2.  The logical order deals runs of RUN consecutive logical
// blocks to the XCDs in turn, so neighbouring logical blocks, which share inputs
// (a leaf's profiles, a parent node's children), meet in one L2.  RUN = 0 gives
// each XCD one contiguous share: the most sharing, for blocks of equal cost (a
// merge); a finite run keeps the XCDs balanced where block costs vary (leaves of
// different sizes: the contiguous form measured 30% slower there).  A bijection
// on [0, n); with a finite run the last partial round keeps the identity order.
// Only speed depends on the dispatch order.
constexpr int kXcds = 8;
template <int RUN>
__device__ __forceinline__ int xcd_block(int b, int n)
{
    const int x = b % kXcds, s = b / kXcds;
    if constexpr (RUN == 0) {
        const int per = n / kXcds, rem = n % kXcds;
        return x * per + min(x, rem) + s;
    } else {
        constexpr int round = kXcds * RUN;
        if (b >= n / round * round) return b;
        return ((s / RUN) * kXcds + x) * RUN + s % RUN;
    }
}

// xcd_block with a run length known only at launch (the same bijection).
__device__ __forceinline__ int xcd_block_run(int b, int n, int run)
{
    const int x = b % kXcds, s = b / kXcds, round = kXcds * run;
    if (b >= n / round * round) return b;
    return ((s / run) * kXcds + x) * run + s % run;
}

// base[i] through a 32-bit unsigned byte offset from a wave-uniform base, so the
// load can take the scalar base + 32-bit vector offset form instead of a 64-bit
// address per lane.  The caller keeps i * sizeof(T) below 2^32.
template <class T>
__device__ __forceinline__ T ld_u32(const T *__restrict__ base, uint32_t i)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + i * (uint32_t)sizeof(T));
}

// floor(x) as int32 in one VALU instruction (the compiler emits floor + convert)
__device__ __forceinline__ int floor_int(float x)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// Positions per staged chunk of the level-1 BP for a bin window of nrb bins:
// as many as kLdsBudget holds (a float4 and nrb float2 each), at most 32.
constexpr int kLeafChunkMax = 32;
// thread-strided steps per round of the final stage's box staging (a box of
// up to kTileCap values takes (kTileCap / kBlock) / kStageRound rounds)
constexpr int kStageRound = 2;
// thread-strided staging steps that cover a kLdsBudget tile of float2
constexpr int kStageSteps = (int)((kLdsBudget / sizeof(float2) + kBlock - 1) / kBlock);
__host__ __device__ inline int leaf_chunk(int nrb)
{
    const int c = (int)(kLdsBudget / (sizeof(float4) + (size_t)nrb * sizeof(float2)));
    return c > kLeafChunkMax ? kLeafChunkMax : (c < 1 ? 1 : c);
}

__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float exp2_f(float x) { return __builtin_amdgcn_exp2f(x); }
// v_sin_f32 / v_cos_f32 take their argument in turns; callers reduce it to [-0.5, 0.5].
__device__ __forceinline__ float sin_turns(float t) { return __builtin_amdgcn_sinf(t); }
__device__ __forceinline__ float cos_turns(float t) { return __builtin_amdgcn_cosf(t); }

// Weights of the W range taps r_first .. r_first+W-1 for fractional offset x in [0, 1)
// of tau = t - W/2 (t the continuous bin coordinate, r_first = floor(tau) + 1).
template <int KERNEL, int W>
__device__ __forceinline__ void range_weights(float x, float beta_log2e, float *w)
{
    if constexpr (KERNEL == HHFFBP_RANGE_LINEAR) {
        w[0] = 1.0f - x;
        w[1] = x;
    } else {
        constexpr float s = 2.0f / W;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            // z = (k + 1 - W/2 - x) (2/W) in [-1, 1];  w = exp(beta (sqrt(1 - z^2) - 1))
            const float z = fmaf(-s, x, ((float)k + 1.0f - 0.5f * W) * s);
            const float a = fmaxf(fmaf(-z, z, 1.0f), 0.0f);
            w[k] = exp2_f(fmaf(beta_log2e, fast_sqrt(a), -beta_log2e));
        }
    }
}

// ---------------------------------------------------------------------------
// A stencil in a child's lattice: base indices floor(t) of the continuous
// lattice coordinate t = gamma (u, v, n) (Sec. III, eq. uvw_xyz) and the
// fractions t - floor(t).
struct ChildCoord {
    int bi, bj, bl;
    float fu, fv, fn;
};

// Lagrange weights on nodes -T/2+1 .. T/2 at x in [0, 1).
template <int T>
__device__ __forceinline__ void lagrange(float x, float *w)
{
#pragma unroll
    for (int a = 0; a < T; ++a) {
        float num = 1.0f, den = 1.0f;
        const float na = (float)(a - T / 2 + 1);
#pragma unroll
        for (int m = 0; m < T; ++m) {
            if (m == a) continue;
            const float nm = (float)(m - T / 2 + 1);
            num *= (x - nm);
            den *= (na - nm);
        }
        w[a] = num * (1.0f / den);  // den is a compile-time integer: a multiply
    }
}

// Weights of the three axes at a child coordinate: Lagrange (K = LAGRANGE),
// or the plan's band-limited polynomials in y = x - 1/2.  The stencil is
// symmetric (tap t at offset x is tap T-1-t at 1 - x, i.e. at -y), so with
// w_t = E_t(y^2) + y O_t(y^2), split into even and odd parts, the mirror tap
// is E_t - y O_t: one pair of short Horner chains for two taps.
template <int T, int A>
__device__ __forceinline__ void poly_weights(const InterpPoly &ip, float x, float *w)
{
    const float y = x - 0.5f, y2 = y * y;
#pragma unroll
    for (int t = 0; t < T / 2; ++t) {
        float e = ip.c[A][t][kPolyDeg - 1], o = ip.c[A][t][kPolyDeg];
#pragma unroll
        for (int d = kPolyDeg - 3; d >= 0; d -= 2) {
            e = fmaf(e, y2, ip.c[A][t][d]);
            o = fmaf(o, y2, ip.c[A][t][d + 1]);
        }
        w[t] = fmaf(y, o, e);
        w[T - 1 - t] = fmaf(-y, o, e);
    }
}

template <int T, int K>
__device__ __forceinline__ void interp_weights3(const InterpPoly &ip, float fu, float fv, float fn,
                                                float *wu, float *wv, float *wn)
{
    if constexpr (K == HHFFBP_INTERP_BANDLIMITED) {
        poly_weights<T, 0>(ip, fu, wu);
        poly_weights<T, 1>(ip, fv, wv);
        poly_weights<T, 2>(ip, fn, wn);
    } else {
        lagrange<T>(fu, wu);
        lagrange<T>(fv, wv);
        lagrange<T>(fn, wn);
    }
}

template <int T, int K>
__device__ __forceinline__ void interp_weights(const InterpPoly &ip, const ChildCoord &g, float *wu,
                                               float *wv, float *wn)
{
    interp_weights3<T, K>(ip, g.fu, g.fv, g.fn, wu, wv, wn);
}

// Separable T^3 interpolation at a plan-time record (InterpIdx): the stencil's
// first column (ci0, cj0) of the child's lattice and first n index l0.  Every
// tap lies inside the child's pencils (checked when the records were built),
// so each of the T^2 columns gives T contiguous values from its base
// colbase[col] = off - lo alone (4 bytes a column instead of a column entry).
template <int T, int ST>
__device__ __forceinline__ float2 interp_rec(const NodeDev &c, const int32_t *__restrict__ colbase,
                                             const typename Store<ST>::C *__restrict__ vals, int ci0,
                                             int cj0, int l0, const float *wu, const float *wv,
                                             const float *wn)
{
    const int32_t *crow = colbase + c.col_base + ci0 * c.nj + cj0;
    const typename Store<ST>::C *base = vals + (c.val_base + l0);
    float are = 0.0f, aim = 0.0f;
#pragma unroll
    for (int a = 0; a < T; ++a) {
        float rre = 0.0f, rim = 0.0f;  // stencil row a: sum over b of wv[b] x column sum
#pragma unroll
        for (int b = 0; b < T; ++b) {
            const typename Store<ST>::C *p = base + crow[a * c.nj + b];
            float sre = 0.0f, sim = 0.0f;
#pragma unroll
            for (int k = 0; k < T; ++k) {
                const float2 v = Store<ST>::ld(p[k]);
                sre = fmaf(wn[k], v.x, sre);
                sim = fmaf(wn[k], v.y, sim);
            }
            rre = fmaf(wv[b], sre, rre);
            rim = fmaf(wv[b], sim, rim);
        }
        are = fmaf(wu[a], rre, are);
        aim = fmaf(wu[a], rim, aim);
        // one stencil row (T columns, T^2 values) in flight at a time: hoisting
        // every gather costs registers and occupancy, not latency
        __builtin_amdgcn_sched_barrier(0);
    }
    return make_float2(are, aim);
}

// acc += v exp(j 2 pi turns), turns in [-1/2, 1/2]
__device__ __forceinline__ void rotate_mac(float2 v, float turns, float &are, float &aim)
{
    const float sn = sin_turns(turns), cs = cos_turns(turns);
    are = fmaf(v.x, cs, fmaf(-v.y, sn, are));
    aim = fmaf(v.x, sn, fmaf(v.y, cs, aim));
}

// The T^3 taps from a dense LDS box: p points at the stencil's first tap, the
// box's (i, j) columns lie cs values apart (CS when CS > 0, a compile-time
// stride), nj columns per i.  Same summation order as interp_rec.
template <int T, int CS>
__device__ __forceinline__ float2 interp_box(const float2 *p, int nj, const float *wu, const float *wv,
                                             const float *wn, int cs = CS)
{
    const int stride = CS > 0 ? CS : cs;
    float are = 0.0f, aim = 0.0f;
#pragma unroll
    for (int a = 0; a < T; ++a) {
        const float2 *row = p + a * nj * stride;
        float rre = 0.0f, rim = 0.0f;
#pragma unroll
        for (int b = 0; b < T; ++b) {
            const float2 *q = row + b * stride;
            float sre = 0.0f, sim = 0.0f;
#pragma unroll
            for (int k = 0; k < T; ++k) {
                const float2 v = q[k];
                sre = fmaf(wn[k], v.x, sre);
                sim = fmaf(wn[k], v.y, sim);
            }
            rre = fmaf(wv[b], sre, rre);
            rim = fmaf(wv[b], sim, rim);
        }
        are = fmaf(wu[a], rre, are);
        aim = fmaf(wu[a], rim, aim);
    }
    return make_float2(are, aim);
}


}  // namespace dev
}  // namespace hh
