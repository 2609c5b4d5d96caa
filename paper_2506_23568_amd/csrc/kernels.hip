// gfx950 kernels of the HHFFBPA hot path and their launcher.
//
//   k_prep_positions  antenna offsets from their leaf centre (float64 -> float32)
//   k_absmax, k_scales  per-call power-of-two scales for half-precision storage
//   k_rc_gemm         range compression, eq. (2): profiles = echoes x W on float32 MFMA
//   k_rc_gemm_x6_br   the same for complex64 echoes as exact bfloat16 splits on bf16
//                     MFMA (float32 accuracy), each block's B fragments resident in
//                     LDS and A loaded to registers (two or more row tiles a wave);
//                     k_rc_gemm_x6_dma with operands through LDS by direct loads,
//                     k_rc_gemm_x6 with operands loaded to registers
//   k_leaf_bp         level-1 BP onto each leaf grid + SDC (Sec. IV-A, eq. sdc_mul)
//   k_merge           interpolate compressed children onto a parent grid, undo
//                     their SDC, sum, compress with the parent's Phi (Sec. IV-A)
//   k_final           the same onto the user voxels, without a parent SDC
//   k_direct_bp       direct BP of eq. (3) on range profiles (mode DIRECT_RC / S = 0)
//
// Precision plan.  Large distances (~0.3 m) never enter float32 phases directly:
// leaf BP works with distance differences to the leaf centre, direct BP with
// differences to a per-tile reference point whose own distance is float64, and
// the merge geometry ((u, v, n) and Phi of each child at each point) is formed
// once per plan in float64 on the host: the merges and the final stage read
// per-pair records of stencil, fractions and a phase already reduced to turns.
// Echoes, profiles and subimages may be stored as half or bfloat16 pairs
// (template parameter ST); every sum is float32.  With IEEE half each stage's
// array carries a power-of-two scale, scales[0] for the profiles and scales[d]
// for depth d (scales[S + 1] for a root grid), chosen per call from the largest echo component and the plan's
// worst-case gain of each stage, so that no stored value can exceed 2^15.
#include <algorithm>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "device_common.hpp"
#include "hhffbp_internal.hpp"

// Workspace of hhffbp_image_noalloc: one array per device, held from the
// module's load until the process ends, shared by every such call on that
// device.  In host code `scratch` names a host-side stand-in; the device
// address comes from hipGetSymbolAddress (noalloc_workspace below).
static __device__ __align__(256) unsigned char scratch[HHFFBP_NOALLOC_WORKSPACE_BYTES];

namespace hh {
namespace {
using namespace dev;

// ---------------------------------------------------------------------------
// Position pass: each antenna's offset from its leaf centre (float64 ->
// float32) and its squared norm, in leaf-sorted order.  The plan's range
// windows and its choice of carrier form hold for positions within `slack` of
// the planned ones along each axis; a coordinate beyond that is clamped to the
// slack box, so that every later kernel stays inside its windows (the image is
// then that of the clamped positions: hhffbp_check_positions reports such
// positions).
__global__ __launch_bounds__(kBlock) void k_prep_positions(const double *__restrict__ pos64,
                                                           const double *__restrict__ plan64,
                                                           double slack,
                                                           const int32_t *__restrict__ perm,
                                                           const int32_t *__restrict__ leaf_of,
                                                           const double *__restrict__ centre,
                                                           int n, float4 *__restrict__ out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int m = perm[i], lf = leaf_of[i];
    double p[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double q = plan64[3 * m + a];
        p[a] = fmin(fmax(pos64[3 * m + a], q - slack), q + slack);
    }
    const double dx = p[0] - centre[2 * lf];
    const double dy = p[1] - centre[2 * lf + 1];
    const double dz = p[2];
    const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
    out[i] = make_float4(fx, fy, fz, fx * fx + fy * fy + fz * fz);
}

// Positions with a coordinate outside [q - slack, q + slack] around the planned
// one q (the box k_prep_positions clamps to), or not finite: the count of each
// block of kBlock positions into counts[block].
__global__ __launch_bounds__(kBlock) void k_check_positions(const double *__restrict__ pos64,
                                                            const double *__restrict__ plan64,
                                                            double slack, int n,
                                                            int32_t *__restrict__ counts)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    bool out = false;
    if (i < n) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double p = pos64[3 * i + a], q = plan64[3 * i + a];
            out = out || !(p >= q - slack && p <= q + slack);
        }
    }
    const int c = __syncthreads_count(out);
    if (threadIdx.x == 0) counts[blockIdx.x] = c;
}

// ---------------------------------------------------------------------------
// Scales for half storage.  k_absmax: the largest |component| of the echoes,
// one partial maximum per block (plain stores: no contended atomics).
// k_scales folds the partials and sets scale_k = 2^-ceil(log2(m mult_k / 2^15)),
// mult_k the worst-case gain from the echoes to stage k; without a mult (other
// storage types) every scale is 1.
template <int ST>
__global__ __launch_bounds__(kBlock) void k_absmax(const typename Store<ST>::R *__restrict__ a,
                                                   int64_t n, int64_t n16, float *__restrict__ part)
{
    // the first n16 * 16 bytes as 16-byte loads (the caller checks alignment), the rest singly
    constexpr int per = 16 / (int)sizeof(typename Store<ST>::R);
    __shared__ float s_m[kBlock / 64];
    float m = 0.0f;
    const int64_t g0 = (int64_t)blockIdx.x * kBlock + threadIdx.x, gs = (int64_t)gridDim.x * kBlock;
    for (int64_t i = g0; i < n16; i += gs) {
        const uint4 u = reinterpret_cast<const uint4 *>(a)[i];
        const uint32_t w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if constexpr (per == 4) {
                m = fmaxf(m, fabsf(__uint_as_float(w4[e])));
            } else {
                m = fmaxf(m, fabsf(Store<ST>::ldr((uint16_t)(w4[e] & 0xffffu))));
                m = fmaxf(m, fabsf(Store<ST>::ldr((uint16_t)(w4[e] >> 16))));
            }
        }
    }
    for (int64_t i = n16 * per + g0; i < n; i += gs)
        m = fmaxf(m, fabsf(Store<ST>::ldr(a[i])));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 1; w < kBlock / 64; ++w) m = fmaxf(m, s_m[w]);
        part[blockIdx.x] = m;
    }
}

__global__ __launch_bounds__(64) void k_scales(const float *__restrict__ part, int nparts,
                                               const float *__restrict__ mult, int n,
                                               float *__restrict__ scales)
{
    const int k = threadIdx.x;
    float m = 0.0f;
    for (int i = k; i < nparts; i += 64) m = fmaxf(m, part[i]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if (k >= n) return;
    float s = 1.0f;
    if (mult) {
        const float b = m * mult[k];
        if (b > 0.0f && isfinite(b)) {
            int e = (int)ceilf(log2f(b)) - 15;
            e = max(-100, min(100, e));
            s = ldexpf(1.0f, -e);
        }
    }
    scales[k] = s;
}

// ---------------------------------------------------------------------------
// Range compression as a real GEMM, C[M x N] = scale A[perm(M) x K] B[K x N], with
// A the echoes as interleaved reals (K = 2 Nf), B the block form of the
// pre-corrected DFT matrix (float32, N = 2 Nr) and C the profiles (interleaved).
// Inputs are widened to float32 in LDS, A stored k-major so that the MFMA
// operand reads (16 consecutive rows per k) are conflict-free; block tile
// 64 x 64, four waves of 32 x 32, each 2 x 2 v_mfma_f32_16x16x4f32.  With
// float32 echoes, K % 8 == 0 and 16-byte aligned rows (vec) a thread stages its
// 8 reals of A and of B with two 16-byte loads each.
constexpr int kGemmKC = 32;
constexpr int kGemmPad = 16;  // row stride 80 floats: the four k groups of an MFMA operand read hit distinct banks
typedef float v4f __attribute__((ext_vector_type(4)));

template <int SA, int SC>
__global__ __launch_bounds__(kBlock) void k_rc_gemm(const typename Store<SA>::R *__restrict__ A,
                                                    const int32_t *__restrict__ perm, int M,
                                                    int K, const float *__restrict__ B, int N,
                                                    typename Store<SC>::R *__restrict__ C,
                                                    const int32_t *__restrict__ c_perm,
                                                    const float *__restrict__ scale, int vec,
                                                    const float *__restrict__ a_w,
                                                    const float *__restrict__ c_w)
{
    __shared__ __align__(16) float As[kGemmKC][64 + kGemmPad];  // [k][row]
    __shared__ __align__(16) float Bs[kGemmKC][64 + kGemmPad];  // [k][col]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // a 1-D grid: the column tiles of one row tile are consecutive logical
    // blocks dealt to one XCD, so its rows of A come from HBM once and from
    // that XCD's L2 for the other column tiles
    const int ncb = (N + 63) / 64;
    const int lb = xcd_block_run((int)blockIdx.x, (int)gridDim.x, ncb);
    const int row0 = (lb / ncb) * 64, col0 = (lb % ncb) * 64;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    v4f acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    // this thread's A row and k offset, B k row and column offset within a tile
    const int ar = tid >> 2, ak = (tid & 3) * 8;
    const int grow = row0 + ar;
    const bool arow_ok = grow < M;
    const int arow = arow_ok ? (perm ? perm[grow] : grow) : 0;
    const float aw = a_w ? a_w[arow] : 1.0f;  // row weight of A (aperture weight of the echo row)
    const int bk = tid >> 3, bc = (tid & 7) * 8;

    for (int k0 = 0; k0 < K; k0 += kGemmKC) {
        float av8[8], bv8[8];
        const int kg = k0 + ak;
        if constexpr (SA == HHFFBP_C64) {
            if (vec && arow_ok && kg + 8 <= K) {
                const float4 *src = reinterpret_cast<const float4 *>(A + (size_t)arow * K + kg);
                const float4 u = src[0], v = src[1];
                av8[0] = u.x; av8[1] = u.y; av8[2] = u.z; av8[3] = u.w;
                av8[4] = v.x; av8[5] = v.y; av8[6] = v.z; av8[7] = v.w;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    av8[e] = (arow_ok && kg + e < K) ? A[(size_t)arow * K + kg + e] : 0.0f;
            }
        } else {
            if (vec && arow_ok && kg + 8 <= K) {
                // eight half-width reals in one 16-byte load
                const uint4 u = *reinterpret_cast<const uint4 *>(A + (size_t)arow * K + kg);
                const uint32_t w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    av8[2 * e] = Store<SA>::ldr((uint16_t)(w4[e] & 0xffffu));
                    av8[2 * e + 1] = Store<SA>::ldr((uint16_t)(w4[e] >> 16));
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    av8[e] = (arow_ok && kg + e < K) ? Store<SA>::ldr(A[(size_t)arow * K + kg + e]) : 0.0f;
            }
        }
        const int kb = k0 + bk, cg = col0 + bc;
        if (vec && kb < K && cg + 8 <= N) {
            const float4 *src = reinterpret_cast<const float4 *>(B + (size_t)kb * N + cg);
            const float4 u = src[0], v = src[1];
            bv8[0] = u.x; bv8[1] = u.y; bv8[2] = u.z; bv8[3] = u.w;
            bv8[4] = v.x; bv8[5] = v.y; bv8[6] = v.z; bv8[7] = v.w;
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                bv8[e] = (kb < K && cg + e < N) ? B[(size_t)kb * N + cg + e] : 0.0f;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) As[ak + e][ar] = av8[e] * aw;
        *reinterpret_cast<float4 *>(&Bs[bk][bc]) = make_float4(bv8[0], bv8[1], bv8[2], bv8[3]);
        *reinterpret_cast<float4 *>(&Bs[bk][bc + 4]) = make_float4(bv8[4], bv8[5], bv8[6], bv8[7]);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kGemmKC; kk += 4) {
            float av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = As[kk + (lane >> 4)][wr + a * 16 + (lane & 15)];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Bs[kk + (lane >> 4)][wc + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    const float sc = scale ? scale[0] : 1.0f;
    if constexpr (SC == HHFFBP_C64) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = row0 + wr + a * 16 + 4 * (lane >> 4) + r;
                    const int col = col0 + wc + b * 16 + (lane & 15);
                    if (row < M && col < N) {
                        const int crow = c_perm ? c_perm[row] : row;
                        const float cw = c_w ? c_w[crow] : 1.0f;
                        C[(size_t)crow * N + col] = Store<SC>::str(acc[a][b][r] * (sc * cw));
                    }
                }
    } else {
        // Half-width output in 4-byte pairs: lanes 2m and 2m + 1 hold adjacent
        // columns of the same rows; they swap one value per row pair, the even
        // lane then writing both columns of row r and the odd lane both columns
        // of row r + 1 (N = 2 Nr is even, so a pair never straddles the edge).
        const bool odd = lane & 1;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int rp = 0; rp < 4; rp += 2) {
                    const float send = odd ? acc[a][b][rp] : acc[a][b][rp + 1];
                    const float got = __shfl_xor(send, 1, 64);
                    const int r = rp + (odd ? 1 : 0);
                    const float own = odd ? acc[a][b][rp + 1] : acc[a][b][rp];
                    const float lo = odd ? got : own, hi = odd ? own : got;
                    const int row = row0 + wr + a * 16 + 4 * (lane >> 4) + r;
                    const int colp = col0 + wc + b * 16 + (lane & 14);
                    if (row < M && colp < N) {
                        const int crow = c_perm ? c_perm[row] : row;
                        const float s2 = sc * (c_w ? c_w[crow] : 1.0f);
                        const uint32_t v = (uint32_t)Store<SC>::str(lo * s2) |
                                           ((uint32_t)Store<SC>::str(hi * s2) << 16);
                        *reinterpret_cast<uint32_t *>(C + (size_t)crow * N + colp) = v;
                    }
                }
    }
}

// 16-byte staging needs K % 8 == 0, N % 4 == 0 and 16-byte aligned operands.
inline int gemm_vec(const void *A, int K, const float *B, int N)
{
    return (K % 8 == 0 && N % 4 == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0 &&
            reinterpret_cast<uintptr_t>(B) % 16 == 0) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Range compression of complex64 echoes on bf16 MFMA at float32 accuracy.
// Every float32 operand x splits exactly into three bfloat16 parts x = x1 + x2
// + x3, each rounded to nearest from the remainder (8 significant bits a part,
// |x - x1 - x2 - x3| <= 2^-27 |x|).  A product a b is then the sum of the six
// partial products a_i b_j with i + j <= 4 (relative size >= 2^-18; the three
// left out are below 2^-26), each exact in float32, accumulated in float32 by
// v_mfma_f32_32x32x16_bf16: the result carries a float32 GEMM's error.  A is
// read straight from global memory (rows gathered through perm, times the row
// weight) and split in registers; B comes split from the plan in fragment
// order, [k16 step][32-column tile][part][lane][8], so a wave loads each of
// its fragments with one 16-byte load per lane.  A wave covers 64 rows (two
// 32-row tiles) and CT 32-column tiles; the four waves of a block take
// consecutive row groups of the same columns, so their B fragments are one set
// (read once from L2, then from the L1), and the column groups of one row block
// are consecutive logical blocks on one XCD (its rows of A come from HBM once).
// Steps alternate between two register sets, each set reloaded for two steps
// ahead as soon as its step is issued; the MFMAs of a step go product by
// product over the wave's 2 x CT tiles so consecutive MFMAs are independent.
// VEC: K % 16 == 0 and 16-byte aligned rows of A, loaded 16 bytes at a time.
// MFMA operand layout (32 x 32 x 16): lane l holds row (A) or column (B)
// l mod 32 at k = 8 (l div 32) + e, e < 8; result register r of lane l is row
// 8 (r div 4) + 4 (l div 32) + r mod 4, column l mod 32.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void split_bf16x3(const float (&a)[8], bf16x8 &x1, bf16x8 &x2, bf16x8 &x3)
{
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const __bf16 h = (__bf16)a[e];
        const float r1 = a[e] - (float)h;
        const __bf16 m = (__bf16)r1;
        x1[e] = h;
        x2[e] = m;
        x3[e] = (__bf16)(r1 - (float)m);
    }
}

template <int CT, bool VEC>
__global__ __launch_bounds__(kBlock, 2) void k_rc_gemm_x6(const float *__restrict__ A,
                                                        const int32_t *__restrict__ perm, int M, int K,
                                                        const bf16x8 *__restrict__ Bx, int NT, int N,
                                                        float *__restrict__ C,
                                                        const float *__restrict__ scale,
                                                        const float *__restrict__ a_w)
{
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    const int ncg = (NT + CT - 1) / CT;
    const int lb = xcd_block_run((int)blockIdx.x, (int)gridDim.x, ncg);
    const int row0 = ((lb / ncg) * (kBlock / 64) + wave) * 64;
    const int ct0 = (lb % ncg) * CT;  // this wave's first column tile
    const int kl = 8 * (lane >> 5);                                   // its k offset in a step
    const float *arow[2];
    float aw[2];
    bool aok[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int r = row0 + 32 * a + (lane & 31);
        aok[a] = r < M;
        const int src = aok[a] ? (perm ? perm[r] : r) : 0;
        arow[a] = A + (size_t)src * K;
        aw[a] = aok[a] ? (a_w ? a_w[src] : 1.0f) : 0.0f;
    }
    const int KS = (K + 15) / 16;
    auto load_a = [&](int ks, float (&dst)[2][8]) {
        const int k = 16 * ks + kl;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            if (VEC) {  // K % 16 == 0 and 16-byte aligned rows
                const float4 u = *reinterpret_cast<const float4 *>(arow[a] + k);
                const float4 v = *reinterpret_cast<const float4 *>(arow[a] + k + 4);
                dst[a][0] = u.x; dst[a][1] = u.y; dst[a][2] = u.z; dst[a][3] = u.w;
                dst[a][4] = v.x; dst[a][5] = v.y; dst[a][6] = v.z; dst[a][7] = v.w;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) dst[a][e] = (k + e < K) ? arow[a][k + e] : 0.0f;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) dst[a][e] *= aw[a];
        }
    };
    auto load_b = [&](int ks, bf16x8 (&dst)[CT][3]) {
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int ct = min(ct0 + c, NT - 1);  // a tile past N reads the last one; its columns are not stored
#pragma unroll
            for (int q = 0; q < 3; ++q) dst[c][q] = Bx[((size_t)(ks * NT + ct) * 3 + q) * 64 + lane];
        }
    };
    f32x16 acc[2][CT];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][c][r] = 0.0f;
    // one k step: split A, then the six products, smallest first, over the
    // wave's 2 x CT tiles ((A part, B part) per product)
    auto step = [&](const float (&av)[2][8], const bf16x8 (&bv)[CT][3]) {
        bf16x8 x[2][3];
#pragma unroll
        for (int a = 0; a < 2; ++a) split_bf16x3(av[a], x[a][0], x[a][1], x[a][2]);
        constexpr int pa[6] = {2, 0, 1, 1, 0, 0}, pb[6] = {0, 2, 1, 0, 1, 0};
#pragma unroll
        for (int t = 0; t < 6; ++t)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < CT; ++c)
                    acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[a][pa[t]], bv[c][pb[t]], acc[a][c],
                                                                        0, 0, 0);
    };
    // two register sets, steps alternating between them: a set's loads for
    // step ks + 2 are issued right after its step ks, so they are in flight
    // during the other set's step (the scheduling barriers keep the compiler
    // from moving them next to their use)
    float a0[2][8], a1[2][8];
    bf16x8 b0[CT][3], b1[CT][3];
    load_a(0, a0);
    load_b(0, b0);
    if (KS > 1) {
        load_a(1, a1);
        load_b(1, b1);
    }
    for (int ks = 0; ks < KS; ks += 2) {
        __builtin_amdgcn_sched_barrier(0);
        step(a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        if (ks + 2 < KS) {
            load_a(ks + 2, a0);
            load_b(ks + 2, b0);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (ks + 1 < KS) step(a1, b1);
        __builtin_amdgcn_sched_barrier(0);
        if (ks + 3 < KS) {
            load_a(ks + 3, a1);
            load_b(ks + 3, b1);
        }
    }
    const float sc = scale ? scale[0] : 1.0f;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int col = 32 * (ct0 + c) + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = row0 + 32 * a + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (row < M && col < N) C[(size_t)row * N + col] = acc[a][c][r] * sc;
            }
        }
}

// The same split GEMM with its operands streamed through a ring of kX6Stages
// LDS stages by direct global-to-LDS loads (global_load_lds_dwordx4: each lane's
// 16 bytes land at the wave-uniform LDS address + 16 x lane, with no registers
// held while they are in flight), so two k steps are in flight while one is
// computed.  A block of kX6Waves waves covers 32 kX6Waves rows, each wave 32
// rows and the block's 3 column tiles (104 VGPRs: four waves per SIMD).  A stage
// holds each wave's rows of A for one k step (2 loads of 1 KB: load h, lane l ->
// row l mod 32, k 8 h + 4 (l div 32) .. +3; the MFMA operand of lane L is then
// the 32 bytes at load L div 32, lanes L mod 32 and L mod 32 + 32) and the
// block's 9 B fragments (1 KB each: wave 0 loads two, waves 1-7 one and a
// discarded tenth, so every wave issues 4 loads a step).  Per step: wait for
// this wave's loads of the step, a barrier (everyone's loads of the step have
// landed and the previous step's stage is free), the loads of the step two
// ahead into that stage, then the fragments from LDS, the split and the 18
// MFMAs.  Needs K % 16 == 0 and 16-byte aligned rows of A.
constexpr int kX6Stages = 3;
constexpr int kX6Waves = 8;  // 32 rows of A each
// two B fragment loads per wave cover the 9 fragments (and a discarded tenth)
static_assert(kX6Waves >= 5 && kX6Waves <= 9, "B fragments per wave");
constexpr int kX6StageBytes = kX6Waves * 2048 + 10 * 1024;
constexpr int kX6LdsBytes = kX6Stages * kX6StageBytes;

// 16 bytes per lane from global memory to LDS address lds + 16 x lane (lds
// wave-uniform).  Issued as assembly so that the compiler's wait insertion,
// which cannot tell which LDS bytes a direct load writes, does not drain every
// load in flight before each LDS read; the kernel waits on vmcnt itself.
__device__ __forceinline__ void dma16(const void *g, uint32_t lds)
{
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
                 :
                 : "v"(g), "s"(lds)
                 : "memory", "m0");
}

__global__ __launch_bounds__(64 * kX6Waves, 2) void k_rc_gemm_x6_dma(const float *__restrict__ A,
                                                            const int32_t *__restrict__ perm, int M, int K,
                                                            const bf16x8 *__restrict__ Bx, int NT, int N,
                                                            float *__restrict__ C,
                                                            const float *__restrict__ scale,
                                                            const float *__restrict__ a_w)
{
    constexpr int CT = 3;
    extern __shared__ __align__(16) unsigned char lds[];
    const int lane = (int)(threadIdx.x & 63);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lds0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned char *)lds;
    const int ncg = (NT + CT - 1) / CT;
    const int lb = xcd_block_run((int)blockIdx.x, (int)gridDim.x, ncg);
    const int row0 = ((lb / ncg) * kX6Waves + wave) * 32;
    const int ct0 = (lb % ncg) * CT;
    const int KS = K / 16;
    const float *asrc;
    float aw;
    {
        const int r = row0 + (lane & 31);
        const bool ok = r < M;
        const int src = ok ? (perm ? perm[r] : r) : 0;
        asrc = A + (size_t)src * K + 4 * (lane >> 5);
        aw = ok ? (a_w ? a_w[src] : 1.0f) : 0.0f;
    }
    const bf16x8 *bsrc[2];
    int bslot[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int f = wave + kX6Waves * i, ff = f < 3 * CT ? f : 0;
        bslot[i] = f < 3 * CT ? f : 3 * CT;
        bsrc[i] = Bx + ((size_t)min(ct0 + ff / 3, NT - 1) * 3 + ff % 3) * 64 + lane;
    }
    __builtin_amdgcn_s_waitcnt(0xF70);
    auto issue = [&](int ks) {
        const uint32_t st = lds0 + (uint32_t)((ks % kX6Stages) * kX6StageBytes);
#pragma unroll
        for (int h = 0; h < 2; ++h) dma16(asrc + 16 * ks + 8 * h, st + wave * 2048 + h * 1024);
#pragma unroll
        for (int i = 0; i < 2; ++i)
            dma16(bsrc[i] + (size_t)ks * NT * 3 * 64, st + kX6Waves * 2048 + bslot[i] * 1024);
    };
    f32x16 acc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[c][r] = 0.0f;
#pragma unroll
    for (int s = 0; s < kX6Stages - 1; ++s)
        if (s < KS) issue(s);
    for (int ks = 0; ks < KS; ++ks) {
        if (ks + 1 < KS)
            __builtin_amdgcn_s_waitcnt(0xF70 | 4);  // vmcnt(4): the next step's loads may remain
        else
            __builtin_amdgcn_s_waitcnt(0xF70);
        __syncthreads();
        if (ks + kX6Stages - 1 < KS) issue(ks + kX6Stages - 1);
        const unsigned char *st = lds + (ks % kX6Stages) * kX6StageBytes;
        float av[8];
        {
            const unsigned char *pa = st + wave * 2048 + (lane >> 5) * 1024 + (lane & 31) * 16;
            const float4 u = *reinterpret_cast<const float4 *>(pa);
            const float4 v = *reinterpret_cast<const float4 *>(pa + 512);
            av[0] = u.x * aw; av[1] = u.y * aw; av[2] = u.z * aw; av[3] = u.w * aw;
            av[4] = v.x * aw; av[5] = v.y * aw; av[6] = v.z * aw; av[7] = v.w * aw;
        }
        bf16x8 bv[CT][3];
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int q = 0; q < 3; ++q)
                bv[c][q] = *reinterpret_cast<const bf16x8 *>(st + kX6Waves * 2048 + (3 * c + q) * 1024 + lane * 16);
        bf16x8 x[3];
        split_bf16x3(av, x[0], x[1], x[2]);
        constexpr int pa_[6] = {0, 0, 1, 0, 1, 2}, pb_[6] = {0, 1, 0, 2, 1, 0};
#pragma unroll
        for (int t = 0; t < 6; ++t)
#pragma unroll
            for (int c = 0; c < CT; ++c)
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[pa_[t]], bv[c][pb_[t]], acc[c], 0, 0, 0);
    }
    const float sc = scale ? scale[0] : 1.0f;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const int col = 32 * (ct0 + c) + (lane & 31);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = row0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            if (row < M && col < N) C[(size_t)row * N + col] = acc[c][r] * sc;
        }
    }
}

// The same split GEMM with the block's B fragments resident in LDS for the whole
// of K.  A block is one CU's 16 waves and one column group (3 tiles); it stages
// the group's K/16 x 9 fragments (9 KB a k step) once, by direct global-to-LDS
// loads and one barrier, and from then on every wave works alone: it takes 32-row
// tiles of A in turn, loading each lane's 32 bytes of a k step straight into
// registers kBrDepth steps ahead (past the end of a tile, the next tile's first
// steps), so no wave waits on another and the MFMAs of one overlap the loads and
// splits of the others.  The aperture weight of a row scales the finished row
// (diag(w) A B), fetched from the lane that holds it.  Blocks map to XCDs so that
// the column groups of one row stream share an XCD and read the same rows of A
// at about the same time (one HBM read, the others from that XCD's L2).  Needs
// K % (16 kBrDepth) == 0, 16-byte aligned rows of A and K/16 x 9 KB of LDS.
constexpr int kBrWaves = 16;
constexpr int kBrDepth = 4;
constexpr int kBrStepBytes = 9 * 1024;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t cvt_pk_bf16(float a, float b)
{
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef __bf16 h2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f2){a, b}, h2));
}

// split_bf16x3 on pairs: one packed round-to-nearest-even conversion per pair
// and part; a part's float32 value is its bfloat16 shifted up (low half) or
// masked (high half), so the remainders are formed without unpacking.
__device__ __forceinline__ void split_bf16x3_pk(const float4 &u, const float4 &v, bf16x8 &x1, bf16x8 &x2,
                                                bf16x8 &x3)
{
    const float a[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
    u32x4 h, m, t;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const float a0 = a[2 * p], a1 = a[2 * p + 1];
        h[p] = cvt_pk_bf16(a0, a1);
        const float r0 = a0 - __uint_as_float(h[p] << 16), r1 = a1 - __uint_as_float(h[p] & 0xFFFF0000u);
        m[p] = cvt_pk_bf16(r0, r1);
        const float s0 = r0 - __uint_as_float(m[p] << 16), s1 = r1 - __uint_as_float(m[p] & 0xFFFF0000u);
        t[p] = cvt_pk_bf16(s0, s1);
    }
    x1 = __builtin_bit_cast(bf16x8, h);
    x2 = __builtin_bit_cast(bf16x8, m);
    x3 = __builtin_bit_cast(bf16x8, t);
}

__global__ __launch_bounds__(64 * kBrWaves, 1) void k_rc_gemm_x6_br(const float *__restrict__ A,
                                                          const int32_t *__restrict__ perm, int M, int K,
                                                          const bf16x8 *__restrict__ Bx, int NT, int N,
                                                          float *__restrict__ C,
                                                          const float *__restrict__ scale,
                                                          const float *__restrict__ a_w, int spx)
{
    constexpr int CT = 3, D = kBrDepth;
    extern __shared__ __align__(16) unsigned char lds[];
    const bf16x8 *sB = reinterpret_cast<const bf16x8 *>(lds);
    const int lane = (int)(threadIdx.x & 63);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int ncg = (NT + CT - 1) / CT;
    // workgroup b runs on XCD b mod kXcds: the ncg column groups of a stream are
    // consecutive workgroups of one XCD
    const int xcd = (int)blockIdx.x % kXcds, j = (int)blockIdx.x / kXcds;
    const int cg = j % ncg, stream = xcd + kXcds * (j / ncg);
    const int ct0 = cg * CT, KS = K / 16, ntiles = (M + 31) / 32;
    const int tstep = kXcds * spx * kBrWaves;
    int tile = stream * kBrWaves + wave;
    // this lane's row of a tile: its A row (32 bytes a k step from k = 8 (lane div 32))
    // and its aperture weight
    auto row_src = [&](int t) {
        const int r = t * 32 + (lane & 31);
        return r < M ? (perm ? perm[r] : r) : -1;
    };
    auto row_ptr = [&](int src) { return A + (size_t)(src < 0 ? 0 : src) * K + 8 * (lane >> 5); };
    int src_cur = row_src(tile);
    const float *cur = row_ptr(src_cur), *nxt = row_ptr(row_src(tile + tstep));
    float4 ab[D][2];
    {
        const uint32_t lds0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned char *)lds;
        for (int f = wave; f < KS * 9; f += kBrWaves) {
            const int ks = f / 9, cq = f - 9 * ks, c = cq / 3, q = cq - 3 * c;
            dma16(Bx + ((size_t)(ks * NT + min(ct0 + c, NT - 1)) * 3 + q) * 64 + lane, lds0 + (uint32_t)f * 1024);
        }
        __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0)
        __syncthreads();
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        ab[d][0] = *reinterpret_cast<const float4 *>(cur + 16 * d);
        ab[d][1] = *reinterpret_cast<const float4 *>(cur + 16 * d + 4);
    }
    const float sc = scale ? scale[0] : 1.0f;
    for (; tile < ntiles; tile += tstep) {
        f32x16 acc[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[c][r] = 0.0f;
        for (int ks0 = 0; ks0 < KS; ks0 += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int ks = ks0 + d;
                bf16x8 x[3];
                split_bf16x3_pk(ab[d][0], ab[d][1], x[0], x[1], x[2]);
                // refill: step ks + D of this tile, else of the next one
                const int kn = ks + D;
                const float *src = kn < KS ? cur + 16 * kn : nxt + 16 * (kn - KS);
                ab[d][0] = *reinterpret_cast<const float4 *>(src);
                ab[d][1] = *reinterpret_cast<const float4 *>(src + 4);
                const bf16x8 *b = sB + (size_t)ks * 9 * 64 + lane;
                constexpr int pa_[6] = {0, 0, 1, 0, 1, 2}, pb_[6] = {0, 1, 0, 2, 1, 0};
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    const bf16x8 b0 = b[(3 * c) * 64], b1 = b[(3 * c + 1) * 64], b2 = b[(3 * c + 2) * 64];
                    const bf16x8 bv[3] = {b0, b1, b2};
#pragma unroll
                    for (int t = 0; t < 6; ++t)
                        acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[pa_[t]], bv[pb_[t]], acc[c], 0, 0, 0);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // C rows: result register r of lane l is row 8 (r div 4) + 4 (l div 32) + r mod 4
        const int rt = tile * 32;
        const float w_own = src_cur < 0 ? 0.0f : (a_w ? a_w[src_cur] : 1.0f);
        float wr[16];
#pragma unroll
        for (int r = 0; r < 16; ++r)
            wr[r] = sc * (a_w ? __shfl(w_own, 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)) : 1.0f);
        float *crow = C + (size_t)(rt + 4 * (lane >> 5)) * N + 32 * ct0 + (lane & 31);
        const bool full = rt + 32 <= M;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            if (ct0 + c >= NT) break;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int ri = 8 * (r >> 2) + (r & 3);
                if (full || rt + 4 * (lane >> 5) + ri < M) crow[(size_t)ri * N + 32 * c] = acc[c][r] * wr[r];
            }
        }
        src_cur = row_src(tile + tstep);
        cur = nxt;
        nxt = row_ptr(row_src(tile + 2 * tstep));
    }
}

// ---------------------------------------------------------------------------
// Level-1 BP.  One lane per leaf grid point q; the leaf's positions are staged
// through LDS in chunks together with their range profiles (leaf-sorted, so a
// chunk's profiles are one contiguous block, widened to float32 on staging).
// Per (q, i):
//   Delta R = |q - p'_i| - |q - c| = (|delta|^2 - 2 d.delta) / (|q - p'_i| + |q - c|)
//   with |q - p'_i| = sqrt(|q - c|^2 + |delta|^2 - 2 d.delta) (one add and a root)
//   g = sum_w phi_w(t) prof_i[r_first + w],   t = (|q - c| - R0)/dR + Delta R / dR
//   acc += g exp(j 2 kc Delta R)
// and f'(q) = acc exp(j (2 kc |q - c| - Phi(q))), the last factor precomputed.
// RED = false drops the reduction of the carrier's argument to [-1/2, 1/2]
// turn: v_sin / v_cos accept [-256, 256] turns, and the plan selects that form
// only when 2 kc |Delta R| / 2 pi <= 2 kc max|p' - c| / 2 pi stays below 128.
template <int KERNEL, int W, int ST, bool RED>
__global__ __launch_bounds__(kBlock) void k_leaf_bp(const NodeDev *__restrict__ leaves,
                                                    const int32_t *__restrict__ order,
                                                    const BlockItem *__restrict__ blocks,
                                                    const BinWindow *__restrict__ wins,
                                                    const LeafPoint *__restrict__ pts,
                                                    const float4 *__restrict__ posoff,
                                                    const typename Store<ST>::C *__restrict__ prof,
                                                    int Nr, float inv_dR,
                                                    float beta_log2e, float kc_turns,
                                                    const float *__restrict__ scales, int S,
                                                    typename Store<ST>::C *__restrict__ out)
{
    extern __shared__ unsigned char smem[];
    // the plan's workgroup -> block map keeps each leaf's blocks on one XCD
    const int lb = order[blockIdx.x];
    if (lb < 0) return;
    const BlockItem blk = blocks[lb];
    // only the block's bin window [r0, r0 + nrb) is staged, as many positions at a
    // time as kLdsBudget holds
    const BinWindow win = wins[lb];
    const int r0 = win.lo, nrb = win.n;
    const int chunk = leaf_chunk(nrb);
    const int i_first = (int)threadIdx.x / nrb, t_first = (int)threadIdx.x % nrb;
    const int di = kBlock / nrb, dt = kBlock % nrb;
    // complex64: the same two bins at a time (nrb even, see below)
    const int nrb2 = nrb >> 1;
    const int i2_first = (int)threadIdx.x / nrb2, t2_first = (int)threadIdx.x % nrb2;
    const int di2 = kBlock / nrb2, dt2 = kBlock % nrb2;
    float4 *s_pos = reinterpret_cast<float4 *>(smem);
    float2 *s_prof = reinterpret_cast<float2 *>(smem + chunk * sizeof(float4));
    const NodeDev nd = leaves[blk.node];
    const int p = blk.start + threadIdx.x;
    const bool active = p < nd.npts;
    LeafPoint q = active ? pts[nd.val_base + p] : LeafPoint{0, 0, 1, 0, 0, 0, 0, 0};
    const float Rc2 = fmaf(q.dx, q.dx, fmaf(q.dy, q.dy, q.dz * q.dz));
    const float Rc = fast_sqrt(Rc2);
    const float frac_w = q.frac - 0.5f * W;  // tau = t - W/2 relative to the point's bin
    const int bin1 = q.bin + 1;
    // the block's window holds every tap of positions within the slack box
    // (where the position pass clamps them), float32 rounding of tau included
    const float m2x = -2.0f * q.dx, m2y = -2.0f * q.dy, m2z = -2.0f * q.dz;
    float acc_re = 0.0f, acc_im = 0.0f;
    for (int c0 = nd.pos_begin; c0 < nd.pos_end; c0 += chunk) {
        const int n = min(chunk, nd.pos_end - c0);
        __syncthreads();
        for (int t = threadIdx.x; t < n; t += kBlock) s_pos[t] = posoff[c0 + t];
        const typename Store<ST>::C *src = prof + (size_t)c0 * Nr + r0;
        if constexpr (ST == HHFFBP_C64) {
            // the n x nrb tile two bins at a time: the plan makes r0 and nrb even
            // (and Nr is even), so each pair is 16 aligned bytes at both ends;
            // pair e = i nrb/2 + t, thread-strided, (i, t) advanced without a
            // division as below
            const int row2 = Nr >> 1, total = n * nrb2;
            const float4 *src4 = reinterpret_cast<const float4 *>(src);
            float4 *dst4 = reinterpret_cast<float4 *>(s_prof);
            int i = i2_first, t = t2_first;
            constexpr int kSteps2 = (kStageSteps + 1) / 2;
            float4 v[kSteps2];
#pragma unroll
            for (int k = 0; k < kSteps2; ++k) {
                const bool in = k * kBlock + (int)threadIdx.x < total;
                v[k] = src4[in ? i * row2 + t : 0];
                i += di2;
                t += dt2;
                if (t >= nrb2) {
                    t -= nrb2;
                    ++i;
                }
            }
            // a step past the tile loaded pair 0 and stores it back there (the same
            // value the pair's own thread stores): the stores stay unconditional,
            // so the compiler keeps the loads together
#pragma unroll
            for (int k = 0; k < kSteps2; ++k) {
                const int e = k * kBlock + (int)threadIdx.x;
                dst4[e < total ? e : 0] = v[k];
            }
            for (int e = kSteps2 * kBlock + threadIdx.x; e < total; e += kBlock)
                dst4[e] = src4[(size_t)(e / nrb2) * row2 + e % nrb2];
        } else {
            // the n x nrb tile, element e = i nrb + t, thread-strided; (i, t) of e
            // advances by (di, dt) per step, so no division in the loop, and the
            // unrolled steps issue their loads together
            const int total = n * nrb;
            int i = i_first, t = t_first;
            float2 v[kStageSteps];
#pragma unroll
            for (int k = 0; k < kStageSteps; ++k) {
                // a step past the tile reads the tile's first element and stores nothing
                const bool in = k * kBlock + (int)threadIdx.x < total;
                v[k] = Store<ST>::ld(src[in ? i * Nr + t : 0]);
                i += di;
                t += dt;
                if (t >= nrb) {
                    t -= nrb;
                    ++i;
                }
            }
#pragma unroll
            for (int k = 0; k < kStageSteps; ++k)
                if (k * kBlock + (int)threadIdx.x < total) s_prof[k * kBlock + threadIdx.x] = v[k];
            for (int e = kStageSteps * kBlock + threadIdx.x; e < total; e += kBlock)
                s_prof[e] = Store<ST>::ld(src[(size_t)(e / nrb) * Nr + e % nrb]);
        }
        __syncthreads();
        if (active) {
            // two positions per step into two accumulators, so that the two
            // dependency chains (root, reciprocal, LDS tap reads, sine) overlap
            auto pair_term = [&](int i, float &are, float &aim) {
                const float4 d = s_pos[i];
                // |q - p'|^2 = |q - c|^2 + num: R enters only the denominator, where
                // float32 rounding of the sum costs ~1e-8 relative of Delta R
                const float num = fmaf(m2x, d.x, fmaf(m2y, d.y, fmaf(m2z, d.z, d.w)));
                const float R = fast_sqrt(num + Rc2);
                const float dR = num * fast_rcp(R + Rc);
                const float tau = fmaf(dR, inv_dR, frac_w);
                const int r = bin1 - r0 + floor_int(tau);
                const float x = __builtin_amdgcn_fractf(tau);
                const float2 *pr = s_prof + i * nrb + r;
                float gre, gim;
                if constexpr (KERNEL == HHFFBP_RANGE_LINEAR) {
                    const float2 v0 = pr[0], v1 = pr[1];
                    gre = fmaf(x, v1.x - v0.x, v0.x);
                    gim = fmaf(x, v1.y - v0.y, v0.y);
                } else {
                    float w[W];
                    range_weights<KERNEL, W>(x, beta_log2e, w);
                    gre = 0.0f;
                    gim = 0.0f;
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        const float2 v = pr[k];
                        gre = fmaf(w[k], v.x, gre);
                        gim = fmaf(w[k], v.y, gim);
                    }
                }
                float ph = dR * kc_turns;
                if constexpr (RED) ph -= rintf(ph);
                const float sn = sin_turns(ph), cs = cos_turns(ph);
                are = fmaf(gre, cs, fmaf(-gim, sn, are));
                aim = fmaf(gre, sn, fmaf(gim, cs, aim));
            };
            float bre = 0.0f, bim = 0.0f;
            int i = 0;
            for (; i + 1 < n; i += 2) {
                pair_term(i, acc_re, acc_im);
                pair_term(i + 1, bre, bim);
            }
            if (i < n) pair_term(i, acc_re, acc_im);
            acc_re += bre;
            acc_im += bim;
        }
    }
    if (active) {
        const float rs = scales[S] / scales[0];
        out[nd.val_base + p] = Store<ST>::st(make_float2(rs * (acc_re * q.pre_re - acc_im * q.pre_im),
                                                         rs * (acc_re * q.pre_im + acc_im * q.pre_re)));
    }
}

// ---------------------------------------------------------------------------
// Level-1 BP with the range compression fused in (eq. 2 and Sec. IV-A; the
// plan's range_fused option, linear range kernel, complex64).  A block of
// kFusedPoints threads takes as many points of one leaf.  Per chunk of
// kFusedChunk of the leaf's positions it forms their profiles over the block's
// bin window straight from the echoes, P[i][b] = w_i sum_f s_if W[f][b]
// (block-real, on v_mfma_f32_16x16x4f32: the echo rows in LDS k-major, W read
// from global memory), into LDS, and then backprojects them as k_leaf_bp does
// with the linear kernel.  No profile array exists; every block of a leaf
// forms the leaf's profiles over its own window.
constexpr int kFusedChunk = 16;
constexpr int kFusedWaves = kFusedPoints / 64;

inline size_t fused_lds_bytes(int K, int win_max)
{
    const int Kp = (K + 3) & ~3;
    return ((size_t)Kp * kFusedChunk + (size_t)kFusedChunk * 2 * win_max) * sizeof(float) +
           kFusedChunk * sizeof(float4);
}

template <bool RED>
__global__ __launch_bounds__(kFusedPoints) void k_leaf_bp_fused(
    const NodeDev *__restrict__ leaves, const BlockItem *__restrict__ blocks,
    const BinWindow *__restrict__ wins, const LeafPoint *__restrict__ pts,
    const float4 *__restrict__ posoff, const float *__restrict__ echoes,
    const int32_t *__restrict__ perm, const float *__restrict__ aw, int K,
    const float *__restrict__ B, int Nr, float inv_dR, float kc_turns, float2 *__restrict__ out)
{
    extern __shared__ unsigned char smem[];
    const int lb = xcd_block<4>((int)blockIdx.x, (int)gridDim.x);
    const BlockItem blk = blocks[lb];
    const BinWindow win = wins[lb];
    const int r0 = win.lo, nrb = win.n, ncol = 2 * nrb, ldb = 2 * Nr;
    const int Kp = (K + 3) & ~3;
    float *As = reinterpret_cast<float *>(smem);         // [Kp][kFusedChunk], k-major
    float *Ps = As + (size_t)Kp * kFusedChunk;           // [kFusedChunk][2 nrb], block-real
    float4 *s_pos = reinterpret_cast<float4 *>(Ps + (size_t)kFusedChunk * ncol);
    const int tid = (int)threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const NodeDev nd = leaves[blk.node];
    const int p = blk.start + tid;
    const bool active = p < nd.npts;
    LeafPoint q = active ? pts[nd.val_base + p] : LeafPoint{0, 0, 1, 0, 0, 0, 0, 0};
    const float Rc2 = fmaf(q.dx, q.dx, fmaf(q.dy, q.dy, q.dz * q.dz));
    const float Rc = fast_sqrt(Rc2);
    const float frac_w = q.frac - 1.0f;  // tau = t - W/2 (W = 2) relative to the point's bin
    const int bin1 = q.bin + 1;
    const float tau_lo = (float)(r0 - bin1), tau_hi = (float)(r0 + nrb - 2 - bin1);
    const float m2x = -2.0f * q.dx, m2y = -2.0f * q.dy, m2z = -2.0f * q.dz;
    float acc_re = 0.0f, acc_im = 0.0f;
    for (int c0 = nd.pos_begin; c0 < nd.pos_end; c0 += kFusedChunk) {
        const int n = min(kFusedChunk, nd.pos_end - c0);
        __syncthreads();  // the previous chunk's profiles are consumed
        // echo rows of the chunk (weighted), k-major: As[k][i]; rows past n are 0
        for (int t = tid; t < kFusedChunk * Kp; t += kFusedPoints) {
            const int i = t / Kp, k = t - i * Kp;
            float v = 0.0f;
            if (i < n && k < K) {
                const int row = perm[c0 + i];
                v = echoes[(size_t)row * K + k] * (aw ? aw[row] : 1.0f);
            }
            As[k * kFusedChunk + i] = v;
        }
        if (tid < kFusedChunk)
            s_pos[tid] = tid < n ? posoff[c0 + tid] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        __syncthreads();
        // profiles: C[16][ncol] = A[16][K] W[K][2 r0 .. 2 r0 + ncol), one 16-column
        // tile per wave at a time
        for (int ct = wave; ct * 16 < ncol; ct += kFusedWaves) {
            const int col = ct * 16 + (lane & 15);
            const bool cin = col < ncol;
            const float *bcol = B + 2 * r0 + (cin ? col : 0);
            v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
            for (int k = 0; k < Kp; k += 4) {
                const int kk = k + (lane >> 4);
                const float a = As[kk * kFusedChunk + (lane & 15)];
                const float b = (cin && kk < K) ? bcol[(size_t)kk * ldb] : 0.0f;
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
            }
            if (cin) {
#pragma unroll
                for (int r = 0; r < 4; ++r) Ps[(4 * (lane >> 4) + r) * ncol + col] = acc[r];
            }
        }
        __syncthreads();
        if (active) {
            const float2 *prof = reinterpret_cast<const float2 *>(Ps);
            for (int i = 0; i < n; ++i) {
                const float4 d = s_pos[i];
                const float num = fmaf(m2x, d.x, fmaf(m2y, d.y, fmaf(m2z, d.z, d.w)));
                const float R = fast_sqrt(num + Rc2);
                const float dR = num * fast_rcp(R + Rc);
                const float tau = fmaf(dR, inv_dR, frac_w);
                const int r = bin1 - r0 + floor_int(tau);
                const float x = __builtin_amdgcn_fractf(tau);
                const float2 v0 = prof[i * nrb + r], v1 = prof[i * nrb + r + 1];
                const float gre = fmaf(x, v1.x - v0.x, v0.x);
                const float gim = fmaf(x, v1.y - v0.y, v0.y);
                float ph = dR * kc_turns;
                if constexpr (RED) ph -= rintf(ph);
                const float sn = sin_turns(ph), cs = cos_turns(ph);
                acc_re = fmaf(gre, cs, fmaf(-gim, sn, acc_re));
                acc_im = fmaf(gre, sn, fmaf(gim, cs, acc_im));
            }
        }
    }
    if (active)
        out[nd.val_base + p] = make_float2(acc_re * q.pre_re - acc_im * q.pre_im,
                                           acc_re * q.pre_im + acc_im * q.pre_re);
}

// Merge at depth d: parent grid points of the depth-d nodes, children at
// depth d + 1.  Output: compressed parent values.  One wave per (64 parent
// points, child), the points taken in the node's merge order (order: lane slot
// -> point): a block of kBlock threads covers kBlock / CL points, wave w
// interpolating child w % CL for point group w / CL, so each wave's gathers
// stay within one child and follow its points' pencils.  Each lane reads its
// pair's plan-time record (stencil, fractions, and the phase Phi_c - Phi_P
// that restores the child's downconversion and applies the parent's), so the
// kernel holds no geometry; the rotated children meet in LDS and are summed in
// child order.  A launch thus has CL times as many waves as points / 64 to
// hide the gathers' latency.
template <int T, int ST, int K, int CL>
__global__ __launch_bounds__(kBlock) void k_merge(const NodeDev *__restrict__ parents,
                                                  const BlockItem *__restrict__ blocks,
                                                  const int32_t *__restrict__ order,
                                                  const InterpIdx *__restrict__ ridx,
                                                  const InterpGeo *__restrict__ rgeo,
                                                  const NodeDev *__restrict__ children,
                                                  const int32_t *__restrict__ ccolbase,
                                                  const typename Store<ST>::C *__restrict__ cvals,
                                                  const InterpPoly ip,
                                                  const float *__restrict__ scales, int sp,
                                                  int sc, typename Store<ST>::C *__restrict__ out)
{
    __shared__ float2 part[kBlock];
    // the wave index is uniform: readfirstlane lets the child's fields be scalar loads
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    const int lane = (int)(threadIdx.x % 64);
    const int c = wave % CL, grp = wave / CL;
    const int lb = xcd_block<0>((int)blockIdx.x, (int)gridDim.x);
    const BlockItem blk = blocks[lb];
    // the parent's fields one by one: a copy of the whole node would go through
    // scratch memory, as child[c] is indexed at run time
    const NodeDev *nd = parents + blk.node;
    const int npts = nd->npts, vbase = nd->val_base;
    const int slot = blk.start + grp * 64 + lane;  // the point is order[vbase + slot]
    const size_t r = (size_t)lb * kBlock + threadIdx.x;
    const InterpIdx ix = ridx[r];
    float are = 0.0f, aim = 0.0f;
    if (ix.cij != kNoPair) {
        const InterpGeo g = rgeo[r];
        const NodeDev ch = children[nd->child[c]];
        float wu[T], wv[T], wn[T];
        interp_weights3<T, K>(ip, g.fu, g.fv, g.fn, wu, wv, wn);
        const float2 v = interp_rec<T, ST>(ch, ccolbase, cvals, (int)(ix.cij & 0xffffu),
                                           (int)(ix.cij >> 16), ix.l0, wu, wv, wn);
        rotate_mac(v, g.turns, are, aim);
    }
    part[threadIdx.x] = make_float2(are, aim);
    __syncthreads();
    if (c == 0 && slot < npts) {
        const int p = order[vbase + slot];
        float sre = 0.0f, sim = 0.0f;
#pragma unroll
        for (int k = 0; k < CL; ++k) {
            const float2 q = part[(grp * CL + k) * 64 + lane];
            sre += q.x;
            sim += q.y;
        }
        // an absent parent point (no preimage) has no pairs and holds 0
        const float rs = scales[sp] / scales[sc];
        out[vbase + p] = Store<ST>::st(make_float2(rs * sre, rs * sim));
    }
}

// Final stage: user voxels, children are the depth-1 nodes (or the root's own
// grid, then the only child); scales[sc] is their storage scale.  One lane per voxel,
// a block per brick of kBrickX x kBrickY x kBrickZ voxels (lane t: z = t mod
// kBrickZ fastest, then y, then x).  Per child, the block first stages the child's
// values over the brick's stencil box (TileBox, from the plan) into LDS: a
// table of the box's columns (where each column's pencil starts and which box
// indices it covers), then every pencil value inside the box, thread-strided.
// Box points outside the pencils are left unwritten: every stencil tap lies in
// a pencil (the plan checks each record's stencil against them).  A lane whose
// stencil lies inside the box then reads its T^3 taps from LDS in the same
// order as the pencil path; one outside it (or a child without a box) gathers
// from the pencils.  Each (voxel, child) pair's stencil, fractions and phase
// Phi_c come from its plan-time record.  CS > 0: every box has column stride
// CS, and the taps' offsets within a stencil row become immediates.
template <int T, int ST, int K, bool BOX_ONLY, int CS>
__global__ __launch_bounds__(kBlock) void k_final(const NodeDev *__restrict__ children,
                                                  int nchild, const ColEntry *__restrict__ ccols,
                                                  const int32_t *__restrict__ ccolbase,
                                                  const typename Store<ST>::C *__restrict__ cvals,
                                                  const TileBox *__restrict__ tiles,
                                                  const InterpIdx *__restrict__ ridx,
                                                  const InterpGeo *__restrict__ rgeo,
                                                  const InterpPoly ip,
                                                  const float *__restrict__ scales, int sc,
                                                  int nx, int ny, int nz, int box_vals,
                                                  float2 *__restrict__ image)
{
    // Dynamic LDS, sized by the plan's largest box: box_vals values (columns
    // tb.cs apart), then one spare value per thread, the target of staging
    // slots that hold nothing (unconditional loads and stores keep a round's
    // loads in flight together), then per box column the value offset of box
    // index l = 0 and lo | n << 16 for the box indices [lo, lo + n) its pencil
    // covers.
    extern __shared__ float2 s_tile[];
    int2 *s_col = reinterpret_cast<int2 *>(s_tile + box_vals + kBlock);
    const int bz = (nz + kBrickZ - 1) / kBrickZ, by = (ny + kBrickY - 1) / kBrickY;
    const int brick = (int)blockIdx.x;
    const int kx = brick / (by * bz), ky = (brick / bz) % by, kz = brick % bz;
    const int t = (int)threadIdx.x;
    const int ix = kx * kBrickX + t / (kBrickY * kBrickZ), iy = ky * kBrickY + (t / kBrickZ) % kBrickY,
              iz = kz * kBrickZ + t % kBrickZ;
    const bool inside = ix < nx && iy < ny && iz < nz;
    float are = 0.0f, aim = 0.0f;
    for (int c = 0; c < nchild; ++c) {
        const NodeDev ch = children[c];
        const TileBox tb = tiles[(size_t)brick * nchild + c];
        const int ncol = tb.ni * tb.nj;
        // this lane's record, loaded before the staging so that its latency
        // overlaps the table and the box (a barrier keeps the compiler from
        // moving global loads above it)
        const size_t r = ((size_t)brick * nchild + c) * kBlock + t;
        const InterpIdx rx = ridx[r];
        const InterpGeo g = rgeo[r];
        __syncthreads();  // the previous child's box and table are consumed
        if (tb.ni > 0) {
            const ColEntry *ccol = ccols + ch.col_base + (tb.i0 - ch.i0) * ch.nj + (tb.j0 - ch.j0);
            for (int k = t; k < ncol; k += kBlock) {
                const int ci = (k * tb.inv_nj) >> 22, cj = k - ci * tb.nj;
                const ColEntry en = ld_u32(ccol, (uint32_t)(ci * ch.nj + cj));
                const int lo = max(en.lo - tb.l0, 0), hi = min(en.hi - tb.l0, tb.nl - 1);
                s_col[k] = make_int2(en.off - en.lo + tb.l0, lo | (max(hi - lo + 1, 0) << 16));
            }
        }
        __syncthreads();
        if (tb.ni > 0) {
            // box point e = column * nl + l, thread-strided in rounds of
            // kStageRound points per thread (a uniform trip count): per round
            // all table reads, then all value loads, then the stores; a point
            // outside the pencils (or past the box) loads the child's first
            // value into this thread's spare slot
            const int items = ncol * tb.nl, stride = CS > 0 ? CS : tb.cs;
            const typename Store<ST>::C *cv = cvals + ch.val_base;
#pragma unroll 1
            for (int e0 = 0; e0 < items; e0 += kStageRound * kBlock) {
                uint32_t src[kStageRound];
                int dst[kStageRound];
#pragma unroll
                for (int k = 0; k < kStageRound; ++k) {
                    const int e = e0 + k * kBlock + t;
                    const int col = min((int)(((uint32_t)e * (uint32_t)tb.inv_nl) >> 22), ncol - 1);
                    const int l = e - col * tb.nl;
                    const int2 q = s_col[col];
                    const bool take = (e < items) & ((unsigned)(l - (q.y & 0xffff)) < (unsigned)(q.y >> 16));
                    src[k] = take ? (uint32_t)(q.x + l) : 0u;
                    dst[k] = take ? col * stride + l : box_vals + t;
                }
                float2 v[kStageRound];
#pragma unroll
                for (int k = 0; k < kStageRound; ++k) v[k] = Store<ST>::ld(ld_u32(cv, src[k]));
#pragma unroll
                for (int k = 0; k < kStageRound; ++k) s_tile[dst[k]] = v[k];
            }
        }
        __syncthreads();
        if (inside && rx.cij != kNoPair) {
            const int ci0 = (int)(rx.cij & 0xffffu), cj0 = (int)(rx.cij >> 16);
            float wu[T], wv[T], wn[T];
            interp_weights3<T, K>(ip, g.fu, g.fv, g.fn, wu, wv, wn);
            const int ti = ci0 + ch.i0 - tb.i0, tj = cj0 + ch.j0 - tb.j0, tl = rx.l0 - tb.l0;
            float2 val;
            // BOX_ONLY: the plan checked that every stencil lies in its box
            if (BOX_ONLY || (tb.ni > 0 && (unsigned)ti <= (unsigned)(tb.ni - T) &&
                             (unsigned)tj <= (unsigned)(tb.nj - T) && (unsigned)tl <= (unsigned)(tb.nl - T)))
                val = CS > 0 ? interp_box<T, CS>(s_tile + (ti * tb.nj + tj) * CS + tl, tb.nj, wu, wv, wn)
                             : interp_box<T, 0>(s_tile + (ti * tb.nj + tj) * tb.cs + tl, tb.nj, wu, wv, wn,
                                                tb.cs);
            else
                val = interp_rec<T, ST>(ch, ccolbase, cvals, ci0, cj0, rx.l0, wu, wv, wn);
            rotate_mac(val, g.turns, are, aim);
        }
    }
    if (inside) {
        const float rs = 1.0f / scales[sc];
        image[((size_t)ix * ny + iy) * nz + iz] = make_float2(rs * are, rs * aim);
    }
}

// ---------------------------------------------------------------------------
// Direct BP on range profiles, eq. (3).  A block is a 4 x 8 x 8 voxel tile with
// a float64 reference point at its centre.  Per staged position the reference
// distance R_ref, its bin and fraction and the carrier exp(j 2 kc R_ref) are
// formed once in float64; per voxel only Delta R = |p - p'| - R_ref enters
// float32:  Delta R = (|e|^2 - 2 e.delta) / (|p - p'| + R_ref), e = p - ref.
struct StagedPos {
    float dx, dy, dz;  // p' - ref
    float rref;        // |p' - ref| (float32, as a denominator only)
    int32_t bin;       // floor((R_ref - R0)/dR) + 1
    float frac;        // fractional part minus W/2
    float car_re, car_im;
};

template <int KERNEL, int W, int ST>
__global__ __launch_bounds__(kBlock) void k_direct_bp(
    const double *__restrict__ pos64, int n_pos, const typename Store<ST>::C *__restrict__ prof,
    int Nr, int chunk, double R0, double dR, float inv_dR, float beta_log2e, double kc,
    float kc_turns, double ox, double oy, double oz, double sx, double sy, double sz, int nx,
    int ny, int nz, const float *__restrict__ scales, float2 *__restrict__ image)
{
    extern __shared__ unsigned char smem[];
    StagedPos *s_pos = reinterpret_cast<StagedPos *>(smem);
    float2 *s_prof = reinterpret_cast<float2 *>(smem + chunk * sizeof(StagedPos));
    const int tnx = (nx + 3) / 4, tny = (ny + 7) / 8;
    const int b = blockIdx.x;
    const int tx = b % tnx, ty = (b / tnx) % tny, tz = b / (tnx * tny);
    const int lx = threadIdx.x >> 6, ly = (threadIdx.x >> 3) & 7, lz = threadIdx.x & 7;
    const int ix = tx * 4 + lx, iy = ty * 8 + ly, iz = tz * 8 + lz;
    const bool active = ix < nx && iy < ny && iz < nz;
    const double rx = ox + (tx * 4 + 1.5) * sx, ry = oy + (ty * 8 + 3.5) * sy,
                 rz = oz + (tz * 8 + 3.5) * sz;
    const float ex = (float)((lx - 1.5) * sx), ey = (float)((ly - 3.5) * sy),
                ez = (float)((lz - 3.5) * sz);
    const float e2 = ex * ex + ey * ey + ez * ez;
    float acc_re = 0.0f, acc_im = 0.0f;
    for (int c0 = 0; c0 < n_pos; c0 += chunk) {
        const int n = min(chunk, n_pos - c0);
        __syncthreads();
        if (threadIdx.x < n) {
            const int i = c0 + threadIdx.x;
            const double dx = pos64[3 * i] - rx, dy = pos64[3 * i + 1] - ry,
                         dz = pos64[3 * i + 2] - rz;
            const double rr = sqrt(dx * dx + dy * dy + dz * dz);
            const double t = (rr - R0) / dR;
            const double fb = floor(t);
            double turns = rr * (kc / kPi);
            turns -= rint(turns);
            double sn, cs;
            sincos(2.0 * kPi * turns, &sn, &cs);
            StagedPos sp;
            sp.dx = (float)dx;
            sp.dy = (float)dy;
            sp.dz = (float)dz;
            sp.rref = (float)rr;
            sp.bin = (int)fb + 1;                   // first tap is floor(t - W/2) + 1
            sp.frac = (float)(t - fb) - 0.5f * W;   // tau = t - W/2 relative to bin
            sp.car_re = (float)cs;
            sp.car_im = (float)sn;
            s_pos[threadIdx.x] = sp;
        }
        const typename Store<ST>::C *src = prof + (size_t)c0 * Nr;
        for (int t = threadIdx.x; t < n * Nr; t += kBlock) s_prof[t] = Store<ST>::ld(src[t]);
        __syncthreads();
        if (active) {
            for (int i = 0; i < n; ++i) {
                const StagedPos sp = s_pos[i];
                // |q - p'|^2 = |p' - ref|^2 + num, R only in the denominator
                const float num = e2 - 2.0f * (ex * sp.dx + ey * sp.dy + ez * sp.dz);
                const float R = fast_sqrt(fmaf(sp.rref, sp.rref, num));
                const float dr = num * fast_rcp(R + sp.rref);
                const float tau = fmaf(dr, inv_dR, sp.frac);
                const float fl = floorf(tau);
                const float x = tau - fl;
                const int r = min(max(sp.bin + (int)fl, 0), Nr - W);
                float w[W];
                range_weights<KERNEL, W>(x, beta_log2e, w);
                const float2 *pr = s_prof + i * Nr + r;
                float gre = 0.0f, gim = 0.0f;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    const float2 v = pr[k];
                    gre = fmaf(w[k], v.x, gre);
                    gim = fmaf(w[k], v.y, gim);
                }
                float ph = dr * kc_turns;
                ph -= rintf(ph);
                const float sn = sin_turns(ph), cs = cos_turns(ph);
                // carrier = exp(j 2 kc R_ref) exp(j 2 kc Delta R)
                const float cre = sp.car_re * cs - sp.car_im * sn;
                const float cim = sp.car_re * sn + sp.car_im * cs;
                acc_re = fmaf(gre, cre, fmaf(-gim, cim, acc_re));
                acc_im = fmaf(gre, cim, fmaf(gim, cre, acc_im));
            }
        }
    }
    if (active) {
        const float rs = 1.0f / scales[0];
        image[((int64_t)ix * ny + iy) * nz + iz] = make_float2(rs * acc_re, rs * acc_im);
    }
}

// Direct BP of eq. (4), f(p) = sum_i sum_f s_if exp(j 2 k_f |p - p'_i|), no range
// compression.  A block is a 4 x 8 x 8 voxel tile with a float64 reference point
// at its centre.  Per staged position the block forms c_if = s_if exp(j 2 k_f
// R_ref) from the float64 reference distance (the phase reduced to turns in
// float64); per voxel only Delta R = |p - p'| - R_ref enters float32, in the
// cancellation-free form of the range-profile kernel, and
//   f(p) += sum_f c_if exp(j 2 k_f Delta R).
// With equispaced frequencies (EQ), k_f = k_0 + f dk, that sum is
// exp(j 2 k_0 Delta R) sum_f c_if z^f with z = exp(j 2 dk Delta R), evaluated by
// Horner's rule: four FMA per frequency and no trigonometry per frequency.
struct ExactPos {
    float dx, dy, dz;  // p' - ref
    float rref;        // |p' - ref| (float32, as a denominator only)
};

inline int exact_chunk(int n_f)
{
    const size_t per = sizeof(ExactPos) + sizeof(double) + sizeof(float) + (size_t)n_f * sizeof(float2);
    const int c = (int)(kLdsBudget / per);
    return c > 32 ? 32 : (c < 1 ? 1 : c);
}

template <int ST, bool EQ>
__global__ __launch_bounds__(kBlock) void k_direct_exact(
    const double *__restrict__ pos64, int n_pos, const typename Store<ST>::C *__restrict__ echoes,
    int n_f, const double *__restrict__ kf, const float *__restrict__ kf_turns, float k0_turns,
    float dk_turns, int chunk, const float *__restrict__ wts, double ox, double oy, double oz,
    double sx, double sy, double sz, int nx, int ny, int nz, float2 *__restrict__ image)
{
    extern __shared__ unsigned char smem[];
    double *s_rref = reinterpret_cast<double *>(smem);
    ExactPos *s_pos = reinterpret_cast<ExactPos *>(smem + chunk * sizeof(double));
    float2 *s_c = reinterpret_cast<float2 *>(smem + chunk * (sizeof(double) + sizeof(ExactPos)));
    float *s_w = reinterpret_cast<float *>(s_c + (size_t)chunk * n_f);
    const int tnx = (nx + 3) / 4, tny = (ny + 7) / 8;
    const int b = blockIdx.x;
    const int tx = b % tnx, ty = (b / tnx) % tny, tz = b / (tnx * tny);
    const int lx = threadIdx.x >> 6, ly = (threadIdx.x >> 3) & 7, lz = threadIdx.x & 7;
    const int ix = tx * 4 + lx, iy = ty * 8 + ly, iz = tz * 8 + lz;
    const bool active = ix < nx && iy < ny && iz < nz;
    const double rx = ox + (tx * 4 + 1.5) * sx, ry = oy + (ty * 8 + 3.5) * sy,
                 rz = oz + (tz * 8 + 3.5) * sz;
    const float ex = (float)((lx - 1.5) * sx), ey = (float)((ly - 3.5) * sy),
                ez = (float)((lz - 3.5) * sz);
    const float e2 = ex * ex + ey * ey + ez * ez;
    float acc_re = 0.0f, acc_im = 0.0f;
    for (int c0 = 0; c0 < n_pos; c0 += chunk) {
        const int n = min(chunk, n_pos - c0);
        __syncthreads();
        if ((int)threadIdx.x < n) {
            const int i = c0 + threadIdx.x;
            const double dx = pos64[3 * i] - rx, dy = pos64[3 * i + 1] - ry,
                         dz = pos64[3 * i + 2] - rz;
            const double rr = sqrt(dx * dx + dy * dy + dz * dz);
            s_rref[threadIdx.x] = rr;
            s_pos[threadIdx.x] = ExactPos{(float)dx, (float)dy, (float)dz, (float)rr};
            s_w[threadIdx.x] = wts ? wts[i] : 1.0f;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < n * n_f; t += kBlock) {
            const int i = t / n_f, f = t - i * n_f;
            double turns = kf[f] * s_rref[i] * (1.0 / kPi);  // 2 k_f R_ref / 2 pi
            turns -= rint(turns);
            const float tf = (float)turns;
            const float sn = sin_turns(tf), cs = cos_turns(tf);
            float2 v = Store<ST>::ld(echoes[(size_t)(c0 + i) * n_f + f]);
            v.x *= s_w[i];
            v.y *= s_w[i];
            s_c[t] = make_float2(v.x * cs - v.y * sn, v.x * sn + v.y * cs);
        }
        __syncthreads();
        if (active) {
            for (int i = 0; i < n; ++i) {
                const ExactPos sp = s_pos[i];
                // |q - p'|^2 = |p' - ref|^2 + num, R only in the denominator
                const float num = e2 - 2.0f * (ex * sp.dx + ey * sp.dy + ez * sp.dz);
                const float R = fast_sqrt(fmaf(sp.rref, sp.rref, num));
                const float dr = num * fast_rcp(R + sp.rref);
                const float2 *cf = s_c + i * n_f;
                float hre, him;
                if constexpr (EQ) {
                    float zt = dr * dk_turns;
                    zt -= rintf(zt);
                    const float zr = cos_turns(zt), zi = sin_turns(zt);
                    hre = cf[n_f - 1].x;
                    him = cf[n_f - 1].y;
#pragma unroll 4
                    for (int f = n_f - 2; f >= 0; --f) {
                        const float2 c = cf[f];
                        const float r = fmaf(hre, zr, fmaf(-him, zi, c.x));
                        him = fmaf(hre, zi, fmaf(him, zr, c.y));
                        hre = r;
                    }
                    float t0 = dr * k0_turns;
                    t0 -= rintf(t0);
                    const float cr = cos_turns(t0), ci = sin_turns(t0);
                    const float r = hre * cr - him * ci;
                    him = hre * ci + him * cr;
                    hre = r;
                } else {
                    hre = 0.0f;
                    him = 0.0f;
                    for (int f = 0; f < n_f; ++f) {
                        float tt = dr * kf_turns[f];
                        tt -= rintf(tt);
                        const float cr = cos_turns(tt), ci = sin_turns(tt);
                        const float2 c = cf[f];
                        hre = fmaf(c.x, cr, fmaf(-c.y, ci, hre));
                        him = fmaf(c.x, ci, fmaf(c.y, cr, him));
                    }
                }
                acc_re += hre;
                acc_im += him;
            }
        }
    }
    if (active) image[((int64_t)ix * ny + iy) * nz + iz] = make_float2(acc_re, acc_im);
}

template <int ST>
hipError_t launch_direct_exact(const Plan &P, const void *echoes, const double *pos64, void *image,
                               hipStream_t st)
{
    using C = typename Store<ST>::C;
    const hhffbp_config &c = P.cfg;
    const int nx = (int)c.grid_dims[0], ny = (int)c.grid_dims[1], nz = (int)c.grid_dims[2];
    const int nblk = ((nx + 3) / 4) * ((ny + 7) / 8) * ((nz + 7) / 8);
    const int nf = (int)c.n_freq;
    const int chunk = exact_chunk(nf);
    const size_t sh =
        (size_t)chunk * (sizeof(double) + sizeof(ExactPos) + sizeof(float) + (size_t)nf * sizeof(float2));
    const float k0t = (float)(P.k0 / kPi), dkt = (float)(P.dk / kPi);
    if (P.k_equispaced)
        hipLaunchKernelGGL((k_direct_exact<ST, true>), dim3(nblk), dim3(kBlock), sh, st, pos64,
                           (int)c.n_pos, (const C *)echoes, nf, (const double *)P.dev.kf,
                           (const float *)P.dev.kf_turns, k0t, dkt, chunk,
                           (const float *)P.dev.weights, c.grid_origin[0],
                           c.grid_origin[1], c.grid_origin[2], c.grid_pitch[0], c.grid_pitch[1],
                           c.grid_pitch[2], nx, ny, nz, (float2 *)image);
    else
        hipLaunchKernelGGL((k_direct_exact<ST, false>), dim3(nblk), dim3(kBlock), sh, st, pos64,
                           (int)c.n_pos, (const C *)echoes, nf, (const double *)P.dev.kf,
                           (const float *)P.dev.kf_turns, k0t, dkt, chunk,
                           (const float *)P.dev.weights, c.grid_origin[0],
                           c.grid_origin[1], c.grid_origin[2], c.grid_pitch[0], c.grid_pitch[1],
                           c.grid_pitch[2], nx, ny, nz, (float2 *)image);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <int KERNEL, int W, int ST>
hipError_t launch_bp_kernels(const Plan &P, const double *pos64, const void *prof,
                             const float4 *posoff, char *ws, void *image, const float *scales,
                             hipStream_t st)
{
    using C = typename Store<ST>::C;
    const float inv_dR = (float)(1.0 / P.dR);
    const float beta_log2e = (float)(P.beta * 1.4426950408889634);
    const float kc_turns = (float)(P.kc / kPi);
    const hhffbp_config &c = P.cfg;
    if (P.S == 0) {
        const int nx = (int)c.grid_dims[0], ny = (int)c.grid_dims[1], nz = (int)c.grid_dims[2];
        const int nblk = ((nx + 3) / 4) * ((ny + 7) / 8) * ((nz + 7) / 8);
        const int chunk = pos_chunk(P.Nr, sizeof(StagedPos));
        const size_t sh = chunk * (sizeof(StagedPos) + P.Nr * sizeof(float2));
        hipLaunchKernelGGL((k_direct_bp<KERNEL, W, ST>), dim3(nblk), dim3(kBlock), sh, st, pos64,
                           (int)c.n_pos, (const C *)prof, (int)P.Nr, chunk, P.R0, P.dR, inv_dR,
                           beta_log2e, P.kc, kc_turns, c.grid_origin[0], c.grid_origin[1],
                           c.grid_origin[2], c.grid_pitch[0], c.grid_pitch[1], c.grid_pitch[2], nx,
                           ny, nz, scales, (float2 *)image);
        return hipGetLastError();
    }
    // leaf_chunk() keeps a chunk within kLdsBudget, but never below one position
    const size_t sh = std::max(kLdsBudget, sizeof(float4) + (size_t)P.leaf_win_max * sizeof(float2));
    // |Delta R| <= |p' - c| (triangle inequality): the carrier's argument stays
    // below 128 turns without reduction when the plan's leaf reach allows it
    if (P.leaf_reach * (P.kc / kPi) < 128.0)
        hipLaunchKernelGGL((k_leaf_bp<KERNEL, W, ST, false>), dim3(P.n_blocks_leaf_phys), dim3(kBlock), sh,
                           st, (const NodeDev *)P.dev.nodes[P.S], (const int32_t *)P.dev.leaf_order,
                           (const BlockItem *)P.dev.leaf_blocks,
                           (const BinWindow *)P.dev.leaf_wins, (const LeafPoint *)P.dev.leafpts,
                           posoff, (const C *)prof, (int)P.Nr, inv_dR, beta_log2e, kc_turns,
                           scales, P.S,
                           (C *)(ws + P.ws_vals[P.S]));
    else
        hipLaunchKernelGGL((k_leaf_bp<KERNEL, W, ST, true>), dim3(P.n_blocks_leaf_phys), dim3(kBlock), sh,
                           st, (const NodeDev *)P.dev.nodes[P.S], (const int32_t *)P.dev.leaf_order,
                           (const BlockItem *)P.dev.leaf_blocks,
                           (const BinWindow *)P.dev.leaf_wins, (const LeafPoint *)P.dev.leafpts,
                           posoff, (const C *)prof, (int)P.Nr, inv_dR, beta_log2e, kc_turns,
                           scales, P.S,
                           (C *)(ws + P.ws_vals[P.S]));
    return hipGetLastError();
}

template <int T, int ST, int K, int CL>
hipError_t launch_merges(const Plan &P, char *ws, void *image, const float *scales, hipStream_t st,
                         hipEvent_t *ev)
{
    using C = typename Store<ST>::C;
    for (int d = P.S - 1; d >= P.F; --d) {
        if (P.n_blocks_merge_fwd[d] > 0) {
            hipLaunchKernelGGL((k_merge<T, ST, K, CL>), dim3(P.n_blocks_merge_fwd[d]), dim3(kBlock),
                               0, st, (const NodeDev *)P.dev.nodes[d],
                               (const BlockItem *)P.dev.merge_blocks_fwd[d],
                               (const int32_t *)P.dev.merge_order[d],
                               (const InterpIdx *)P.dev.merge_idx[d], (const InterpGeo *)P.dev.merge_geo[d],
                               (const NodeDev *)P.dev.nodes[d + 1],
                               (const int32_t *)P.dev.colbase[d + 1],
                               (const C *)(ws + P.ws_vals[d + 1]), P.ipoly_for(d + 1), scales,
                               P.scale_slot(d), P.scale_slot(d + 1), (C *)(ws + P.ws_vals[d]));
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (ev) (void)hipEventRecord(*ev++, st);
    }
    const hhffbp_config &c = P.cfg;
    const int nx = (int)c.grid_dims[0], ny = (int)c.grid_dims[1], nz = (int)c.grid_dims[2];
    auto final_kernel = !P.final_box_only       ? k_final<T, ST, K, false, 0>
                        : P.final_cs == kFinalCS ? k_final<T, ST, K, true, kFinalCS>
                                                 : k_final<T, ST, K, true, 0>;
    hipLaunchKernelGGL(final_kernel, dim3(P.n_bricks), dim3(kBlock), final_lds_bytes(P), st,
                       (const NodeDev *)P.dev.nodes[P.F], (int)P.compact_to_tree[P.F].size(),
                       (const ColEntry *)P.dev.cols[P.F], (const int32_t *)P.dev.colbase[P.F],
                       (const C *)(ws + P.ws_vals[P.F]), (const TileBox *)P.dev.final_tiles, (const InterpIdx *)P.dev.final_idx,
                       (const InterpGeo *)P.dev.final_geo, P.ipoly_for(P.F), scales, P.scale_slot(P.F), nx, ny,
                       nz, (int)P.final_box_vals, (float2 *)image);
    hipError_t e = hipGetLastError();
    if (ev && e == hipSuccess) (void)hipEventRecord(*ev, st);
    return e;
}

template <int ST, int CL>
hipError_t dispatch_merges(const Plan &P, char *ws, void *image, const float *scales,
                           hipStream_t st, hipEvent_t *ev)
{
    if (P.ipoly.kind == HHFFBP_INTERP_BANDLIMITED)
        return (P.T == 4) ? launch_merges<4, ST, HHFFBP_INTERP_BANDLIMITED, CL>(P, ws, image, scales, st, ev)
                          : launch_merges<6, ST, HHFFBP_INTERP_BANDLIMITED, CL>(P, ws, image, scales, st, ev);
    return (P.T == 4) ? launch_merges<4, ST, HHFFBP_INTERP_LAGRANGE, CL>(P, ws, image, scales, st, ev)
                      : launch_merges<6, ST, HHFFBP_INTERP_LAGRANGE, CL>(P, ws, image, scales, st, ev);
}

template <int ST>
hipError_t launch_scales(const Plan &P, const void *echoes, char *ws, hipStream_t st)
{
    float *scales = (float *)(ws + P.ws_scales);
    float *part = (float *)(ws + P.ws_amax);
    const int ns = P.n_scales();
    if (ST == HHFFBP_F16) {
        const int64_t n = 2 * P.cfg.n_pos * P.cfg.n_freq;
        const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kAbsmaxParts, (n + kBlock - 1) / kBlock));
        const int64_t per = 16 / (int64_t)sizeof(typename Store<ST>::R);
        const int64_t n16 = reinterpret_cast<uintptr_t>(echoes) % 16 == 0 ? n / per : 0;
        hipLaunchKernelGGL((k_absmax<ST>), dim3(nb), dim3(kBlock), 0, st,
                           (const typename Store<ST>::R *)echoes, n, n16, part);
        hipLaunchKernelGGL(k_scales, dim3(1), dim3(64), 0, st, (const float *)part, nb,
                           (const float *)P.dev.scale_mult, ns, scales);
    } else {
        hipLaunchKernelGGL(k_scales, dim3(1), dim3(64), 0, st, (const float *)nullptr, 0,
                           (const float *)nullptr, ns, scales);
    }
    return hipGetLastError();
}

template <int ST>
hhffbp_status image_for_storage(const Plan &P, const void *echoes, const double *pos64,
                                void *image, char *ws, hipStream_t st, hipEvent_t *ev)
{
    const hhffbp_config &c = P.cfg;
    const int n = (int)c.n_pos;
    void *prof = ws + P.ws_prof;
    float4 *posoff = (float4 *)(ws + P.ws_posoff);
    const float *scales = (const float *)(ws + P.ws_scales);
    if (c.mode == HHFFBP_DIRECT_EXACT) {
        if (launch_direct_exact<ST>(P, echoes, pos64, image, st) != hipSuccess) return HHFFBP_E_DEVICE;
        if (ev) (void)hipEventRecord(*ev, st);
        return HHFFBP_OK;
    }
    // Factorised plans: without scaling (c64, bf16) the storage scales are the
    // plan's unit array, and at the plan's own positions the leaf offsets are the
    // plan's too, so such an image starts with the range compression.
    const bool unit = ST != HHFFBP_F16 && P.S > 0;
    hipError_t e = hipSuccess;
    if (unit)
        scales = (const float *)P.dev.unit_scales;
    else if ((e = launch_scales<ST>(P, echoes, ws, st)) != hipSuccess)
        return HHFFBP_E_DEVICE;
    if (P.S > 0) {
        if (pos64 == (const double *)P.dev.pos64) {
            posoff = (float4 *)P.dev.posoff;
        } else {
            if ((e = launch_prep(P, pos64, posoff, st)) != hipSuccess) return HHFFBP_E_DEVICE;
        }
        if (ev) (void)hipEventRecord(*ev++, st);
    }
    if (P.cfg.range_fused) {
        if constexpr (ST == HHFFBP_C64) {
            const int K = (int)(2 * c.n_freq);
            const size_t sh = fused_lds_bytes(K, P.fused_win_max);
            const float inv_dR = (float)(1.0 / P.dR);
            const float kc_turns = (float)(P.kc / kPi);
            if (P.leaf_reach * (P.kc / kPi) < 128.0)
                hipLaunchKernelGGL((k_leaf_bp_fused<false>), dim3(P.n_blocks_fused), dim3(kFusedPoints),
                                   sh, st, (const NodeDev *)P.dev.nodes[P.S],
                                   (const BlockItem *)P.dev.fused_blocks, (const BinWindow *)P.dev.fused_wins,
                                   (const LeafPoint *)P.dev.leafpts, posoff, (const float *)echoes,
                                   (const int32_t *)P.dev.perm, (const float *)P.dev.weights, K,
                                   (const float *)P.dev.B, (int)P.Nr, inv_dR, kc_turns,
                                   (float2 *)(ws + P.ws_vals[P.S]));
            else
                hipLaunchKernelGGL((k_leaf_bp_fused<true>), dim3(P.n_blocks_fused), dim3(kFusedPoints),
                                   sh, st, (const NodeDev *)P.dev.nodes[P.S],
                                   (const BlockItem *)P.dev.fused_blocks, (const BinWindow *)P.dev.fused_wins,
                                   (const LeafPoint *)P.dev.leafpts, posoff, (const float *)echoes,
                                   (const int32_t *)P.dev.perm, (const float *)P.dev.weights, K,
                                   (const float *)P.dev.B, (int)P.Nr, inv_dR, kc_turns,
                                   (float2 *)(ws + P.ws_vals[P.S]));
            if ((e = hipGetLastError()) != hipSuccess) return HHFFBP_E_DEVICE;
            if (ev) (void)hipEventRecord(*ev++, st);
            e = (P.Q == 4) ? dispatch_merges<ST, 4>(P, ws, image, scales, st, ev)
                           : dispatch_merges<ST, 2>(P, ws, image, scales, st, ev);
            return e == hipSuccess ? HHFFBP_OK : HHFFBP_E_DEVICE;
        } else {
            return HHFFBP_E_UNSUPPORTED;
        }
    }
    {
        const int M = n, K = (int)(2 * c.n_freq), N = (int)(2 * P.Nr);
        if (ST == HHFFBP_C64 && P.dev.Bx) {
            constexpr int CT = 3;
            const int NT = P.gemm_nt, rows_per_block = (kBlock / 64) * 64;
            const bool vec = K % 16 == 0 && reinterpret_cast<uintptr_t>(echoes) % 16 == 0;
            const dim3 grid(((M + rows_per_block - 1) / rows_per_block) * ((NT + CT - 1) / CT));
            if (vec && P.gemm_br_spx > 0) {
                const int ncg = (NT + CT - 1) / CT;
                hipLaunchKernelGGL(k_rc_gemm_x6_br, dim3(kXcds * ncg * P.gemm_br_spx), dim3(64 * kBrWaves),
                                   (size_t)(K / 16) * kBrStepBytes, st, (const float *)echoes,
                                   (const int32_t *)P.dev.perm, M, K, (const bf16x8 *)P.dev.Bx, NT, N,
                                   (float *)prof, scales, (const float *)P.dev.weights, (int)P.gemm_br_spx);
            } else if (vec && P.gemm_dma) {
                const dim3 grid_dma(((M + 32 * kX6Waves - 1) / (32 * kX6Waves)) * ((NT + CT - 1) / CT));
                hipLaunchKernelGGL(k_rc_gemm_x6_dma, grid_dma, dim3(64 * kX6Waves), kX6LdsBytes, st,
                                   (const float *)echoes,
                                   (const int32_t *)P.dev.perm, M, K, (const bf16x8 *)P.dev.Bx, NT, N,
                                   (float *)prof, scales, (const float *)P.dev.weights);
            } else {
                auto kern = vec ? k_rc_gemm_x6<CT, true> : k_rc_gemm_x6<CT, false>;
                hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, st, (const float *)echoes,
                                   (const int32_t *)P.dev.perm, M, K, (const bf16x8 *)P.dev.Bx, NT, N,
                                   (float *)prof, scales, (const float *)P.dev.weights);
            }
        } else {
            dim3 grid(((M + 63) / 64) * ((N + 63) / 64));
            hipLaunchKernelGGL((k_rc_gemm<ST, ST>), grid, dim3(kBlock), 0, st,
                               (const typename Store<ST>::R *)echoes, (const int32_t *)P.dev.perm, M, K,
                               (const float *)P.dev.B, N, (typename Store<ST>::R *)prof,
                               (const int32_t *)nullptr, scales, gemm_vec(echoes, K, (const float *)P.dev.B, N),
                               (const float *)P.dev.weights, (const float *)nullptr);
        }
        if ((e = hipGetLastError()) != hipSuccess) return HHFFBP_E_DEVICE;
        if (ev) (void)hipEventRecord(*ev++, st);
    }
    if (P.kernel == HHFFBP_RANGE_LINEAR) {
        e = launch_bp_kernels<HHFFBP_RANGE_LINEAR, 2, ST>(P, pos64, prof, posoff, ws, image, scales, st);
    } else {
        switch (P.W) {
        case 4: e = launch_bp_kernels<HHFFBP_RANGE_ES, 4, ST>(P, pos64, prof, posoff, ws, image, scales, st); break;
        case 5: e = launch_bp_kernels<HHFFBP_RANGE_ES, 5, ST>(P, pos64, prof, posoff, ws, image, scales, st); break;
        case 6: e = launch_bp_kernels<HHFFBP_RANGE_ES, 6, ST>(P, pos64, prof, posoff, ws, image, scales, st); break;
        case 7: e = launch_bp_kernels<HHFFBP_RANGE_ES, 7, ST>(P, pos64, prof, posoff, ws, image, scales, st); break;
        case 8: e = launch_bp_kernels<HHFFBP_RANGE_ES, 8, ST>(P, pos64, prof, posoff, ws, image, scales, st); break;
        default: return HHFFBP_E_UNSUPPORTED;
        }
    }
    if (e != hipSuccess) return HHFFBP_E_DEVICE;
    if (ev) (void)hipEventRecord(*ev++, st);
    if (P.S == 0) return HHFFBP_OK;
    if (P.Q == 4)
        e = dispatch_merges<ST, 4>(P, ws, image, scales, st, ev);
    else
        e = dispatch_merges<ST, 2>(P, ws, image, scales, st, ev);
    return e == hipSuccess ? HHFFBP_OK : HHFFBP_E_DEVICE;
}

}  // namespace

hipError_t launch_prep(const Plan &P, const double *pos64, float4 *posoff, hipStream_t st)
{
    const int n = (int)P.cfg.n_pos;
    hipLaunchKernelGGL(k_prep_positions, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                       pos64, (const double *)P.dev.pos64, P.cfg.position_slack,
                       (const int32_t *)P.dev.perm, (const int32_t *)P.dev.leaf_of_sorted,
                       (const double *)P.dev.leaf_centre, n, posoff);
    return hipGetLastError();
}

hipError_t launch_check_positions(const Plan &P, const double *pos64, int32_t *counts,
                                  hipStream_t st)
{
    const int n = (int)P.cfg.n_pos;
    hipLaunchKernelGGL(k_check_positions, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                       pos64, (const double *)P.dev.pos64, P.cfg.position_slack, n, counts);
    return hipGetLastError();
}

hipError_t prepare_forward(Plan &P)
{
    // the split GEMM's direct-load form needs kX6LdsBytes of LDS a block and its
    // B-resident form K/16 x kBrStepBytes, more than the default: opt in where the
    // device allows it, else the register form
    P.gemm_dma = false;
    P.gemm_br_spx = 0;
    if (P.dev.Bx == nullptr) return hipSuccess;
    int dev = 0, optin = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (optin < kX6LdsBytes) return hipSuccess;
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rc_gemm_x6_dma),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kX6LdsBytes);
    if (e != hipSuccess) return e;
    P.gemm_dma = true;
    const int K = (int)(2 * P.cfg.n_freq), ncg = (P.gemm_nt + 2) / 3;
    const int br_lds = (K / 16) * kBrStepBytes;
    if (K % (16 * kBrDepth) == 0 && br_lds <= optin && ncg > 0) {
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rc_gemm_x6_br),
                                hipFuncAttributeMaxDynamicSharedMemorySize, br_lds);
        if (e != hipSuccess) return e;
        // one block per CU: as many row streams per XCD as its CUs hold column
        // groups.  Taken only where every wave gets two or more 32-row tiles, so
        // that the staging of B and each wave's first loads are amortised (with
        // fewer rows the direct-load form is faster)
        const int spx = std::max(1, ncu / (kXcds * ncg));
        const int64_t groups = (P.cfg.n_pos + 32 * kBrWaves - 1) / (32 * kBrWaves);
        if (groups >= 2 * (int64_t)kXcds * spx) P.gemm_br_spx = spx;
    }
    return hipSuccess;
}

hipError_t launch_rc_gemm(int storage_a, const void *A, const int32_t *a_perm, int M, int K,
                          const float *B, int N, float *C, const int32_t *c_perm, hipStream_t st,
                          const float *a_w, const float *c_w)
{
    dim3 grid(((M + 63) / 64) * ((N + 63) / 64));
    switch (storage_a) {
    case HHFFBP_F16:
        hipLaunchKernelGGL((k_rc_gemm<HHFFBP_F16, HHFFBP_C64>), grid, dim3(kBlock), 0, st,
                           (const uint16_t *)A, a_perm, M, K, B, N, C, c_perm, (const float *)nullptr,
                           gemm_vec(A, K, B, N), a_w, c_w);
        break;
    case HHFFBP_BF16:
        hipLaunchKernelGGL((k_rc_gemm<HHFFBP_BF16, HHFFBP_C64>), grid, dim3(kBlock), 0, st,
                           (const uint16_t *)A, a_perm, M, K, B, N, C, c_perm, (const float *)nullptr,
                           gemm_vec(A, K, B, N), a_w, c_w);
        break;
    default:
        hipLaunchKernelGGL((k_rc_gemm<HHFFBP_C64, HHFFBP_C64>), grid, dim3(kBlock), 0, st,
                           (const float *)A, a_perm, M, K, B, N, C, c_perm, (const float *)nullptr,
                           gemm_vec(A, K, B, N), a_w, c_w);
    }
    return hipGetLastError();
}

std::vector<std::string> Plan::stage_names() const
{
    std::vector<std::string> n;
    if (cfg.mode == HHFFBP_DIRECT_EXACT) {
        n = {"direct_exact"};
    } else if (S == 0) {
        n = {"rc_gemm", "direct_bp"};
    } else if (cfg.range_fused) {
        n = {"prep_positions", "leaf_bp_fused"};
        for (int d = S - 1; d >= F; --d) n.push_back("merge_d" + std::to_string(d));
        n.push_back("final");
    } else {
        n = {"prep_positions", "rc_gemm", "leaf_bp"};
        for (int d = S - 1; d >= F; --d) n.push_back("merge_d" + std::to_string(d));
        n.push_back("final");
    }
    return n;
}

// The device address of this device's `scratch`, looked up once per device
// with that device current and kept; later calls reuse it.
hipError_t noalloc_workspace(int device, char **ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0) return hipErrorInvalidValue;
        addr[device] = p;
    }
    *ptr = static_cast<char *>(addr[device]);
    return hipSuccess;
}

hhffbp_status launch_image(const Plan &P, const void *echoes, const double *positions,
                           void *image, char *ws, hipStream_t st, hipEvent_t *ev)
{
    if (ev) (void)hipEventRecord(*ev++, st);
    const double *pos64 = positions ? positions : (const double *)P.dev.pos64;
    switch (P.cfg.storage) {
    case HHFFBP_F16: return image_for_storage<HHFFBP_F16>(P, echoes, pos64, image, ws, st, ev);
    case HHFFBP_BF16: return image_for_storage<HHFFBP_BF16>(P, echoes, pos64, image, ws, st, ev);
    default: return image_for_storage<HHFFBP_C64>(P, echoes, pos64, image, ws, st, ev);
    }
}

}  // namespace hh
