// gfx950 adjoint kernels of HHFFBPA: echo and antenna-position gradients.
//
// The image is linear in the echoes, f = F M_{S-1} .. M_1 L R s (final stage,
// merges, level-1 BP, range compression).  For an image cotangent g
// (dL/dRe f + j dL/dIm f) the backward pass forms
//   grad_s  = R^H L^H M_1^H .. F^H g
//   grad_p' = Re sum_q conj(G_q) d f'_q / d p'     (G = leaf-level cotangent)
// with the plan frozen: only the level-1 BP depends on the positions.
//
//   k_zero        clear the cotangent arrays (a kernel, never a memset)
//   k_final_adj   F^H: scatter voxel cotangents into the depth-1 grids, or the
//                 root grid when the plan has one (float atomics)
//   k_merge_adj   M_d^H: scatter parent-grid cotangents into the children
//   k_leaf_adj    L^H and the position gradient: one block per kAdjPos positions of a
//                 leaf, looping over all its grid points; the range-profile
//                 cotangents accumulate in LDS and the position gradients in
//                 registers, so each output is written exactly once
//   k_pos_out     float32 partials -> float64 gradients in caller order
// R^H is k_rc_gemm with the conjugate-transposed DFT matrix.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "device_common.hpp"
#include "hhffbp_internal.hpp"

namespace hh {
namespace {
using namespace dev;

constexpr size_t kLdsLimit = 64 * 1024;  // dynamic LDS available without opting in

__global__ __launch_bounds__(kBlock) void k_zero(float4 *__restrict__ p, int64_t n4)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * kBlock)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Transpose of the separable interpolation: grad[tap] += w(tap) * (gre + j gim),
// taps outside the child's pencils skipped.
template <int T, int K>
__device__ __forceinline__ void scatter_child(const NodeDev &c, const ColEntry *__restrict__ cols,
                                              float2 *__restrict__ grad, const ChildCoord &g,
                                              const InterpPoly &ip, float gre, float gim)
{
    float wu[T], wv[T], wn[T];
    interp_weights<T, K>(ip, g, wu, wv, wn);
#pragma unroll
    for (int a = 0; a < T; ++a) {
        const int ci = g.bi + a - T / 2 + 1 - c.i0;
        if ((unsigned)ci >= (unsigned)c.ni) continue;
#pragma unroll
        for (int b = 0; b < T; ++b) {
            const int cj = g.bj + b - T / 2 + 1 - c.j0;
            if ((unsigned)cj >= (unsigned)c.nj) continue;
            const ColEntry e = cols[c.col_base + ci * c.nj + cj];
            float2 *colg = grad + c.val_base + e.off - e.lo;
            const float wab = wu[a] * wv[b];
#pragma unroll
            for (int k = 0; k < T; ++k) {
                const int l = g.bl + k - T / 2 + 1;
                if (l >= e.lo && l <= e.hi) {
                    const float w = wab * wn[k];
                    unsafeAtomicAdd(&colg[l].x, w * gre);
                    unsafeAtomicAdd(&colg[l].y, w * gim);
                }
            }
        }
    }
}

// (gre + j gim) = v exp(-j 2 pi turns), turns in [-1/2, 1/2]
__device__ __forceinline__ void rotate_back(float2 v, float turns, float &gre, float &gim)
{
    const float sn = sin_turns(turns), cs = cos_turns(turns);
    gre = v.x * cs + v.y * sn;
    gim = v.y * cs - v.x * sn;
}

// The stencil base and fractions of a plan-time record (InterpIdx, InterpGeo)
// as the child coordinates the scatter takes.
template <int T>
__device__ __forceinline__ ChildCoord record_coord(const NodeDev &c, InterpIdx ix, const InterpGeo &g)
{
    ChildCoord cc;
    cc.bi = (int)(ix.cij & 0xffffu) + c.i0 + T / 2 - 1;
    cc.bj = (int)(ix.cij >> 16) + c.j0 + T / 2 - 1;
    cc.bl = ix.l0 + T / 2 - 1;
    cc.fu = g.fu;
    cc.fv = g.fv;
    cc.fn = g.fn;
    return cc;
}

// Nearest integer of x, ties to even.  Rounding ties up (floor(x + 1/2), one
// instruction) would bias the fixed-point sums: above 2^22 a float32 is often
// a half-integer, and those ties would all round the same way.
__device__ __forceinline__ int cvt_round_i32(float x) { return (int)rintf(x); }

// --- block-aggregated scatter --------------------------------------------
// The stencils of one block's points cover a small box of the child's (i, j, l)
// index space.  The block accumulates its contributions there in LDS (int32
// fixed point: float LDS atomics are serialised on gfx950, integer ones are not)
// and then adds each non-zero box entry to the child's grid with one float
// atomic.  The fixed-point scale 2^31 / (1.3 sum |g|) over the block cannot
// overflow (a Lagrange weight product is below 1.3 and each point adds to a box
// entry at most once) and resolves every contribution to ~1.5e-7 of itself.
constexpr int kBoxCap = 4096;

struct BoxShared {
    int mn[3], mx[3];
    float gsum;
    float gpart[kBlock / 64];
    int ipart[kBlock / 64][6];
    // one 64-bit entry per box point: real part in the high half, imaginary in
    // the low half (see block_scatter_child)
    unsigned long long box[kBoxCap];
};

__device__ __forceinline__ int wave_min_i(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_sum_f(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Every lane of the block calls this (inactive lanes with active = false).
template <int T, int K, int VSHIFT>
__device__ void block_scatter_child(BoxShared &sh, bool active, const NodeDev &c,
                                    const ColEntry *__restrict__ cols, float2 *__restrict__ grad,
                                    const ChildCoord &g, const InterpPoly &ip, float gre,
                                    float gim)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int lo = -T / 2 + 1;
    int v6[6] = {active ? g.bi : INT_MAX, active ? g.bj : INT_MAX, active ? g.bl : INT_MAX,
                 active ? g.bi : INT_MIN, active ? g.bj : INT_MIN, active ? g.bl : INT_MIN};
    float ga = active ? fabsf(gre) + fabsf(gim) : 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) v6[a] = wave_min_i(v6[a]);
#pragma unroll
    for (int a = 3; a < 6; ++a) v6[a] = wave_max_i(v6[a]);
    ga = wave_sum_f(ga);
    if (lane == 0) {
#pragma unroll
        for (int a = 0; a < 6; ++a) sh.ipart[wave][a] = v6[a];
        sh.gpart[wave] = ga;
    }
    __syncthreads();
    if (tid == 0) {
        float gs = 0.0f;
        for (int a = 0; a < 3; ++a) {
            int m = INT_MAX, M = INT_MIN;
            for (int w = 0; w < kBlock / 64; ++w) {
                m = min(m, sh.ipart[w][a]);
                M = max(M, sh.ipart[w][a + 3]);
            }
            sh.mn[a] = m;
            sh.mx[a] = M;
        }
        for (int w = 0; w < kBlock / 64; ++w) gs += sh.gpart[w];
        sh.gsum = gs;
    }
    __syncthreads();
    if (sh.mn[0] > sh.mx[0] || !(sh.gsum > 0.0f)) {  // nothing to scatter
        __syncthreads();
        return;
    }
    const int o0 = sh.mn[0] + lo, o1 = sh.mn[1] + lo, o2 = sh.mn[2] + lo;
    const int B0 = sh.mx[0] - sh.mn[0] + T, B1 = sh.mx[1] - sh.mn[1] + T, B2 = sh.mx[2] - sh.mn[2] + T;
    const long long nbox = (long long)B0 * B1 * B2;
    if (nbox > kBoxCap) {
        // box too large for LDS: direct global atomics
        if (active) scatter_child<T, K>(c, cols, grad, g, ip, gre, gim);
        __syncthreads();
        return;
    }
    const int nb = (int)nbox;
    for (int t = tid; t < nb; t += kBlock) sh.box[t] = 0ull;
    const float q = 1651910204.0f / sh.gsum;  // 2^31 / 1.3
    __syncthreads();
    if (active) {
        float wu[T], wv[T], wn[T];
        interp_weights<T, K>(ip, g, wu, wv, wn);
        const float qre = gre * q, qim = gim * q;
        const int bi = g.bi + lo - o0, bj = g.bj + lo - o1, bl = g.bl + lo - o2;
        // Neighbouring points often share a stencil base; taken in the same tap
        // order their atomics would hit one LDS address per instruction.  Each
        // lane rotates its n tap order by its lowest bits and its v tap order by
        // the bits above the brick's fastest axis (VSHIFT = log2 of its length:
        // l and j of a merge brick, z and y of a voxel brick), so such lanes add
        // to different entries at once; integer sums do not depend on the order.
        const int rn = lane % T, rv = (lane >> VSHIFT) % T;
        float wvr[T], wnr[T];
        int ov[T], on[T];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int iv = (t + rv) % T, in = (t + rn) % T;
            float x = wv[0], y = wn[0];
#pragma unroll
            for (int u = 1; u < T; ++u) {
                x = (iv == u) ? wv[u] : x;
                y = (in == u) ? wn[u] : y;
            }
            wvr[t] = x;
            wnr[t] = y;
            ov[t] = iv;
            on[t] = in;
        }
        // the n weights times the scaled cotangent, once per point
        float nre[T], nim[T];
#pragma unroll
        for (int k = 0; k < T; ++k) {
            nre[k] = wnr[k] * qre;
            nim[k] = wnr[k] * qim;
        }
#pragma unroll
        for (int a = 0; a < T; ++a)
#pragma unroll
            for (int b = 0; b < T; ++b) {
                const float wab = wu[a] * wvr[b];
                unsigned long long *rowp = sh.box + ((bi + a) * B1 + (bj + ov[b])) * B2 + bl;
#pragma unroll
                for (int k = 0; k < T; ++k) {
                    // re 2^32 + im in one 64-bit add: both sums stay within int32
                    // (the scale q), so the low half is the imaginary sum exactly
                    // and the carries it leaves make the high half the real sum.
                    // The word is formed in 32-bit halves: the high half takes
                    // the sign of im (two's complement of the 64-bit sum).
                    const int ar = cvt_round_i32(wab * nre[k]), ai = cvt_round_i32(wab * nim[k]);
                    const uint32_t hi = (uint32_t)ar + (uint32_t)(ai >> 31);
                    atomicAdd(rowp + on[k], ((unsigned long long)hi << 32) | (uint32_t)ai);
                }
            }
    }
    __syncthreads();
    const float inv = 1.0f / q;
    for (int t = tid; t < nb; t += kBlock) {
        const long long x = (long long)sh.box[t];
        if (x == 0) continue;
        const int vi = (int)(unsigned)(unsigned long long)x;
        const int vr = (int)((x - (long long)vi) >> 32);
        const int l = o2 + t % B2;
        const int j = o1 + (t / B2) % B1;
        const int i = o0 + t / (B2 * B1);
        const int ci = i - c.i0, cj = j - c.j0;
        if ((unsigned)ci >= (unsigned)c.ni || (unsigned)cj >= (unsigned)c.nj) continue;
        const ColEntry e = cols[c.col_base + ci * c.nj + cj];
        if (l < e.lo || l > e.hi) continue;  // not a point of the child's grid
        float2 *dst = grad + c.val_base + e.off + (l - e.lo);
        unsafeAtomicAdd(&dst->x, (float)vr * inv);
        unsafeAtomicAdd(&dst->y, (float)vi * inv);
    }
    __syncthreads();
}

// F^H: a block per brick of the final stage (kBrickX x kBrickY x kBrickZ voxels, numbered and
// laid out as k_final's); each voxel's cotangent is rotated by -Phi_child and
// scattered into the child's grid through the block's box, with the stencil,
// fractions and phase of the forward's plan-time record of that (voxel, child).
template <int T, int K>
__global__ __launch_bounds__(kBlock) void k_final_adj(const NodeDev *__restrict__ children,
                                                      int nchild, const ColEntry *__restrict__ ccols,
                                                      float2 *__restrict__ cgrad,
                                                      const InterpIdx *__restrict__ ridx,
                                                      const InterpGeo *__restrict__ rgeo,
                                                      const InterpPoly ip, int nx, int ny, int nz,
                                                      const float2 *__restrict__ gimg)
{
    __shared__ BoxShared sh;
    const int bz = (nz + kBrickZ - 1) / kBrickZ, by = (ny + kBrickY - 1) / kBrickY;
    const int brick = (int)blockIdx.x;
    const int kx = brick / (by * bz), ky = (brick / bz) % by, kz = brick % bz;
    const int t = (int)threadIdx.x;
    const int ix = kx * kBrickX + t / (kBrickY * kBrickZ), iy = ky * kBrickY + (t / kBrickZ) % kBrickY,
              iz = kz * kBrickZ + t % kBrickZ;
    bool active = ix < nx && iy < ny && iz < nz;
    float2 g = make_float2(0.f, 0.f);
    if (active) g = gimg[((int64_t)ix * ny + iy) * nz + iz];
    active = active && (g.x != 0.0f || g.y != 0.0f);
    for (int c = 0; c < nchild; ++c) {
        const NodeDev ch = children[c];
        const size_t r = ((size_t)brick * nchild + c) * kBlock + t;
        // both records at once (every slot has them), so that the geometry's
        // load does not wait for the index's
        const InterpIdx rx = ridx[r];
        const InterpGeo rg = rgeo[r];
        const bool on = active && rx.cij != kNoPair;
        ChildCoord cc{};
        float gre = 0.0f, gim = 0.0f;
        if (on) {
            cc = record_coord<T>(ch, rx, rg);
            rotate_back(g, rg.turns, gre, gim);
        }
        block_scatter_child<T, K, __builtin_ctz(kBrickZ)>(sh, on, ch, ccols, cgrad, cc, ip, gre, gim);
    }
}

// M_d^H on a merge brick (4 x 4 columns x 16 steps of a parent grid; lane t:
// l = t mod 16 fastest, then j, then i): each point's cotangent is rotated by
// -(Phi_child - Phi_parent) and scattered into the child's grid through the
// block's box.  The stencil, fractions and phase are the forward's plan-time
// record of that (point, child): with s the point's lane slot in the node's
// merge order (rank), block fwd_block0 + s / (256 / Q) of the forward merge,
// wave (s mod (256 / Q)) / 64 * Q + c, lane s mod 64.  Bricks
// keep the box, and so the number of global atomics per point, smaller than
// runs of points along the pencils would.
template <int T, int K>
__global__ __launch_bounds__(kBlock) void k_merge_adj(const NodeDev *__restrict__ parents,
                                                      const ColEntry *__restrict__ pcols,
                                                      const MergeBrick *__restrict__ bricks,
                                                      const float2 *__restrict__ pgrad,
                                                      const NodeDev *__restrict__ children,
                                                      const ColEntry *__restrict__ ccols,
                                                      float2 *__restrict__ cgrad,
                                                      const InterpIdx *__restrict__ ridx,
                                                      const InterpGeo *__restrict__ rgeo,
                                                      const int32_t *__restrict__ rank, int Q,
                                                      const InterpPoly ip)
{
    __shared__ BoxShared sh;
    const MergeBrick mb = bricks[blockIdx.x];
    const NodeDev *ndp = parents + mb.node;
    const int ni = ndp->ni, nj = ndp->nj, i0 = ndp->i0, j0 = ndp->j0, col_base = ndp->col_base;
    const int val_base = ndp->val_base, nchild = ndp->nchild, fb0 = ndp->fwd_block0;
    const int t = (int)threadIdx.x;
    const int ci = mb.i + t / (kMBrickJ * kMBrickL) - i0, cj = mb.j + (t / kMBrickL) % kMBrickJ - j0;
    const int l = mb.l + t % kMBrickL;
    bool active = false;
    int p = 0;
    if ((unsigned)ci < (unsigned)ni && (unsigned)cj < (unsigned)nj) {
        const ColEntry pe = pcols[col_base + ci * nj + cj];
        if (l >= pe.lo && l <= pe.hi) {
            active = true;
            p = pe.off + (l - pe.lo);
        }
    }
    float2 g = make_float2(0.f, 0.f);
    if (active) g = pgrad[val_base + p];
    active = active && (g.x != 0.0f || g.y != 0.0f);
    // the forward merge's lane slot of this point, and its records
    const int s = active ? rank[val_base + p] : 0;
    const int pb = kBlock / Q;
    const size_t rbase = (size_t)(fb0 + s / pb) * kBlock + (size_t)((s % pb) / 64 * Q) * 64 + s % 64;
    // the records of child c + 1 are loaded before child c's scatter (whose
    // barriers would otherwise hold them back); every slot has both records
    InterpIdx rx_next = ridx[rbase];
    InterpGeo rg_next = rgeo[rbase];
    for (int c = 0; c < nchild; ++c) {
        const NodeDev ch = children[ndp->child[c]];
        const InterpIdx rx = rx_next;
        const InterpGeo rg = rg_next;
        if (c + 1 < nchild) {
            rx_next = ridx[rbase + (size_t)(c + 1) * 64];
            rg_next = rgeo[rbase + (size_t)(c + 1) * 64];
        }
        const bool on = active && rx.cij != kNoPair;  // absent parent points hold nothing
        ChildCoord cc{};
        float gre = 0.0f, gim = 0.0f;
        if (on) {
            cc = record_coord<T>(ch, rx, rg);
            rotate_back(g, rg.turns, gre, gim);
        }
        block_scatter_child<T, K, __builtin_ctz(kMBrickL)>(sh, on, ch, ccols, cgrad, cc, ip, gre, gim);
    }
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Largest |Re|, |Im| of each leaf's grid cotangents: the fixed-point scale of the
// leaf's range-profile cotangents.  One block per leaf.
__global__ __launch_bounds__(kBlock) void k_leaf_gmax(const NodeDev *__restrict__ leaves,
                                                      const float2 *__restrict__ gleaf,
                                                      float *__restrict__ gmax)
{
    __shared__ float s_m[kBlock / 64];
    const NodeDev nd = leaves[blockIdx.x];
    float m = 0.0f;
    for (int p = threadIdx.x; p < nd.npts; p += kBlock) {
        const float2 g = gleaf[nd.val_base + p];
        m = fmaxf(m, fmaxf(fabsf(g.x), fabsf(g.y)));
    }
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = 0.0f;
        for (int w = 0; w < kBlock / 64; ++w) r = fmaxf(r, s_m[w]);
        gmax[blockIdx.x] = r;
    }
}

// L^H and the position gradient for the kAdjPos positions [p0, p0 + n) of one leaf.
// For each (grid point q, position i), with gi = conj(pre_q e^{j 2 kc dR}) G_q:
//   profile cotangent  gprof_i[r_w] += phi_w gi
//   position gradient  grad p'_i  += Re{conj(gi) sum_w phi_w dprof_i[r_w]} * (-(q - p'_i)/|q - p'_i|)
// where dprof holds the range profiles of the echoes weighted by j 2 k_f (the
// range derivative of the compressed data).
template <int KERNEL, int W, bool WANT_S, bool WANT_P, bool RED>
__global__ __launch_bounds__(kBlock) void k_leaf_adj(
    const NodeDev *__restrict__ leaves, const BlockItem *__restrict__ blocks,
    const LeafPoint *__restrict__ pts, const float4 *__restrict__ posoff,
    const float2 *__restrict__ dprof, int Nr, float inv_dR, float beta_log2e, float kc_turns,
    const float2 *__restrict__ gleaf, const float *__restrict__ gmax, float2 *__restrict__ gprof,
    float4 *__restrict__ gpos)
{
    extern __shared__ unsigned char smem[];
    __shared__ float4 s_pos[kAdjPos];
    __shared__ float s_red[kBlock / 64][kAdjPos][3];
    // Range-profile cotangents accumulate in fixed point: float LDS atomics are
    // serialised on gfx950 while 64-bit integer ones run at full rate.  Every
    // contribution (|.| <= max |G| of the leaf) is rounded to an int32 at scale
    // 2^30 / max |G| and summed exactly in int64; real and imaginary parts are
    // separate arrays so that neighbouring bins fall in different banks.
    float2 *s_dprof = reinterpret_cast<float2 *>(smem);
    const int gs = Nr + 1;
    unsigned long long *s_gre = reinterpret_cast<unsigned long long *>(
        smem + (WANT_P ? (size_t)kAdjPos * Nr * sizeof(float2) : 0));
    unsigned long long *s_gim = s_gre + (size_t)kAdjPos * gs;
    const BlockItem blk = blocks[blockIdx.x];
    const NodeDev nd = leaves[blk.node];
    const int p0 = blk.start;
    const int n = min(kAdjPos, nd.pos_end - p0);
    const int tid = threadIdx.x;
    if (tid < kAdjPos) s_pos[tid] = (tid < n) ? posoff[p0 + tid] : make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (WANT_P) {
        const float2 *src = dprof + (size_t)p0 * Nr;
        for (int t = tid; t < kAdjPos * Nr; t += kBlock)
            s_dprof[t] = (t < n * Nr) ? src[t] : make_float2(0.f, 0.f);
    }
    float qscale = 0.0f;
    if constexpr (WANT_S) {
        for (int t = tid; t < kAdjPos * gs; t += kBlock) {
            s_gre[t] = 0ull;
            s_gim[t] = 0ull;
        }
        const float gm = gmax[blk.node];
        qscale = gm > 0.0f ? 1073741824.0f / gm : 0.0f;
    }
    __syncthreads();
    float ap[kAdjPos][3];
#pragma unroll
    for (int i = 0; i < kAdjPos; ++i) ap[i][0] = ap[i][1] = ap[i][2] = 0.0f;
    for (int pt0 = 0; pt0 < nd.npts; pt0 += kBlock) {
        const int p = pt0 + tid;
        if (p >= nd.npts) continue;
        const LeafPoint q = pts[nd.val_base + p];
        const float2 G = gleaf[nd.val_base + p];
        // f' = pre * sum  ->  cotangent of the sum is conj(pre) G
        const float gcre = q.pre_re * G.x + q.pre_im * G.y;
        const float gcim = q.pre_re * G.y - q.pre_im * G.x;
        if (gcre == 0.0f && gcim == 0.0f) continue;
        const float Rc2 = q.dx * q.dx + q.dy * q.dy + q.dz * q.dz;
        const float Rc = fast_sqrt(Rc2);
        const float frac_w = q.frac - 0.5f * W;
        const int bin1 = q.bin + 1;
        // the taps stay inside the staged profiles, r in [0, Nr - W]: the range
        // grid covers every distance from a leaf point to its positions' slack box
        // with (W / 2 + 2) bins to spare, and positions are clamped to that box
        const float m2x = -2.0f * q.dx, m2y = -2.0f * q.dy, m2z = -2.0f * q.dz;
#pragma unroll
        for (int i = 0; i < kAdjPos; ++i) {
            if (i < n) {  // predicated, so every ap[i] index stays a constant
                const float4 d = s_pos[i];
                const float ex = q.dx - d.x, ey = q.dy - d.y, ez = q.dz - d.z;
                // |q - p'|^2 = |q - c|^2 + num (as in the forward level-1 BP)
                const float num = fmaf(m2x, d.x, fmaf(m2y, d.y, fmaf(m2z, d.z, d.w)));
                const float R = fast_sqrt(num + Rc2);
                const float dR = num * fast_rcp(R + Rc);
                const float tau = fmaf(dR, inv_dR, frac_w);
                const int r = bin1 + floor_int(tau);
                const float x = __builtin_amdgcn_fractf(tau);
                float w[W];
                range_weights<KERNEL, W>(x, beta_log2e, w);
                float ph = dR * kc_turns;
                if constexpr (RED) ph -= rintf(ph);
                const float sn = sin_turns(ph), cs = cos_turns(ph);
                const float gire = gcre * cs + gcim * sn;
                const float giim = gcim * cs - gcre * sn;
                if constexpr (WANT_S) {
                    unsigned long long *rre = s_gre + i * gs + r;
                    unsigned long long *rim = s_gim + i * gs + r;
                    const float qre = gire * qscale, qim = giim * qscale;
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        const long long a = (long long)(int)rintf(w[k] * qre);
                        const long long b = (long long)(int)rintf(w[k] * qim);
                        atomicAdd(&rre[k], (unsigned long long)a);
                        atomicAdd(&rim[k], (unsigned long long)b);
                    }
                }
                if constexpr (WANT_P) {
                    const float2 *pr = s_dprof + i * Nr + r;
                    float dre = 0.0f, dim = 0.0f;
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        const float2 v = pr[k];
                        dre = fmaf(w[k], v.x, dre);
                        dim = fmaf(w[k], v.y, dim);
                    }
                    const float val = gire * dre + giim * dim;
                    const float sc = -val * fast_rcp(R);
                    ap[i][0] = fmaf(sc, ex, ap[i][0]);
                    ap[i][1] = fmaf(sc, ey, ap[i][1]);
                    ap[i][2] = fmaf(sc, ez, ap[i][2]);
                }
            }
        }
    }
    if constexpr (WANT_P) {
        const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
        for (int i = 0; i < kAdjPos; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float v = wave_sum(ap[i][c]);
                if (lane == 0) s_red[wave][i][c] = v;
            }
    }
    __syncthreads();
    if constexpr (WANT_P) {
        if (tid < n * 3) {
            const int i = tid / 3, c = tid % 3;
            float v = 0.0f;
#pragma unroll
            for (int wv = 0; wv < kBlock / 64; ++wv) v += s_red[wv][i][c];
            reinterpret_cast<float *>(gpos + p0 + i)[c] = v;
        }
    }
    if constexpr (WANT_S) {
        float2 *dst = gprof + (size_t)p0 * Nr;
        const double inv = qscale > 0.0f ? 1.0 / (double)qscale : 0.0;
        for (int t = tid; t < n * Nr; t += kBlock) {
            const int o = (t / Nr) * gs + (t % Nr);
            dst[t] = make_float2((float)((double)(long long)s_gre[o] * inv),
                                 (float)((double)(long long)s_gim[o] * inv));
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_pos_out(const float4 *__restrict__ gpos,
                                                    const int32_t *__restrict__ perm, int n,
                                                    double *__restrict__ out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float4 g = gpos[i];
    const int m = perm[i];
    out[3 * m] = (double)g.x;
    out[3 * m + 1] = (double)g.y;
    out[3 * m + 2] = (double)g.z;
}

template <bool S_, bool P_>
size_t leaf_adj_lds(const Plan &P)
{
    return (P_ ? (size_t)kAdjPos * P.Nr * sizeof(float2) : 0) +
           (S_ ? (size_t)kAdjPos * (P.Nr + 1) * 2 * sizeof(unsigned long long) : 0);
}

template <int KERNEL, int W, bool S_, bool P_, bool RED>
hipError_t launch_leaf_adj(const Plan &P, const float4 *posoff, const float2 *dprof,
                           const float2 *gleaf, const float *gmax, float2 *gprof, float4 *gpos,
                           hipStream_t st)
{
    const size_t sh = leaf_adj_lds<S_, P_>(P);
    // beyond the default dynamic LDS the plan has opted the kernel in, up to the
    // device's per-block limit (prepare_backward)
    if (sh > P.adj_lds_max) return hipErrorInvalidConfiguration;  // caller maps to UNSUPPORTED
    hipLaunchKernelGGL((k_leaf_adj<KERNEL, W, S_, P_, RED>), dim3(P.n_blocks_adj), dim3(kBlock), sh, st,
                       (const NodeDev *)P.dev.nodes[P.S], (const BlockItem *)P.dev.adj_blocks,
                       (const LeafPoint *)P.dev.leafpts, posoff, dprof, (int)P.Nr,
                       (float)(1.0 / P.dR), (float)(P.beta * 1.4426950408889634),
                       (float)(P.kc / kPi), gleaf, gmax, gprof, gpos);
    return hipGetLastError();
}

template <int KERNEL, int W, bool S_, bool P_, bool RED>
hipError_t leaf_adj_optin_one(const Plan &P)
{
    const size_t sh = leaf_adj_lds<S_, P_>(P);
    if (sh <= kLdsLimit || sh > P.adj_lds_max) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_leaf_adj<KERNEL, W, S_, P_, RED>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
}

template <int KERNEL, int W>
hipError_t leaf_adj_optin(const Plan &P)
{
    hipError_t e = hipSuccess;
    if (P.leaf_reach * (P.kc / kPi) < 128.0) {
        if (e == hipSuccess) e = leaf_adj_optin_one<KERNEL, W, true, true, false>(P);
        if (e == hipSuccess) e = leaf_adj_optin_one<KERNEL, W, true, false, false>(P);
        if (e == hipSuccess) e = leaf_adj_optin_one<KERNEL, W, false, true, false>(P);
    } else {
        if (e == hipSuccess) e = leaf_adj_optin_one<KERNEL, W, true, true, true>(P);
        if (e == hipSuccess) e = leaf_adj_optin_one<KERNEL, W, true, false, true>(P);
        if (e == hipSuccess) e = leaf_adj_optin_one<KERNEL, W, false, true, true>(P);
    }
    return e;
}

template <int KERNEL, int W>
hipError_t leaf_adj_dispatch(const Plan &P, bool want_s, bool want_p, const float4 *posoff,
                             const float2 *dprof, const float2 *gleaf, const float *gmax,
                             float2 *gprof, float4 *gpos, hipStream_t st)
{
    // the carrier's argument needs no reduction below 128 turns, as in the forward
    if (P.leaf_reach * (P.kc / kPi) < 128.0) {
        if (want_s && want_p)
            return launch_leaf_adj<KERNEL, W, true, true, false>(P, posoff, dprof, gleaf, gmax, gprof, gpos, st);
        if (want_s)
            return launch_leaf_adj<KERNEL, W, true, false, false>(P, posoff, dprof, gleaf, gmax, gprof, gpos, st);
        return launch_leaf_adj<KERNEL, W, false, true, false>(P, posoff, dprof, gleaf, gmax, gprof, gpos, st);
    }
    if (want_s && want_p)
        return launch_leaf_adj<KERNEL, W, true, true, true>(P, posoff, dprof, gleaf, gmax, gprof, gpos, st);
    if (want_s)
        return launch_leaf_adj<KERNEL, W, true, false, true>(P, posoff, dprof, gleaf, gmax, gprof, gpos, st);
    return launch_leaf_adj<KERNEL, W, false, true, true>(P, posoff, dprof, gleaf, gmax, gprof, gpos, st);
}

template <int T, int K>
hipError_t launch_scatters(const Plan &P, const void *grad_image, char *ws, hipStream_t st)
{
    const hhffbp_config &c = P.cfg;
    const int nx = (int)c.grid_dims[0], ny = (int)c.grid_dims[1], nz = (int)c.grid_dims[2];
    hipLaunchKernelGGL((k_final_adj<T, K>), dim3(P.n_bricks), dim3(kBlock), 0, st,
                       (const NodeDev *)P.dev.nodes[P.F], (int)P.compact_to_tree[P.F].size(),
                       (const ColEntry *)P.dev.cols[P.F], (float2 *)(ws + P.ws_gvals[P.F]),
                       (const InterpIdx *)P.dev.final_idx, (const InterpGeo *)P.dev.final_geo,
                       P.ipoly_for(P.F), nx, ny, nz, (const float2 *)grad_image);
    hipError_t e = hipGetLastError();
    for (int d = P.F; d < P.S && e == hipSuccess; ++d) {
        const int64_t nb = (int64_t)P.merge_bricks[d].size();
        if (nb == 0) continue;
        hipLaunchKernelGGL((k_merge_adj<T, K>), dim3(nb), dim3(kBlock), 0, st,
                           (const NodeDev *)P.dev.nodes[d], (const ColEntry *)P.dev.cols[d],
                           (const MergeBrick *)P.dev.merge_bricks[d],
                           (const float2 *)(ws + P.ws_gvals[d]),
                           (const NodeDev *)P.dev.nodes[d + 1], (const ColEntry *)P.dev.cols[d + 1],
                           (float2 *)(ws + P.ws_gvals[d + 1]), (const InterpIdx *)P.dev.merge_idx[d],
                           (const InterpGeo *)P.dev.merge_geo[d],
                           (const int32_t *)P.dev.merge_rank[d], P.Q, P.ipoly_for(d + 1));
        e = hipGetLastError();
    }
    return e;
}

}  // namespace

hipError_t prepare_backward(Plan &P)
{
    P.adj_lds_max = kLdsLimit;
    if (P.S < 1 || P.cfg.range_fused) return hipSuccess;
    int dev = 0, optin = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev);
    if (e != hipSuccess) return e;
    P.adj_lds_max = std::max(kLdsLimit, (size_t)optin);
    if (P.kernel == HHFFBP_RANGE_LINEAR) return leaf_adj_optin<HHFFBP_RANGE_LINEAR, 2>(P);
    switch (P.W) {
    case 4: return leaf_adj_optin<HHFFBP_RANGE_ES, 4>(P);
    case 5: return leaf_adj_optin<HHFFBP_RANGE_ES, 5>(P);
    case 6: return leaf_adj_optin<HHFFBP_RANGE_ES, 6>(P);
    case 7: return leaf_adj_optin<HHFFBP_RANGE_ES, 7>(P);
    case 8: return leaf_adj_optin<HHFFBP_RANGE_ES, 8>(P);
    default: return hipSuccess;
    }
}

hhffbp_status launch_backward(const Plan &P, const void *echoes, const double *positions,
                              const void *grad_image, void *grad_echoes, double *grad_positions,
                              char *ws, hipStream_t st)
{
    const hhffbp_config &c = P.cfg;
    const int n = (int)c.n_pos;
    const bool want_s = grad_echoes != nullptr, want_p = grad_positions != nullptr;
    const double *pos64 = positions ? positions : (const double *)P.dev.pos64;
    float2 *dprof = (float2 *)(ws + P.ws_prof);
    float4 *posoff = (float4 *)(ws + P.ws_posoff);
    float2 *gprof = (float2 *)(ws + P.ws_gprof);
    float4 *gpos = (float4 *)(ws + P.ws_gpos);
    hipError_t e;
    // positions relative to their leaf centres
    if ((e = launch_prep(P, pos64, posoff, st)) != hipSuccess) return HHFFBP_E_DEVICE;
    // range-derivative profiles (only the position gradient needs them)
    if (want_p) {
        e = launch_rc_gemm(c.storage, echoes, (const int32_t *)P.dev.perm, n,
                           (int)(2 * c.n_freq), (const float *)P.dev.Bd, (int)(2 * P.Nr),
                           (float *)dprof, nullptr, st, (const float *)P.dev.weights, nullptr);
        if (e != hipSuccess) return HHFFBP_E_DEVICE;
    }
    // clear every grid cotangent: depths F..S are contiguous and end at the
    // 256-byte aligned start of gprof (a point count may be odd, so the float4
    // clear runs to that aligned end rather than to the last point)
    {
        const size_t b0 = P.ws_gvals[P.F];
        const size_t b1 = P.ws_gprof;
        const int64_t n4 = (int64_t)((b1 - b0) / sizeof(float4));
        hipLaunchKernelGGL(k_zero, dim3(1024), dim3(kBlock), 0, st, (float4 *)(ws + b0), n4);
        if ((e = hipGetLastError()) != hipSuccess) return HHFFBP_E_DEVICE;
    }
    if (P.ipoly.kind == HHFFBP_INTERP_BANDLIMITED)
        e = (P.T == 4) ? launch_scatters<4, HHFFBP_INTERP_BANDLIMITED>(P, grad_image, ws, st)
                       : launch_scatters<6, HHFFBP_INTERP_BANDLIMITED>(P, grad_image, ws, st);
    else
        e = (P.T == 4) ? launch_scatters<4, HHFFBP_INTERP_LAGRANGE>(P, grad_image, ws, st)
                       : launch_scatters<6, HHFFBP_INTERP_LAGRANGE>(P, grad_image, ws, st);
    if (e != hipSuccess) return HHFFBP_E_DEVICE;
    const float2 *gleaf = (const float2 *)(ws + P.ws_gvals[P.S]);
    float *gmax = (float *)(ws + P.ws_gmax);
    if (want_s) {
        hipLaunchKernelGGL(k_leaf_gmax, dim3((unsigned)P.compact_to_tree[P.S].size()), dim3(kBlock), 0,
                           st, (const NodeDev *)P.dev.nodes[P.S], gleaf, gmax);
        if ((e = hipGetLastError()) != hipSuccess) return HHFFBP_E_DEVICE;
    }
    if (P.kernel == HHFFBP_RANGE_LINEAR) {
        e = leaf_adj_dispatch<HHFFBP_RANGE_LINEAR, 2>(P, want_s, want_p, posoff, dprof, gleaf, gmax,
                                                      gprof, gpos, st);
    } else {
        switch (P.W) {
        case 4: e = leaf_adj_dispatch<HHFFBP_RANGE_ES, 4>(P, want_s, want_p, posoff, dprof, gleaf, gmax, gprof, gpos, st); break;
        case 5: e = leaf_adj_dispatch<HHFFBP_RANGE_ES, 5>(P, want_s, want_p, posoff, dprof, gleaf, gmax, gprof, gpos, st); break;
        case 6: e = leaf_adj_dispatch<HHFFBP_RANGE_ES, 6>(P, want_s, want_p, posoff, dprof, gleaf, gmax, gprof, gpos, st); break;
        case 7: e = leaf_adj_dispatch<HHFFBP_RANGE_ES, 7>(P, want_s, want_p, posoff, dprof, gleaf, gmax, gprof, gpos, st); break;
        case 8: e = leaf_adj_dispatch<HHFFBP_RANGE_ES, 8>(P, want_s, want_p, posoff, dprof, gleaf, gmax, gprof, gpos, st); break;
        default: return HHFFBP_E_UNSUPPORTED;
        }
    }
    if (e == hipErrorInvalidConfiguration) return HHFFBP_E_UNSUPPORTED;  // profile window too long
    if (e != hipSuccess) return HHFFBP_E_DEVICE;
    if (want_s) {
        // grad_s = gprof conj(W)^T, rows back to the caller's position order
        e = launch_rc_gemm(HHFFBP_C64, gprof, nullptr, n, (int)(2 * P.Nr),
                           (const float *)P.dev.Badj, (int)(2 * c.n_freq), (float *)grad_echoes,
                           (const int32_t *)P.dev.perm, st, nullptr, (const float *)P.dev.weights);
        if (e != hipSuccess) return HHFFBP_E_DEVICE;
    }
    if (want_p) {
        hipLaunchKernelGGL(k_pos_out, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, gpos,
                           (const int32_t *)P.dev.perm, n, grad_positions);
        if ((e = hipGetLastError()) != hipSuccess) return HHFFBP_E_DEVICE;
    }
    return HHFFBP_OK;
}

}  // namespace hh
