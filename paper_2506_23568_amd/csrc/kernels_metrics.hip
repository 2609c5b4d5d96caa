// Image reductions on gfx950: the quality metrics of an image (energy, NRMSE
// against a reference, entropy, peak) and the autofocus loss with its cotangent.
//
//   k_stats_partial   one grid-stride pass: per-block float64 sums and argmax
//   k_stats_final     one block folds the partials in a fixed order
//   k_loss_value      L = w_ent H + w_l2 sum |f - c|^2 / sum |c|^2 from the folded stats
//   k_loss_grad       the cotangent dL/dRe f + j dL/dIm f, elementwise
//   k_box_peaks       argmax of |f|^2 inside each voxel box, one block per box
//
// |f|^2 is formed in float64 from the float32 parts (both squares are exact),
// so an argmax is decided identically by any IEEE float64 evaluation; ties
// take the lowest linear index.  Every sum runs in a fixed order (fixed grid,
// fixed shuffle tree, fixed fold), so results repeat bit for bit.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hhffbp_internal.hpp"

namespace hh {
namespace {

constexpr int kRedBlock = 256;
constexpr int kRedGrid = 1024;  // partial slots; the workspace holds kRedGrid x 8 doubles
constexpr int kStats = 8;

struct Acc {
    double a, r2, d2, alna, amax;
    int64_t imax;
};

__device__ __forceinline__ double abs2(float2 v)
{
    return (double)v.x * (double)v.x + (double)v.y * (double)v.y;
}

// larger |f|^2 wins; equal values keep the lower index (INT64_MAX = none)
__device__ __forceinline__ void take_max(double &am, int64_t &im, double b, int64_t ib)
{
    if (b > am || (b == am && ib < im)) {
        am = b;
        im = ib;
    }
}

__device__ __forceinline__ void wave_fold(Acc &s)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        s.a += __shfl_xor(s.a, o, 64);
        s.r2 += __shfl_xor(s.r2, o, 64);
        s.d2 += __shfl_xor(s.d2, o, 64);
        s.alna += __shfl_xor(s.alna, o, 64);
        const double bm = __shfl_xor(s.amax, o, 64);
        const int64_t bi = __shfl_xor(s.imax, o, 64);
        take_max(s.amax, s.imax, bm, bi);
    }
}

// Block fold of s (all kRedBlock threads call it); the result is valid in thread 0.
__device__ Acc block_fold(Acc s)
{
    __shared__ Acc sh[kRedBlock / 64];
    wave_fold(s);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kRedBlock / 64; ++w) {
            s.a += sh[w].a;
            s.r2 += sh[w].r2;
            s.d2 += sh[w].d2;
            s.alna += sh[w].alna;
            take_max(s.amax, s.imax, sh[w].amax, sh[w].imax);
        }
    }
    return s;
}

template <bool REF>
__global__ __launch_bounds__(kRedBlock) void k_stats_partial(const float2 *__restrict__ f,
                                                             const float2 *__restrict__ r,
                                                             int64_t n, double *__restrict__ part)
{
    Acc s{0.0, 0.0, 0.0, 0.0, -1.0, INT64_MAX};
    const int64_t stride = (int64_t)gridDim.x * kRedBlock;
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < n; i += stride) {
        const float2 v = f[i];
        const double a = abs2(v);
        s.a += a;
        if (a > 0.0) s.alna += a * log(a);
        if (a > s.amax) {  // indices rise along a thread's walk: strict > keeps the lowest
            s.amax = a;
            s.imax = i;
        }
        if constexpr (REF) {
            const float2 w = r[i];
            s.r2 += abs2(w);
            const double dx = (double)v.x - (double)w.x, dy = (double)v.y - (double)w.y;
            s.d2 += dx * dx + dy * dy;
        }
    }
    s = block_fold(s);
    if (threadIdx.x == 0) {
        double *p = part + (size_t)blockIdx.x * kStats;
        p[0] = s.a;
        p[1] = s.r2;
        p[2] = s.d2;
        p[3] = s.alna;
        p[4] = s.amax;
        p[5] = (double)s.imax;  // INT64_MAX as a double is never a real index
    }
}

__global__ __launch_bounds__(kRedBlock) void k_stats_final(const double *__restrict__ part,
                                                           int nparts, int has_ref,
                                                           double *__restrict__ stats)
{
    Acc s{0.0, 0.0, 0.0, 0.0, -1.0, INT64_MAX};
    for (int b = threadIdx.x; b < nparts; b += kRedBlock) {
        const double *p = part + (size_t)b * kStats;
        s.a += p[0];
        s.r2 += p[1];
        s.d2 += p[2];
        s.alna += p[3];
        const int64_t ib = (p[5] >= 9.2e18) ? INT64_MAX : (int64_t)p[5];
        take_max(s.amax, s.imax, p[4], ib);
    }
    s = block_fold(s);
    if (threadIdx.x == 0) {
        const bool any = s.imax != INT64_MAX;
        stats[0] = s.a;
        stats[1] = s.r2;
        stats[2] = s.d2;
        stats[3] = s.alna;
        stats[4] = any ? s.amax : 0.0;
        stats[5] = any ? (double)s.imax : -1.0;
        stats[6] = s.a > 0.0 ? log(s.a) - s.alna / s.a : 0.0;  // H = ln S - sum a ln a / S
        stats[7] = (has_ref && s.r2 > 0.0) ? sqrt(s.d2 / s.r2) : __builtin_nan("");
    }
}

__global__ void k_loss_value(const double *__restrict__ stats, int has_clean, double w_ent,
                             double w_l2, double *__restrict__ loss)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        loss[0] = w_ent * stats[6] + (has_clean ? w_l2 * stats[2] / stats[1] : 0.0);
}

// g = w_ent (-2 f (ln q + H) / S) + w_l2 (2 (f - c) / sum |c|^2),  q = |f|^2 / S;
// voxels with f = 0 take no entropy term (the limit of f ln |f|^2).
template <bool CLEAN>
__global__ __launch_bounds__(kRedBlock) void k_loss_grad(const float2 *__restrict__ f,
                                                         const float2 *__restrict__ c, int64_t n,
                                                         const double *__restrict__ stats,
                                                         double w_ent, double w_l2,
                                                         float2 *__restrict__ grad)
{
    const double S = stats[0], H = stats[6];
    const double lnS = S > 0.0 ? log(S) : 0.0;
    const double invS = S > 0.0 ? w_ent / S : 0.0;
    const double ic2 = CLEAN ? 2.0 * w_l2 / stats[1] : 0.0;
    const int64_t stride = (int64_t)gridDim.x * kRedBlock;
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < n; i += stride) {
        const float2 v = f[i];
        const double a = abs2(v);
        const double ge = a > 0.0 ? -2.0 * (log(a) - lnS + H) * invS : 0.0;
        double gx = ge * (double)v.x, gy = ge * (double)v.y;
        if constexpr (CLEAN) {
            const float2 w = c[i];
            gx += ic2 * ((double)v.x - (double)w.x);
            gy += ic2 * ((double)v.y - (double)w.y);
        }
        grad[i] = make_float2((float)gx, (float)gy);
    }
}

__global__ __launch_bounds__(kRedBlock) void k_box_peaks(const float2 *__restrict__ f, int64_t d0,
                                                         int64_t d1, int64_t d2,
                                                         const int32_t *__restrict__ boxes,
                                                         int64_t *__restrict__ peaks)
{
    const int32_t *b = boxes + (size_t)blockIdx.x * 6;
    const int64_t x0 = max((int64_t)b[0], (int64_t)0), x1 = min((int64_t)b[1], d0 - 1);
    const int64_t y0 = max((int64_t)b[2], (int64_t)0), y1 = min((int64_t)b[3], d1 - 1);
    const int64_t z0 = max((int64_t)b[4], (int64_t)0), z1 = min((int64_t)b[5], d2 - 1);
    Acc s{0.0, 0.0, 0.0, 0.0, -1.0, INT64_MAX};
    if (x1 >= x0 && y1 >= y0 && z1 >= z0) {
        const int64_t nz = z1 - z0 + 1, ny = y1 - y0 + 1, nx = x1 - x0 + 1;
        const int64_t nb = nx * ny * nz;
        // box order (x, y, z) with z fastest is the image's linear order
        for (int64_t t = threadIdx.x; t < nb; t += kRedBlock) {
            const int64_t iz = z0 + t % nz, iy = y0 + (t / nz) % ny, ix = x0 + t / (nz * ny);
            const int64_t li = (ix * d1 + iy) * d2 + iz;
            const double a = abs2(f[li]);
            if (a > s.amax) {
                s.amax = a;
                s.imax = li;
            }
        }
    }
    s = block_fold(s);
    if (threadIdx.x == 0) peaks[blockIdx.x] = (s.imax == INT64_MAX) ? -1 : s.imax;
}

}  // namespace

size_t stats_workspace_bytes() { return (size_t)kRedGrid * kStats * sizeof(double); }

hipError_t launch_image_stats(const void *image, const void *ref, int64_t n, double *stats,
                              void *ws, hipStream_t st)
{
    const int64_t nb = (n + kRedBlock - 1) / kRedBlock;
    const int g = (int)(nb < kRedGrid ? (nb > 0 ? nb : 1) : kRedGrid);
    double *part = (double *)ws;
    if (ref)
        hipLaunchKernelGGL(k_stats_partial<true>, dim3(g), dim3(kRedBlock), 0, st,
                           (const float2 *)image, (const float2 *)ref, n, part);
    else
        hipLaunchKernelGGL(k_stats_partial<false>, dim3(g), dim3(kRedBlock), 0, st,
                           (const float2 *)image, (const float2 *)nullptr, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(kRedBlock), 0, st, (const double *)part, g,
                       ref ? 1 : 0, stats);
    return hipGetLastError();
}

hipError_t launch_loss_grad(const void *image, const void *clean, int64_t n, const double *stats,
                            double w_ent, double w_l2, double *loss, void *grad, hipStream_t st)
{
    if (loss) {
        hipLaunchKernelGGL(k_loss_value, dim3(1), dim3(64), 0, st, stats, clean ? 1 : 0, w_ent,
                           w_l2, loss);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (grad && n > 0) {
        const int64_t nb = (n + kRedBlock - 1) / kRedBlock;
        const unsigned g = (unsigned)(nb < 8192 ? nb : 8192);
        if (clean)
            hipLaunchKernelGGL(k_loss_grad<true>, dim3(g), dim3(kRedBlock), 0, st,
                               (const float2 *)image, (const float2 *)clean, n, stats, w_ent, w_l2,
                               (float2 *)grad);
        else
            hipLaunchKernelGGL(k_loss_grad<false>, dim3(g), dim3(kRedBlock), 0, st,
                               (const float2 *)image, (const float2 *)nullptr, n, stats, w_ent,
                               w_l2, (float2 *)grad);
    }
    return hipGetLastError();
}

hipError_t launch_box_peaks(const void *image, const int64_t dims[3], int32_t n_boxes,
                            const int32_t *boxes, int64_t *peaks, hipStream_t st)
{
    if (n_boxes <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_box_peaks, dim3((unsigned)n_boxes), dim3(kRedBlock), 0, st,
                       (const float2 *)image, dims[0], dims[1], dims[2], boxes, peaks);
    return hipGetLastError();
}

}  // namespace hh
