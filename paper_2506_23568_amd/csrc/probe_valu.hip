// VALU issue-rate probe (libhhffbp_probe.so): the rate at which a CU issues
// wave64 FP32 FMAs and transcendental instructions (sine, square root), alone
// and mixed.  The roofline figures count VALU lane-operations against
// 256 CU x 4 SIMD x 2.4 GHz x 64 lanes / 4 cycles; this measures what that
// nominal rate comes to on the device, and what a transcendental costs.
//
// Each thread runs `iters` steps of kChains independent dependency chains, 4
// instructions per chain per step, of the mode's mix:
//   0: 4 FMA      1: 4 sine       2: 3 FMA + 1 sine (same chain)
//   3: 4 sqrt     4: 2 FMA + 2 sine
//   5: 3 FMA + 1 sine on an independent chain
//   6: 4 FMA on two interleaved chains
//   7: the level-1 BP's mix: 20 FMA and one each of square root, reciprocal,
//      sine and cosine per step on two interleaved chains (24 instructions per
//      chain and step; 20 of 24 are plain FP32 ops, as in that loop)
#include <hip/hip_runtime.h>

namespace {
constexpr int kChains = 8;

template <int MODE>
__global__ __launch_bounds__(256) void k_probe(float *__restrict__ out, int iters, float a, float b)
{
    float x[kChains], z[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        x[c] = threadIdx.x * 1e-3f + c * 1e-4f;
        z[c] = threadIdx.x * 2e-3f + c * 3e-4f;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if constexpr (MODE == 0) {
                x[c] = fmaf(x[c], a, b); x[c] = fmaf(x[c], a, b);
                x[c] = fmaf(x[c], a, b); x[c] = fmaf(x[c], a, b);
            } else if constexpr (MODE == 1) {
                x[c] = __builtin_amdgcn_sinf(x[c]); x[c] = __builtin_amdgcn_sinf(x[c]);
                x[c] = __builtin_amdgcn_sinf(x[c]); x[c] = __builtin_amdgcn_sinf(x[c]);
            } else if constexpr (MODE == 2) {
                x[c] = fmaf(x[c], a, b); x[c] = fmaf(x[c], a, b); x[c] = fmaf(x[c], a, b);
                x[c] = __builtin_amdgcn_sinf(x[c]);
            } else if constexpr (MODE == 3) {
                x[c] = __builtin_amdgcn_sqrtf(x[c]); x[c] = __builtin_amdgcn_sqrtf(x[c]);
                x[c] = __builtin_amdgcn_sqrtf(x[c]); x[c] = __builtin_amdgcn_sqrtf(x[c]);
            } else if constexpr (MODE == 4) {
                x[c] = fmaf(x[c], a, b); x[c] = __builtin_amdgcn_sinf(x[c]);
                x[c] = fmaf(x[c], a, b); x[c] = __builtin_amdgcn_sinf(x[c]);
            } else if constexpr (MODE == 5) {
                x[c] = fmaf(x[c], a, b); x[c] = fmaf(x[c], a, b); x[c] = fmaf(x[c], a, b);
                z[c] = __builtin_amdgcn_sinf(z[c]);
            } else if constexpr (MODE == 6) {
                x[c] = fmaf(x[c], a, b); z[c] = fmaf(z[c], a, b);
                x[c] = fmaf(x[c], a, b); z[c] = fmaf(z[c], a, b);
            } else {
                x[c] = fmaf(x[c], a, b); z[c] = fmaf(z[c], a, b); x[c] = fmaf(x[c], a, b);
                z[c] = fmaf(z[c], a, b); x[c] = fmaf(x[c], a, b); z[c] = __builtin_amdgcn_sqrtf(z[c]);
                x[c] = fmaf(x[c], a, b); z[c] = fmaf(z[c], a, b); x[c] = fmaf(x[c], a, b);
                z[c] = fmaf(z[c], a, b); x[c] = fmaf(x[c], a, b); z[c] = __builtin_amdgcn_rcpf(z[c]);
                x[c] = fmaf(x[c], a, b); z[c] = fmaf(z[c], a, b); x[c] = fmaf(x[c], a, b);
                z[c] = fmaf(z[c], a, b); x[c] = fmaf(x[c], a, b); z[c] = __builtin_amdgcn_sinf(z[c]);
                x[c] = fmaf(x[c], a, b); z[c] = fmaf(z[c], a, b); x[c] = fmaf(x[c], a, b);
                z[c] = fmaf(z[c], a, b); x[c] = fmaf(x[c], a, b); z[c] = __builtin_amdgcn_cosf(z[c]);
            }
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c] + z[c];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <int MODE>
hipError_t launch(float *out, int blocks, int iters, hipStream_t st)
{
    hipLaunchKernelGGL((k_probe<MODE>), dim3(blocks), dim3(256), 0, st, out, iters, 0.999f, 1e-3f);
    return hipGetLastError();
}

hipError_t launch_mode(int mode, float *out, int blocks, int iters, hipStream_t st)
{
    switch (mode) {
    case 0: return launch<0>(out, blocks, iters, st);
    case 1: return launch<1>(out, blocks, iters, st);
    case 2: return launch<2>(out, blocks, iters, st);
    case 3: return launch<3>(out, blocks, iters, st);
    case 4: return launch<4>(out, blocks, iters, st);
    case 5: return launch<5>(out, blocks, iters, st);
    case 6: return launch<6>(out, blocks, iters, st);
    default: return launch<7>(out, blocks, iters, st);
    }
}
}  // namespace

// Runs mode `mode` (0..7) once untimed, then `reps` times between two events
// on `stream`, and stores the issued rate in wave64 VALU instructions per
// second (the loop's kChains x 4 instructions per step, x 24 in mode 7; its
// few scalar instructions are not counted).  `out` is caller-owned device memory of
// blocks * 256 floats.  Returns 0, or -1 for invalid arguments, or the HIP
// error code of a failed launch.
extern "C" int hhffbp_probe_valu(int mode, int blocks, int iters, int reps, float *out,
                                 void *stream, double *wave_instr_per_s)
{
    if (mode < 0 || mode > 7 || blocks <= 0 || iters <= 0 || reps <= 0 || !out || !wave_instr_per_s)
        return -1;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = launch_mode(mode, out, blocks, iters, st);
    if (e != hipSuccess) return (int)e;
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return (int)e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return (int)e;
    }
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_mode(mode, out, blocks, iters, st);
    (void)hipEventRecord(e1, st);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return (int)e;
    const double per_step = (mode == 7) ? 24.0 : 4.0;  // instructions per chain and step
    const double instr = (double)blocks * 4.0 * iters * kChains * per_step * reps;
    *wave_instr_per_s = instr / (ms * 1e-3);
    return 0;
}
