/*
 * hhffbp.h - C ABI of the MI355X (gfx950) HHFFBPA library.
 *
 * Near-range handheld-SAR imaging by fast factorised backprojection with
 * analytic spectrum compression (Wang, Yao, Song, Sun, "A Fast and Accurate
 * 3-D Reconstruction Algorithm for Near-Range Microwave Imaging with Handheld
 * Synthetic Aperture Radar").
 *
 * Problem (Sec. II-A): antenna positions p'_i = (x', y', z') in metres, an
 * arbitrary and non-uniform set; stepped frequencies f_j with k_j = 2 pi f_j / c;
 * echoes s(p'_i, k_j); the output is the complex reflectivity f(p) on a regular
 * voxel grid in front of the aperture.  Direct BPA is eq. (4):
 *     f(p) = sum_i sum_j s(p'_i, k_j) exp(+j 2 k_j |p - p'_i|)
 * (unit weights for the integral measures).  HHFFBPA (Sec. III, IV-A)
 * approximates it: range compression (eq. 2), backprojection of each level-1
 * subarray onto a coarse grid that is uniform in the LLT coordinates (u, v, n)
 * of eq. uvw_xyz, spatial downconversion by exp(-j Phi) (eq. sdc_mul,
 * eq. sdc_phi), and recursive merges that interpolate the compressed children
 * onto the parent's grid, undo the downconversion and sum them.
 *
 * Conventions
 *  - Every function returns an hhffbp_status; out-parameters are untouched on
 *    error and no exception crosses the ABI.  hhffbp_last_error() gives a
 *    human-readable detail for the calling thread's last failure.
 *  - Complex values are interleaved (re, im) pairs: float32 pairs
 *    (HHFFBP_C64), IEEE half pairs (HHFFBP_F16) or bfloat16 pairs (HHFFBP_BF16).
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *    memory on the plan's device.  The caller owns every device buffer,
 *    including the workspace; the library owns only the plan (its host tables
 *    and a plan-time device upload of the geometry).
 *  - Compute calls enqueue work on `stream` (a hipStream_t, passed as void*),
 *    do not allocate and do not synchronise.
 */
#ifndef HHFFBP_H
#define HHFFBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hhffbp_plan_s *hhffbp_plan_t; /* opaque, owned by the library */

typedef enum {
    HHFFBP_OK = 0,
    HHFFBP_E_INVALID = -1,     /* bad argument or configuration            */
    HHFFBP_E_UNSUPPORTED = -2, /* valid but not implemented                */
    HHFFBP_E_NOMEM = -3,       /* host or plan-time device allocation      */
    HHFFBP_E_DEVICE = -4,      /* HIP runtime or launch failure            */
    HHFFBP_E_WORKSPACE = -5,   /* workspace missing or too small           */
    HHFFBP_E_NUMERIC = -6      /* plan geometry failed (e.g. no inverse)   */
} hhffbp_status;

/* Imaging mode. */
enum {
    HHFFBP_FACTORIZED = 0,   /* HHFFBPA (Sec. IV-A); stages = 0 is one subarray */
    HHFFBP_DIRECT_RC = 1,    /* direct BPA of eq. (3) on range-compressed data   */
    HHFFBP_DIRECT_EXACT = 2  /* direct BPA of eq. (4): the frequency sum per
                                (voxel, position), no range compression; with
                                equispaced frequencies a Horner sum in
                                exp(j 2 dk Delta R).  Forward only.          */
};

/* Storage type of the echoes, range profiles and subimages.  Sums, phases and
 * interpolation are float32 in every case; the image is always complex64.
 * HHFFBP_F16 arrays carry per-stage power-of-two scales chosen per call from the
 * largest echo component, so that no stored value exceeds 2^15. */
enum { HHFFBP_C64 = 0, HHFFBP_F16 = 1, HHFFBP_BF16 = 2 };

/* Kernel used to evaluate a range profile between its samples. */
enum {
    HHFFBP_RANGE_ES = 0,     /* exponential-of-semicircle, pre-corrected DFT    */
    HHFFBP_RANGE_LINEAR = 1  /* two-tap linear, pre-corrected by the triangle
                                kernel's transform (fast; ~-61 dB vs ES at U = 8) */
};

/* Interpolation weights of the merges (separable, interp_taps per axis).
 * LAGRANGE: the Lagrange polynomial through the stencil.  BANDLIMITED: for
 * each fractional offset x the weights minimising the squared error over all
 * signals band-limited to |omega| <= pi / gamma per grid step, integrated over
 * the band: the compressed subimages have unit spectral support per LLT unit
 * (Sec. III) and gamma grid points per unit; the plan fits each weight with a
 * degree-7 polynomial in x (error < 1e-6, checked at plan time). */
enum { HHFFBP_INTERP_LAGRANGE = 0, HHFFBP_INTERP_BANDLIMITED = 1 };

/* Range-compression GEMM (eq. 2) of an image with C64 storage.  SPLIT_BF16:
 * every float32 operand splits exactly into three bfloat16 parts (8 significant
 * bits each, remainder <= 2^-27 relative) and the six partial products above
 * 2^-26 relative, each exact in float32, accumulate in float32 on bf16 MFMA;
 * the profiles then carry a float32 GEMM's error.  F32: float32 MFMA.  Half
 * storage, the fused form and hhffbp_backward always take the float32 kernel. */
enum { HHFFBP_GEMM_SPLIT_BF16 = 0, HHFFBP_GEMM_F32 = 1 };

typedef struct {
    int64_t n_pos;              /* number of antenna positions, >= 1              */
    int64_t n_freq;             /* number of frequency samples, >= 2              */
    const double *positions;    /* host, [n_pos][3] metres; scene at z > max z'  */
    const double *freqs_hz;     /* host, [n_freq], any order and spacing, > 0     */
    double grid_origin[3];      /* centre of voxel (0,0,0), metres                */
    double grid_pitch[3];       /* voxel pitch per axis, > 0                      */
    int64_t grid_dims[3];       /* (nx, ny, nz); image index (ix*ny + iy)*nz + iz */
    int32_t mode;               /* HHFFBP_FACTORIZED, HHFFBP_DIRECT_RC or _EXACT  */
    int32_t stages;             /* S >= 0: number of merge stages; S = -K (factorised
                                   mode): the S in 1..K that minimises the operation
                                   count of Sec. IV-B on the candidates' exact pair
                                   counts (per-pair costs measured on MI355X)      */
    int32_t merge_factor;       /* Q = 2 (binary, alternating axes) or 4          */
    double oversample[3];       /* gamma per LLT axis (u, v, n), each in [1, 8]   */
    int32_t interp_taps;        /* T, Lagrange taps per axis: 4 or 6              */
    int32_t range_kernel;       /* HHFFBP_RANGE_ES or HHFFBP_RANGE_LINEAR         */
    double range_oversample;    /* U: range-bin spacing pi / (U (kmax - kmin))    */
    int32_t range_taps;         /* W: ES taps (4..8); ignored for linear          */
    int32_t storage;            /* HHFFBP_C64, HHFFBP_F16 or HHFFBP_BF16          */
    double position_slack;      /* metres the positions may move after planning  */
    int32_t device;             /* HIP device ordinal; -1 plans on the host only  */
    int32_t interp_kernel;      /* HHFFBP_INTERP_LAGRANGE or HHFFBP_INTERP_BANDLIMITED */
    int32_t final_staging;      /* 1: the final stage stages each voxel brick's child
                                   values through LDS (the default); 0: it gathers
                                   every stencil from the pencils.  Same result bit
                                   for bit (same summation order); 0 is for tests. */
    const double *weights;      /* host [n_pos] aperture weights w_i, the measure of
                                   dp' in eq. (4): f = sum_i w_i sum_f s_if e^{...};
                                   NULL: unit weights.  Must be finite; read only
                                   during hhffbp_plan.  The gradients follow:
                                   grad_s_i carries w_i, grad_p'_i the weighted sum. */
    int32_t root_grid;          /* 0: the root's grid is the voxel grid (Sec. IV-A; the
                                   default).  1: the root also gets a compressed grid
                                   in the full aperture's (u, v, n), built like every
                                   other grid; the last merge lands on it and one
                                   single-child interpolation takes it to the voxels.
                                   Fewer interpolations where the voxel grid is finer
                                   than the full aperture's band, at the error of one
                                   more interpolation.  Needs FACTORIZED with S >= 1. */
    int32_t range_fused;        /* 0: range compression (eq. 2) as its own MFMA GEMM
                                   writing every profile to the workspace, then the
                                   level-1 BP (the default).  1: one kernel per block
                                   of 1024 leaf points forms the profiles of its bin
                                   window from the echoes on MFMA into LDS and
                                   backprojects them, with no profile array; the
                                   blocks of a leaf each form its profiles.  Needs
                                   FACTORIZED with S >= 1, the linear range kernel
                                   and C64 storage, and an image only: hhffbp_backward
                                   returns HHFFBP_E_UNSUPPORTED for such a plan.     */
    double oversample_leaf[3];  /* gamma of the level-1 (leaf) grids per LLT axis, each
                                   in [1, 8]; 0 (the default): `oversample`.  The
                                   level-1 BP's work scales with the leaf grids and
                                   only the first merge interpolates from them, so a
                                   coarser leaf grid trades that one interpolation's
                                   error for level-1 work (Sec. III sampling, Sec.
                                   IV-B operation count).  Factorised plans only.   */
    int32_t range_gemm;         /* HHFFBP_GEMM_SPLIT_BF16 (the default) or
                                   HHFFBP_GEMM_F32                                  */
} hhffbp_config;

/* Fill `cfg` with defaults: FACTORIZED, S = 3, Q = 4, gamma = (3, 3, 3.5), T = 4, ES with
 * U = 2 and W = 7, C64 storage, 5 mm slack, device 0, Lagrange interpolation, final-stage
 * staging on, no root grid, leaf grids at `oversample`, the split-bfloat16 GEMM.  Pointers and sizes are
 * zeroed and must be set by the caller. */
void hhffbp_config_default(hhffbp_config *cfg);

/*
 * Build a plan (Sec. IV-A): the subarray tree, the sampling grid G of every
 * subarray below the root (and of the root with cfg->root_grid), the (x, y, z) preimage of every grid point, the
 * range window and the range-compression matrix, uploaded to `cfg->device`.
 * Runs on the host in float64; one small kernel on the device's null stream
 * forms the plan positions' leaf offsets, and the call waits for it.  Reads
 * `cfg` and the host arrays it points to only during the call.  On success
 * *out receives a plan that must be released
 * with hhffbp_plan_destroy.  With cfg->device = -1 nothing touches a GPU: the
 * plan holds its host tables only (for inspection) and hhffbp_image refuses it.  Errors: HHFFBP_E_INVALID (non-finite input, empty
 * grid, grid not in front of the aperture, unsupported Q/T/W/U/gamma),
 * HHFFBP_E_NUMERIC (a grid point without a preimage), HHFFBP_E_NOMEM,
 * HHFFBP_E_DEVICE.
 */
hhffbp_status hhffbp_plan(const hhffbp_config *cfg, hhffbp_plan_t *out);

/* Release a plan and its device tables.  NULL is ignored.  No call that uses
 * the plan may still be running on any stream. */
void hhffbp_plan_destroy(hhffbp_plan_t plan);

/* Bytes of device workspace that hhffbp_image (with_backward = 0) or
 * hhffbp_backward (with_backward = 1) needs. */
hhffbp_status hhffbp_workspace_bytes(hhffbp_plan_t plan, int32_t with_backward,
                                     size_t *bytes);

/*
 * Form the image.
 *   echoes      device, [n_pos][n_freq] complex pairs in the plan's storage
 *               type (float32, IEEE half or bfloat16 re/im), rows in the order
 *               of cfg->positions.
 *   positions   device float64 [n_pos][3] to backproject with, or NULL for
 *               the plan's own positions.  The tree and grids stay as planned;
 *               each coordinate is clamped to within cfg->position_slack of the
 *               planned one, the box the range windows hold (see
 *               hhffbp_check_positions).
 *   image       device complex64 [nx][ny][nz] (z fastest), overwritten.
 *   workspace   device, at least hhffbp_workspace_bytes(plan, 0) bytes,
 *               256-byte aligned; its contents on entry do not matter.
 * Enqueued on `stream`; returns after the launches.  Errors: HHFFBP_E_INVALID
 * (NULL echoes or image), HHFFBP_E_WORKSPACE, HHFFBP_E_DEVICE.
 */
hhffbp_status hhffbp_image(hhffbp_plan_t plan, const void *echoes, const double *positions,
                           void *image, void *workspace, size_t ws_bytes, void *stream);

/*
 * Form the image without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same work and result as hhffbp_image, bit for bit,
 * with the workspace taken from a static array that the library holds on each
 * device it runs on (HHFFBP_NOALLOC_WORKSPACE_BYTES bytes, kept from the
 * module's load until the process ends).  The call itself allocates nothing:
 * no hipMalloc, hipFree or allocating library routine.
 *   echoes, positions, image   as for hhffbp_image (caller-owned, device)
 * Every such call on one device shares that device's array, which keeps the
 * last call's contents: calls that may overlap on one device (other streams,
 * other threads) race and must be ordered by the caller.  hhffbp_profile_begin
 * does not apply to these calls.  Errors: HHFFBP_E_INVALID (NULL echoes or
 * image), HHFFBP_E_WORKSPACE (the plan needs more than
 * HHFFBP_NOALLOC_WORKSPACE_BYTES of workspace; nothing is launched),
 * HHFFBP_E_DEVICE.
 */
#define HHFFBP_NOALLOC_WORKSPACE_BYTES ((size_t)256 << 20)
hhffbp_status hhffbp_image_noalloc(hhffbp_plan_t plan, const void *echoes,
                                   const double *positions, void *image, void *stream);

/*
 * Check device positions against the plan's slack: the plan's range windows and
 * carrier form hold for positions within cfg->position_slack of the planned ones
 * along each axis (hhffbp_image and hhffbp_backward clamp every coordinate into
 * that box, so their results are those of the clamped positions).
 *   positions   device float64 [n_pos][3], as for hhffbp_image
 *   n_outside   host, optional: receives the number of positions with a coordinate
 *               beyond the slack (or not finite)
 * Enqueues one kernel and a 4-byte-per-256-positions copy on `stream` and waits
 * for the stream.  Calls on one plan must not overlap (they share the plan's
 * count buffer).  Returns HHFFBP_OK when every position is inside, and
 * HHFFBP_E_INVALID (with *n_outside set) when any is not; HHFFBP_E_DEVICE on a
 * HIP failure.
 */
hhffbp_status hhffbp_check_positions(hhffbp_plan_t plan, const double *positions,
                                     int64_t *n_outside, void *stream);

/*
 * Gradients of a real loss L(image) with respect to the echoes and the antenna
 * positions (autofocus of handheld motion errors, Sec. I), with the plan frozen:
 * the tree and grids stay as planned and only the level-1 backprojection
 * depends on the positions.  The image is linear in the echoes, f = A s, so
 *     grad_echoes    = A^H grad_image                 (the transposed HHFFBPA)
 *     grad_positions = Re sum_q conj(G_q) d f'_q / d p'   (G: level-1 cotangents)
 * with the complex convention grad = dL/dRe + j dL/dIm.
 *   echoes          device, as for hhffbp_image (needed for grad_positions)
 *   positions       device float64 [n_pos][3] used by the forward, or NULL
 *   grad_image      device complex64 [nx][ny][nz]
 *   grad_echoes     device complex64 [n_pos][n_freq] or NULL, overwritten
 *   grad_positions  device float64 [n_pos][3] or NULL, overwritten
 *   workspace       at least hhffbp_workspace_bytes(plan, 1) bytes, 256-B aligned
 * The transposed merges scatter with float atomics, so results may differ in
 * the last bits between calls.  Needs a factorised plan with stages >= 1
 * (HHFFBP_E_UNSUPPORTED otherwise).  Errors as for hhffbp_image.
 */
hhffbp_status hhffbp_backward(hhffbp_plan_t plan, const void *echoes, const double *positions,
                              const void *grad_image, void *grad_echoes, double *grad_positions,
                              void *workspace, size_t ws_bytes, void *stream);

/* Read-only description of a plan, for sizing and work accounting. */
typedef struct {
    int32_t stages, merge_factor, n_leaves, n_nodes;
    int64_t n_pos, n_freq, n_vox;
    int64_t n_range_bins;           /* N_r                                      */
    double range_lo, range_step;    /* R_0 and delta R of the profile grid (m); R_0 is a
                                       whole multiple of delta R (samples at b delta R) */
    int64_t level_points[16];       /* grid points summed over depth d = 1..S;
                                       [0]: the root grid's points (0 without one) */
    int64_t leaf_pairs;             /* sum over leaves of points x positions    */
    int64_t merge_pairs;            /* (parent point, child) pairs, depths 1..S-1
                                       (0..S-1 with a root grid)                 */
    int64_t final_pairs;            /* (voxel, child) pairs at the root (with a
                                       root grid: voxels, the root its one child) */
    double plan_seconds;            /* host time spent in hhffbp_plan           */
    int32_t storage;                /* storage type of profiles and subimages   */
    int64_t ws_scales_offset;       /* workspace byte offset of float scale[S+1]
                                       (S+2 with a root grid): stored profiles
                                       carry scale[0], depth-d subimages scale[d],
                                       the root grid scale[S+1]; written by
                                       hhffbp_image with HHFFBP_F16 storage only
                                       (the other types store values unscaled) */
    int64_t device_bytes;           /* device memory the plan holds (its tables) */
    double model_ms;                /* Sec. IV-B cost model: level-1 BP + interpolation,
                                       with the per-pair costs of hhffbp_config.stages */
    int64_t final_bricks;           /* final stage: voxel bricks of 4 x 8 x 8 (x, y, z) */
    int64_t final_boxed;            /* (brick, depth-1 node) pairs (with a root grid:
                                       (brick, root)) whose stencils fit one staged
                                       box (the rest read the pencils directly)  */
    int32_t root_grid;              /* the plan's cfg->root_grid                */
    int64_t merge_pairs_depth[16];  /* (parent point, child) pairs of the merge at depth d
                                       (d < S; with a root grid d = 0 is the merge onto
                                       it); their sum is merge_pairs              */
    double level_estimate[16];      /* per depth d = 0..S: gamma_u gamma_v gamma_n times
                                       the integral of |det J| over the voxel box, J the
                                       Jacobian of (u, v, n) of eq. uvw_xyz, summed over
                                       the depth's nodes: the sample count of Sec. IV-B
                                       (eq. 4_subimgsmppresimp) before the interpolation
                                       stencils' halos (midpoint rule on <= 32^3 cells) */
    int32_t range_gemm_form;        /* the range-compression (eq. 2) kernel hhffbp_image
                                       runs (modes other than HHFFBP_DIRECT_EXACT), for
                                       echoes at a 16-byte aligned address:
                                       HHFFBP_GEMM_FORM_* below (the form of
                                       hhffbp_config.range_gemm the device and K allow) */
} hhffbp_plan_info;

/* Values of hhffbp_plan_info.range_gemm_form.  FUSED: none, range compression
 * is fused into the level-1 BP (range_fused).  F32: float32 MFMA.  SPLIT_REG:
 * split bfloat16 with operands loaded to registers.  SPLIT_DMA: split, operands
 * streamed through LDS by direct global-to-LDS loads (K a multiple of 16).
 * SPLIT_BRES: split, each block's B fragments resident in LDS for all of K and A
 * loaded to registers (K a multiple of 64, K/16 x 9 KB of LDS a block). */
enum {
    HHFFBP_GEMM_FORM_FUSED = -1,
    HHFFBP_GEMM_FORM_F32 = 0,
    HHFFBP_GEMM_FORM_SPLIT_REG = 1,
    HHFFBP_GEMM_FORM_SPLIT_DMA = 2,
    HHFFBP_GEMM_FORM_SPLIT_BRES = 3
};

hhffbp_status hhffbp_get_plan_info(hhffbp_plan_t plan, hhffbp_plan_info *info);

/*
 * Where the compressed subimage f' of node (depth, index) lives in the
 * workspace after hhffbp_image, and its grid: lattice column (i, j) covers
 * i in [i0, i0 + ni), j in [j0, j0 + nj); column c = (i - i0) * nj + (j - j0)
 * holds l in [l_lo[c], l_hi[c]] contiguously from point offset col_off[c].
 * Values are complex pairs of the plan's storage type (8 bytes per point for
 * HHFFBP_C64, 4 for HHFFBP_F16 and HHFFBP_BF16) at byte offset
 * *ws_offset + size * point, with HHFFBP_F16 multiplied by the depth's scale
 * (see hhffbp_plan_info.ws_scales_offset).  Arrays may be
 * NULL to query sizes only; otherwise they must hold ni * nj entries.
 * Depth 0 is the root: with cfg->root_grid its grid is node (0, 0); without,
 * the root's grid is the user grid and has no lattice (HHFFBP_E_INVALID); an empty
 * node reports npoints = 0.
 */
hhffbp_status hhffbp_node_layout(hhffbp_plan_t plan, int32_t depth, int32_t index,
                                 int32_t dims[4] /* i0, j0, ni, nj */, int64_t *npoints,
                                 int64_t *ws_offset, int32_t *l_lo, int32_t *l_hi,
                                 int64_t *col_off);

/* Float64 (x, y, z) preimages of a node's grid points, [npoints][3], host. */
hhffbp_status hhffbp_node_points(hhffbp_plan_t plan, int32_t depth, int32_t index,
                                 double *xyz);

/*
 * Optional per-stage timing with HIP events on the caller's stream.  After
 * hhffbp_profile_begin(plan, max_calls) the next max_calls hhffbp_image calls
 * record an event before their first kernel and after each stage.
 * hhffbp_profile_end waits for the last recorded event, writes into
 * stage_ms[k] (k < min(max_stages, *n_stages)) the milliseconds stage k took
 * summed over the recorded calls, reports the stage count and the number of
 * recorded calls, and releases the events.  hhffbp_stage_name(plan, k) names
 * stage k ("rc_gemm", "leaf_bp", "merge_d<d>", "final", "direct_bp", ...).
 * Creating the events allocates (host side); use it outside capture regions.
 */
hhffbp_status hhffbp_profile_begin(hhffbp_plan_t plan, int32_t max_calls);
hhffbp_status hhffbp_profile_end(hhffbp_plan_t plan, double *stage_ms, int32_t max_stages,
                                 int32_t *n_stages, int32_t *n_calls);
const char *hhffbp_stage_name(hhffbp_plan_t plan, int32_t index);

/*
 * Image reductions: quality metrics and the autofocus loss (no plan; they run
 * on the current HIP device).  image, reference and clean are device
 * complex64 arrays of n elements in linear order (n = 0 is allowed).  |f|^2 is
 * formed in float64 from the float32 parts and every sum accumulates in
 * float64 in a fixed order, so results repeat bit for bit.
 *
 * hhffbp_image_stats writes 8 doubles to the device array stats:
 *   [0] S = sum |f|^2       [1] sum |r|^2         [2] sum |f - r|^2
 *   [3] sum |f|^2 ln |f|^2, voxels with f = 0 counting 0
 *   [4] max |f|^2 (0 if n = 0)   [5] its lowest linear index (-1 if n = 0)
 *   [6] entropy H = -sum q ln q, q = |f|^2 / S, computed as ln S - [3] / S
 *       (0 if S = 0); the autofocus sharpness measure mentioned in Sec. I
 *   [7] NRMSE ||f - r|| / ||r|| (NaN without a reference or if ||r|| = 0)
 * reference may be NULL ([1] = [2] = 0).  workspace: device memory of at least
 * hhffbp_stats_workspace_bytes() bytes, 8-byte aligned, clobbered.
 *
 * hhffbp_loss_grad: from stats of hhffbp_image_stats(image, clean, ...),
 * enqueued earlier on the same stream, the loss
 *     L = w_entropy H(f) + w_l2 sum |f - c|^2 / sum |c|^2
 * (second term dropped if clean = NULL) into the device double *loss (if not
 * NULL) and its cotangent in the convention dL/dRe f + j dL/dIm f into the
 * device complex64 array grad (if not NULL):
 *     grad = w_entropy (-2 f (ln q + H) / S) + w_l2 (2 (f - c) / sum |c|^2)
 * (voxels with f = 0 take no entropy term).  Weights must be finite; grad may
 * alias neither input.
 *
 * hhffbp_box_peaks: for each of n_boxes voxel boxes of a [d0][d1][d2] image
 * (z fastest), boxes = device int32 [n_boxes][6] (x_lo, x_hi, y_lo, y_hi, z_lo,
 * z_hi) inclusive and clipped to the grid, writes to the device int64 array
 * peaks the lowest linear index (ix d1 + iy) d2 + iz of the largest |f|^2 in
 * the box, or -1 for a box with no voxel inside.
 */
hhffbp_status hhffbp_stats_workspace_bytes(size_t *bytes);
hhffbp_status hhffbp_image_stats(const void *image, const void *reference, int64_t n,
                                 double *stats, void *workspace, size_t ws_bytes, void *stream);
hhffbp_status hhffbp_loss_grad(const void *image, const void *clean, int64_t n,
                               const double *stats, double w_entropy, double w_l2, double *loss,
                               void *grad, void *stream);
hhffbp_status hhffbp_box_peaks(const void *image, const int64_t dims[3], int32_t n_boxes,
                               const int32_t *boxes, int64_t *peaks, void *stream);

/* Static strings; never NULL. */
const char *hhffbp_status_string(hhffbp_status status);
const char *hhffbp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HHFFBP_H */
