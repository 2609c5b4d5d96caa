// Internal structures shared by the host plan and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hhffbp.h"

namespace hh {

constexpr double kLight = 299792458.0;  // m/s
constexpr double kPi = 3.14159265358979323846;
// Base index of an interpolation stencil: floor(t + kStencilEps).  A parent grid
// point seen by a child that shares an edge with it (Q = 2) sits on a child node
// up to rounding; the offset makes every code path choose the same stencil.
constexpr double kStencilEps = 1e-9;
// Threads of every imaging kernel's block (four waves of 64).
constexpr int kBlockThreads = 256;

// One non-empty subarray as the kernels see it.  Rectangles are the cell
// rectangles of the bisection (aperture plane z' = 0).
struct NodeDev {
    double x0, x1, y0, y1, d2;  // rectangle and D^2 = 4 Lx^2 + 4 Ly^2
    int32_t i0, j0, ni, nj;     // lattice columns (i, j) in [i0, i0+ni) x [j0, j0+nj)
    int32_t col_base;           // first entry in this depth's column table
    int32_t val_base;           // first value in this depth's value array
    int32_t npts;               // grid points
    int32_t nchild;             // non-empty children (compact indices at depth + 1)
    int32_t child[4];
    int32_t pos_begin, pos_end; // leaves: range in leaf-sorted position order
    int32_t fwd_block0;         // depths F..S-1: the node's first block of the forward merge
                                // (the point in lane slot s of its merge order lies in block
                                // fwd_block0 + s / (256 / Q))
    int32_t pad1;
};

// One pencil (column) of a lattice: l in [lo, hi] stored from value offset `off`
// (relative to the node's val_base).  An empty column has hi < lo.
struct ColEntry {
    int32_t off, lo, hi, pad;
};

// Per leaf grid point, precomputed in float64 on the host:
//   d      = q - c (float32), c = leaf centre on the aperture plane
//   bin    = floor((|q - c| - R0) / dR), frac the remainder in [0, 1)
//   pre    = exp(j (2 kc |q - c| - Phi(q)))
struct LeafPoint {
    float dx, dy, dz;
    int32_t bin;
    float frac;
    float pre_re, pre_im;
    int32_t pad;
};

// Interpolation weights of the merges: per axis (u, v, n) and tap t < T/2,
// the coefficients of a polynomial in the fractional offset x (BANDLIMITED;
// tap T-1-t is tap t at 1 - x), or kind = LAGRANGE (weights formed
// directly).  Passed to kernels by value.
constexpr int kPolyDeg = 7;
constexpr int kMaxTaps = 6;
struct InterpPoly {
    int32_t kind;
    float c[3][kMaxTaps / 2][kPolyDeg + 1];
};

// Work item of a per-node point loop: node (compact index) and first point.
struct BlockItem {
    int32_t node, start;
};

// Final stage: voxels are processed in bricks of kBrickX x kBrickY x kBrickZ
// (z fastest in a brick, as in the image), and each (brick, depth-1 node) has
// the box of that node's lattice indices [i0, i0 + ni) x [j0, j0 + nj) x
// [l0, l0 + nl) its stencils use: first from the maps with one index of margin
// on every side for rounding, then, once the plan-time records exist, the
// exact hull of the records' stencils.  In LDS the box's columns lie cs >= nl
// values apart (ni * nj * cs <= kTileCap + kTileCap / 4); ni = 0 marks a box
// of more than kTileCap values at 2^lsh >= nl per column (the kernel then
// gathers from the pencils) or one no stencil uses.
constexpr int kBrickX = 4, kBrickY = 8, kBrickZ = 8;
static_assert(kBrickX * kBrickY * kBrickZ == kBlockThreads, "one voxel per thread of a block");
constexpr int kTileCap = 2048;
// The final stage's LDS column stride for boxes of nl <= 24 (TileBox::cs), which
// the kernel also takes as a compile-time constant when every box has it.
constexpr int kFinalCS = 24;
// Positions per block of the level-1 adjoint (one block per leaf and kAdjPos
// of its leaf-sorted positions).
constexpr int kAdjPos = 8;
struct TileBox {
    int32_t i0, j0, l0, ni, nj, nl, lsh;
    int32_t inv_nj;  // ceil(2^22 / nj): column c of the box is (c * inv_nj >> 22, c mod nj)
    int32_t inv_nl;  // ceil(2^22 / nl): point e of the box, column-major, is in column e * inv_nl >> 22
    int32_t cs;      // LDS column stride (values)
};

// Bricks of a parent grid for the merge adjoint: kMBrickI x kMBrickJ columns
// (i, j) x kMBrickL lattice steps l of one node's grid, with origin (i, j, l); a
// lane's grid point is found through the node's column table (lanes outside
// every pencil are idle).  Their stencils cover a smaller box of the child grid
// than a run of points along the pencils does.
constexpr int kMBrickI = 4, kMBrickJ = 4, kMBrickL = 16;
static_assert(kMBrickI * kMBrickJ * kMBrickL == kBlockThreads, "one grid point per thread of a block");
struct MergeBrick {
    int32_t node, i, j, l;
};

// Interpolation record of one (point, child) pair of a merge or of the final
// stage, formed at plan time in float64 with the same arithmetic that builds
// the grids (Sec. III maps, stencil base floor(gamma w + kStencilEps)):
//   cij    first stencil column (ci | cj << 16) relative to the child's lattice
//          columns (i0, j0); kNoPair: the pair contributes nothing (an absent
//          parent point, a padding lane, no such child)
//   l0     first stencil index along n
//   fu, fv, fn   fractional lattice coordinates in [0, 1]
//   turns  phase in turns, reduced to [-1/2, 1/2]: Phi_child - Phi_parent in a
//          merge (restores the child's downconversion and applies the parent's),
//          Phi_child in the final stage
// Every stencil is checked at plan time to lie inside the child's pencils.
struct InterpIdx {
    uint32_t cij;
    int32_t l0;
};
struct InterpGeo {
    float fu, fv, fn, turns;
};
constexpr uint32_t kNoPair = 0xffffffffu;

// Leaf points per block of the fused range-compression + level-1 BP kernel.
constexpr int kAbsmaxParts = 1024;  // blocks of the echo max-reduction
constexpr int kFusedPoints = 1024;

// Range bins [lo, lo + n) that a level-1 BP block can read: every tap of its
// points for positions within the leaf's reach.
struct BinWindow {
    int32_t lo, n;
};

struct Rect {
    double x0, x1, y0, y1;
};

// Host view of one grid G of a subarray.
struct HostLattice {
    double gamma[3] = {3, 3, 3};  // the grid's oversampling per axis: point (i, j, l) at (i, j, l) / gamma
    int32_t i0 = 0, j0 = 0, ni = 0, nj = 0;
    std::vector<int32_t> lo, hi;  // per column
    std::vector<int64_t> off;     // per column, first point
    int64_t npts = 0;
    int64_t n_absent = 0;         // points without a preimage (xyz = NaN, value 0)
    std::vector<double> xyz;      // [npts][3]
};

struct HostNode {
    int depth = 0;
    Rect rect{};
    std::vector<int32_t> members;  // position indices (caller order)
    std::vector<int32_t> children; // tree indices at depth + 1
    int32_t parent = -1;
    int32_t compact = -1;          // index among the non-empty nodes of its depth
    HostLattice lat;
    bool empty() const { return members.empty(); }
};

struct DeviceBuffers {
    void *B = nullptr;              // range-compression matrix, float [2 Nf][2 Nr]
    void *Bx = nullptr;             // the same split for the bf16 GEMM (Plan::Bx), or none
    void *perm = nullptr;           // int32 [n_pos], sorted -> caller index
    void *leaf_of_sorted = nullptr; // int32 [n_pos]
    void *leaf_centre = nullptr;    // double2 [n_leaves]
    void *pos64 = nullptr;          // double [n_pos][3], caller order
    void *check_counts = nullptr;   // int32 [blocks of kBlockThreads positions]: hhffbp_check_positions
    void *posoff = nullptr;         // float4 [n_pos]: the plan positions' leaf offsets and
                                    // squared norms (as k_prep_positions writes them)
    void *unit_scales = nullptr;    // float [n_scales()] of 1: storage scales of c64, bf16
    void *weights = nullptr;        // float [n_pos] aperture weights, caller order (or none)
    void *kf = nullptr;             // double [n_freq]: k_f (exact direct mode)
    void *kf_turns = nullptr;       // float [n_freq]: k_f / pi (exact mode, general spacing)
    std::vector<void *> nodes;      // per depth: NodeDev[]
    std::vector<void *> cols;       // per depth: ColEntry[]
    std::vector<void *> colbase;    // per depth: int32 off - lo per column (the value index of
                                    // lattice point l of column c is val_base + colbase[c] + l)
    void *leafpts = nullptr;        // LeafPoint[] of depth S
    void *leaf_blocks = nullptr;    // BlockItem[]
    void *leaf_wins = nullptr;      // BinWindow[], one per leaf block
    void *leaf_order = nullptr;     // int32[n_blocks_leaf_phys]: workgroup -> leaf block, -1 idle
    void *fused_blocks = nullptr;   // BlockItem[] of kFusedPoints leaf points (range_fused)
    void *fused_wins = nullptr;     // BinWindow[], one per fused block
    void *final_tiles = nullptr;    // TileBox[n_bricks][n nodes at depth F]
    void *adj_blocks = nullptr;     // BlockItem[]: (leaf, first sorted position of kAdjPos)
    void *Bd = nullptr;             // range-derivative matrix (rows x j 2 k_f), [2 Nf][2 Nr]
    void *Badj = nullptr;           // conj-transposed DFT matrix, [2 Nr][2 Nf]
    void *scale_mult = nullptr;     // float [n_scales()]: worst-case gain from echoes to each stage
    std::vector<void *> merge_blocks;  // per depth F..S-1: BlockItem[] of 256 points (adjoint)
    std::vector<void *> merge_blocks_fwd;  // per depth F..S-1: BlockItem[] of 256 / Q points
    std::vector<void *> merge_bricks;      // per depth F..S-1: MergeBrick[] (merge adjoint)
    std::vector<void *> merge_order;       // per depth F..S-1: int32 per point, lane slot -> point
    std::vector<void *> merge_rank;        // per depth F..S-1: int32 per point, point -> lane slot
    std::vector<void *> merge_idx, merge_geo;  // per depth F..S-1: InterpIdx[], InterpGeo[] of
                                               // the forward merge, [block][lane]
    void *final_idx = nullptr;      // InterpIdx[n_bricks][nodes at depth F][kBlockThreads]
    void *final_geo = nullptr;      // InterpGeo[n_bricks][nodes at depth F][kBlockThreads]
};

struct Plan {
    hhffbp_config cfg{};
    int S = 0, Q = 4, T = 4;
    // first depth with a grid: 1, or 0 when the root holds a compressed grid of
    // its own (then the final stage resamples that one node onto the voxels)
    int F = 1;
    double gamma[3] = {3, 3, 3};
    double gamma_leaf[3] = {3, 3, 3};  // the level-1 (depth S) grids' oversampling
    const double *gamma_of(int depth) const { return depth == S ? gamma_leaf : gamma; }
    // band
    std::vector<double> k;
    double kmin = 0, kmax = 0, kc = 0;
    bool k_equispaced = false;  // k_f = k_0 + f dk to 1e-9 dk (exact direct mode's Horner sum)
    double k0 = 0, dk = 0;
    // range profiles
    int W = 7, kernel = HHFFBP_RANGE_ES;
    double U = 2, dR = 0, R0 = 0, beta = 0;
    int64_t Nr = 0;
    std::vector<float> Bmat;  // [2 Nf][2 Nr]
    std::vector<uint16_t> Bx; // Bmat split into bfloat16 parts in MFMA fragment order (split GEMM)
    int32_t gemm_nt = 0;      // its 32-column tiles
    bool gemm_dma = false;    // the split GEMM's direct-load form may run (LDS opt-in granted)
    int32_t gemm_br_spx = 0;  // row streams per XCD of its B-resident form (0: that form is off)
    std::vector<float> Bdmat; // [2 Nf][2 Nr]
    std::vector<float> Badjmat; // [2 Nr][2 Nf]
    // tree
    std::vector<std::vector<HostNode>> levels;
    std::vector<int32_t> perm;           // sorted -> caller index
    std::vector<int32_t> leaf_of_sorted; // compact leaf index per sorted position
    std::vector<double> leaf_centre;     // [n_leaves][2]
    std::vector<double> positions;       // caller order, [n_pos][3]
    std::vector<float> weights;          // caller order, empty for unit weights
    std::vector<std::vector<int32_t>> compact_to_tree;  // per depth
    std::vector<int64_t> depth_points;   // per depth
    std::vector<int64_t> n_blocks_merge; // per depth
    std::vector<int64_t> n_blocks_merge_fwd; // per depth
    std::vector<std::vector<MergeBrick>> merge_bricks;  // per depth, host copy
    // per depth F..S-1 and non-empty node (compact order): the node's points in
    // the order the forward merge's lanes take them (see build_merge_order)
    std::vector<std::vector<std::vector<int32_t>>> merge_order;
    int64_t n_blocks_leaf = 0, n_blocks_adj = 0, n_blocks_fused = 0;
    int64_t n_blocks_leaf_phys = 0;  // workgroups of the level-1 BP launch (leaf_order)
    int32_t fused_win_max = 0;  // widest BinWindow of the fused blocks
    int32_t leaf_win_max = 0;  // widest BinWindow of the level-1 BP blocks
    std::vector<TileBox> final_tiles;  // host copy, brick-major
    int64_t n_bricks = 0, n_tiled = 0;  // final-stage bricks; (brick, node) pairs with a box
    bool final_box_only = false;        // every final-stage stencil lies in its brick's box
    int32_t final_cs = 0;               // the column stride every staged box shares, else 0
    int64_t final_box_vals = 0;         // largest ni * nj * cs of a staged box
    int64_t final_box_cols = 0;         // largest ni * nj of a staged box
    int64_t leaf_pairs = 0, merge_pairs = 0, final_pairs = 0;
    std::vector<int64_t> merge_pairs_depth;  // per depth < S
    std::vector<double> level_estimate;      // per depth: gamma^3 * integral of |det J| over the voxels
    // workspace layout (bytes)
    size_t ws_prof = 0, ws_posoff = 0, ws_total = 0;
    size_t ws_scales = 0, ws_amax = 0;  // per-call storage scales (float [n_scales()]) and
                                        // per-block max |echo| (float [kAbsmaxParts])
    size_t ws_gprof = 0, ws_gpos = 0, ws_gmax = 0, ws_total_bwd = 0;  // backward additions
    size_t device_bytes = 0;  // plan tables uploaded to the device (owned by the plan)
    double leaf_reach = 0.0;  // max |p' - c| over leaf members and their leaf centres c (z = 0), plus slack
    double model_s = 0.0;     // the Sec. IV-B cost model's level-1 BP + interpolation time
    size_t adj_lds_max = 0;   // dynamic LDS per block the level-1 adjoint may use (plan time)
    InterpPoly ipoly{};       // interpolation weights from grids at gamma
    InterpPoly ipoly_leaf{};  // ... from the level-1 grids (gamma_leaf)
    // weights of an interpolation whose children sit at depth `child_depth`
    const InterpPoly &ipoly_for(int child_depth) const { return child_depth == S ? ipoly_leaf : ipoly; }
    std::vector<size_t> ws_gvals;        // backward: float32 cotangents per depth
    std::vector<float> scale_mult;       // host copy of dev.scale_mult
    std::vector<size_t> ws_vals;         // per depth
    DeviceBuffers dev;
    double plan_seconds = 0;
    double z_valid = 0;
    // optional per-stage HIP events (hhffbp_profile_begin/_end)
    std::vector<hipEvent_t> prof_events;  // [max_calls][n_stages + 1]
    int prof_max_calls = 0, prof_calls = 0;
    std::vector<std::string> stage_names() const;
    int64_t n_vox() const { return cfg.grid_dims[0] * cfg.grid_dims[1] * cfg.grid_dims[2]; }
    // storage-scale slot of depth d's subimages: d, except S + 1 for the root grid
    // (slot 0 belongs to the profiles)
    int scale_slot(int d) const { return d == 0 ? S + 1 : d; }
    int n_scales() const { return S + 1 + (F == 0 ? 1 : 0); }
};

// Dynamic LDS of the final stage: the largest staged box, one spare value per
// thread and the largest box's column table (float2 and int2 entries).
inline size_t final_lds_bytes(const Plan &P)
{
    return ((size_t)P.final_box_vals + kBlockThreads + (size_t)P.final_box_cols) * 8;
}

// Plan construction (host, float64).  Throws hh::Error on failure.
struct Error {
    hhffbp_status status;
    std::string msg;
};

void build_plan_host(Plan &plan);
void choose_stages(hhffbp_config &c);  // stages < 0: pick S by the cost model
void upload_plan(Plan &plan);
void release_plan(Plan &plan);

// Launchers (kernels.hip, kernels_adjoint.hip).
hipError_t launch_prep(const Plan &P, const double *pos64, float4 *posoff, hipStream_t st);
// Per block of kBlockThreads positions, the count beyond the slack box into counts.
hipError_t launch_check_positions(const Plan &P, const double *pos64, int32_t *counts,
                                  hipStream_t st);
// Range-compression GEMM with float32 output; A stored as `storage_a` reals.
// a_w / c_w: optional per-row weights of A (indexed by A's row) and of C
// (indexed by C's row after c_perm); NULL for none.
hipError_t launch_rc_gemm(int storage_a, const void *A, const int32_t *a_perm, int M, int K,
                          const float *B, int N, float *C, const int32_t *c_perm, hipStream_t st,
                          const float *a_w, const float *c_w);
// Plan time: the dynamic LDS the level-1 adjoint may use (adj_lds_max) and the
// opt-in of its instances that need more than the default (kernels_adjoint.hip).
hipError_t prepare_backward(Plan &P);
// Plan time: the LDS opt-ins of the split GEMM's direct-load (gemm_dma) and
// B-resident (gemm_br_spx) forms.
hipError_t prepare_forward(Plan &P);
hhffbp_status launch_backward(const Plan &P, const void *echoes, const double *positions,
                              const void *grad_image, void *grad_echoes, double *grad_positions,
                              char *ws, hipStream_t st);
// `events`, when non-null, holds stage_names().size() + 1 events recorded on
// `stream` before the first stage and after each stage.
hhffbp_status launch_image(const Plan &plan, const void *echoes, const double *positions,
                           void *image, char *ws, hipStream_t stream, hipEvent_t *events);
// Device address of the library-held workspace of hhffbp_image_noalloc on
// `device`, which must be the current device (kernels.hip).
hipError_t noalloc_workspace(int device, char **ptr);

// Image reductions (kernels_metrics.hip); no plan, current device.
size_t stats_workspace_bytes();
hipError_t launch_image_stats(const void *image, const void *ref, int64_t n, double *stats,
                              void *ws, hipStream_t st);
hipError_t launch_loss_grad(const void *image, const void *clean, int64_t n, const double *stats,
                            double w_ent, double w_l2, double *loss, void *grad, hipStream_t st);
hipError_t launch_box_peaks(const void *image, const int64_t dims[3], int32_t n_boxes,
                            const int32_t *boxes, int64_t *peaks, hipStream_t st);

}  // namespace hh
