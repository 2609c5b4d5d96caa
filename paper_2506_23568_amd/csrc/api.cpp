// extern "C" entry points of libhhffbp (declared in include/hhffbp.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hhffbp_internal.hpp"

struct hhffbp_plan_s {
    hh::Plan plan;
};

namespace {

thread_local std::string g_last_error = "no error";

hhffbp_status fail(hhffbp_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

}  // namespace

static void destroy_events(hh::Plan &P);

extern "C" {

void hhffbp_config_default(hhffbp_config *cfg)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->mode = HHFFBP_FACTORIZED;
    cfg->stages = 3;
    cfg->merge_factor = 4;
    cfg->oversample[0] = cfg->oversample[1] = 3.0;
    cfg->oversample[2] = 3.5;  // the n axis carries the widest compressed spectrum
    cfg->interp_taps = 4;
    cfg->range_kernel = HHFFBP_RANGE_ES;
    cfg->range_oversample = 2.0;
    cfg->range_taps = 7;
    cfg->storage = HHFFBP_C64;
    cfg->position_slack = 5e-3;
    cfg->device = 0;
    cfg->interp_kernel = HHFFBP_INTERP_LAGRANGE;
    cfg->final_staging = 1;
    cfg->weights = nullptr;
    cfg->root_grid = 0;
    cfg->range_fused = 0;
    cfg->oversample_leaf[0] = cfg->oversample_leaf[1] = cfg->oversample_leaf[2] = 0.0;
    cfg->range_gemm = HHFFBP_GEMM_SPLIT_BF16;
}

hhffbp_status hhffbp_plan(const hhffbp_config *cfg, hhffbp_plan_t *out)
{
    if (!cfg || !out) return fail(HHFFBP_E_INVALID, "hhffbp_plan: NULL argument");
    hhffbp_plan_s *h = nullptr;
    try {
        h = new hhffbp_plan_s();
        h->plan.cfg = *cfg;
        hh::choose_stages(h->plan.cfg);
        hh::build_plan_host(h->plan);
        h->plan.cfg.positions = nullptr;
        h->plan.cfg.freqs_hz = nullptr;
        hh::upload_plan(h->plan);
    } catch (const hh::Error &e) {
        if (h) {
            hh::release_plan(h->plan);
            delete h;
        }
        return fail(e.status, e.msg);
    } catch (const std::bad_alloc &) {
        if (h) {
            hh::release_plan(h->plan);
            delete h;
        }
        return fail(HHFFBP_E_NOMEM, "host allocation failed while planning");
    } catch (...) {
        if (h) {
            hh::release_plan(h->plan);
            delete h;
        }
        return fail(HHFFBP_E_INVALID, "unexpected error while planning");
    }
    *out = h;
    return HHFFBP_OK;
}

void hhffbp_plan_destroy(hhffbp_plan_t plan)
{
    if (!plan) return;
    destroy_events(plan->plan);
    hh::release_plan(plan->plan);
    delete plan;
}

hhffbp_status hhffbp_workspace_bytes(hhffbp_plan_t plan, int32_t with_backward, size_t *bytes)
{
    if (!plan || !bytes) return fail(HHFFBP_E_INVALID, "hhffbp_workspace_bytes: NULL argument");
    *bytes = with_backward ? plan->plan.ws_total_bwd : plan->plan.ws_total;
    return HHFFBP_OK;
}

hhffbp_status hhffbp_backward(hhffbp_plan_t plan, const void *echoes, const double *positions,
                              const void *grad_image, void *grad_echoes, double *grad_positions,
                              void *workspace, size_t ws_bytes, void *stream)
{
    if (!plan || !grad_image) return fail(HHFFBP_E_INVALID, "hhffbp_backward: NULL argument");
    const hh::Plan &P = plan->plan;
    if (P.cfg.device < 0) return fail(HHFFBP_E_DEVICE, "hhffbp_backward: host-only plan");
    if (P.S < 1)
        return fail(HHFFBP_E_UNSUPPORTED, "hhffbp_backward: needs a factorised plan with stages >= 1");
    if (P.cfg.range_fused)
        return fail(HHFFBP_E_UNSUPPORTED, "hhffbp_backward: not for a plan with range_fused");
    if (!grad_echoes && !grad_positions) return HHFFBP_OK;
    if (grad_positions && !echoes)
        return fail(HHFFBP_E_INVALID, "hhffbp_backward: the position gradient needs the echoes");
    if (!workspace || ws_bytes < P.ws_total_bwd)
        return fail(HHFFBP_E_WORKSPACE, "hhffbp_backward: workspace missing or smaller than " +
                                            std::to_string(P.ws_total_bwd) + " bytes");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(HHFFBP_E_WORKSPACE, "hhffbp_backward: workspace must be 256-byte aligned");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(HHFFBP_E_DEVICE, "hipGetDevice failed");
    if (cur != P.cfg.device && hipSetDevice(P.cfg.device) != hipSuccess)
        return fail(HHFFBP_E_DEVICE, "hipSetDevice failed");
    hhffbp_status st = hh::launch_backward(P, echoes, positions, grad_image, grad_echoes,
                                           grad_positions, (char *)workspace, (hipStream_t)stream);
    if (cur != P.cfg.device) (void)hipSetDevice(cur);
    if (st != HHFFBP_OK) return fail(st, std::string("hhffbp_backward: launch failed: ") +
                                             hipGetErrorString(hipGetLastError()));
    return HHFFBP_OK;
}

hhffbp_status hhffbp_image(hhffbp_plan_t plan, const void *echoes, const double *positions,
                           void *image, void *workspace, size_t ws_bytes, void *stream)
{
    if (!plan || !echoes || !image) return fail(HHFFBP_E_INVALID, "hhffbp_image: NULL argument");
    const hh::Plan &P = plan->plan;
    if (P.cfg.device < 0) return fail(HHFFBP_E_DEVICE, "hhffbp_image: host-only plan (device < 0)");
    if (!workspace || ws_bytes < P.ws_total)
        return fail(HHFFBP_E_WORKSPACE, "hhffbp_image: workspace missing or smaller than " +
                                            std::to_string(P.ws_total) + " bytes");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(HHFFBP_E_WORKSPACE, "hhffbp_image: workspace must be 256-byte aligned");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(HHFFBP_E_DEVICE, "hipGetDevice failed");
    if (cur != P.cfg.device && hipSetDevice(P.cfg.device) != hipSuccess)
        return fail(HHFFBP_E_DEVICE, "hipSetDevice failed");
    hipEvent_t *ev = nullptr;
    hh::Plan &Pm = plan->plan;
    if (Pm.prof_calls < Pm.prof_max_calls) {
        ev = &Pm.prof_events[(size_t)Pm.prof_calls * (Pm.stage_names().size() + 1)];
        ++Pm.prof_calls;
    }
    hhffbp_status st = hh::launch_image(P, echoes, positions, image, (char *)workspace,
                                        (hipStream_t)stream, ev);
    if (cur != P.cfg.device) (void)hipSetDevice(cur);
    if (st != HHFFBP_OK) return fail(st, std::string("hhffbp_image: launch failed: ") +
                                             hipGetErrorString(hipGetLastError()));
    return HHFFBP_OK;
}

hhffbp_status hhffbp_image_noalloc(hhffbp_plan_t plan, const void *echoes,
                                   const double *positions, void *image, void *stream)
{
    if (!plan || !echoes || !image)
        return fail(HHFFBP_E_INVALID, "hhffbp_image_noalloc: NULL argument");
    const hh::Plan &P = plan->plan;
    if (P.cfg.device < 0)
        return fail(HHFFBP_E_DEVICE, "hhffbp_image_noalloc: host-only plan (device < 0)");
    if (P.ws_total > HHFFBP_NOALLOC_WORKSPACE_BYTES)
        return fail(HHFFBP_E_WORKSPACE, "hhffbp_image_noalloc: the plan needs " +
                                            std::to_string(P.ws_total) +
                                            " bytes of workspace, more than the library's " +
                                            std::to_string(HHFFBP_NOALLOC_WORKSPACE_BYTES));
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(HHFFBP_E_DEVICE, "hipGetDevice failed");
    if (cur != P.cfg.device && hipSetDevice(P.cfg.device) != hipSuccess)
        return fail(HHFFBP_E_DEVICE, "hipSetDevice failed");
    char *ws = nullptr;
    hipError_t e = hh::noalloc_workspace(P.cfg.device, &ws);
    hhffbp_status st = HHFFBP_E_DEVICE;
    if (e == hipSuccess)
        st = hh::launch_image(P, echoes, positions, image, ws, (hipStream_t)stream, nullptr);
    if (cur != P.cfg.device) (void)hipSetDevice(cur);
    if (e != hipSuccess)
        return fail(HHFFBP_E_DEVICE, std::string("hhffbp_image_noalloc: workspace address: ") +
                                         hipGetErrorString(e));
    if (st != HHFFBP_OK) return fail(st, std::string("hhffbp_image_noalloc: launch failed: ") +
                                             hipGetErrorString(hipGetLastError()));
    return HHFFBP_OK;
}

hhffbp_status hhffbp_check_positions(hhffbp_plan_t plan, const double *positions,
                                     int64_t *n_outside, void *stream)
{
    if (!plan || !positions) return fail(HHFFBP_E_INVALID, "hhffbp_check_positions: NULL argument");
    const hh::Plan &P = plan->plan;
    if (P.cfg.device < 0)
        return fail(HHFFBP_E_DEVICE, "hhffbp_check_positions: host-only plan (device < 0)");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(HHFFBP_E_DEVICE, "hipGetDevice failed");
    if (cur != P.cfg.device && hipSetDevice(P.cfg.device) != hipSuccess)
        return fail(HHFFBP_E_DEVICE, "hipSetDevice failed");
    const size_t nb = (size_t)((P.cfg.n_pos + hh::kBlockThreads - 1) / hh::kBlockThreads);
    std::vector<int32_t> counts(nb, 0);
    hipError_t e = hh::launch_check_positions(P, positions, (int32_t *)P.dev.check_counts,
                                              (hipStream_t)stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(counts.data(), P.dev.check_counts, nb * sizeof(int32_t),
                           hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (cur != P.cfg.device) (void)hipSetDevice(cur);
    if (e != hipSuccess)
        return fail(HHFFBP_E_DEVICE, std::string("hhffbp_check_positions: ") + hipGetErrorString(e));
    int64_t tot = 0;
    for (int32_t c : counts) tot += c;
    if (n_outside) *n_outside = tot;
    if (tot > 0)
        return fail(HHFFBP_E_INVALID, "hhffbp_check_positions: " + std::to_string(tot) +
                                          " positions lie beyond the planned slack of " +
                                          std::to_string(P.cfg.position_slack) + " m");
    return HHFFBP_OK;
}

hhffbp_status hhffbp_get_plan_info(hhffbp_plan_t plan, hhffbp_plan_info *info)
{
    if (!plan || !info) return fail(HHFFBP_E_INVALID, "hhffbp_get_plan_info: NULL argument");
    const hh::Plan &P = plan->plan;
    std::memset(info, 0, sizeof(*info));
    info->stages = P.S;
    info->merge_factor = P.Q;
    info->n_leaves = (int32_t)P.compact_to_tree[P.S].size();
    int32_t nn = 0;
    for (auto &v : P.compact_to_tree) nn += (int32_t)v.size();
    info->n_nodes = nn;
    info->n_pos = P.cfg.n_pos;
    info->n_freq = P.cfg.n_freq;
    info->n_vox = P.n_vox();
    info->n_range_bins = P.Nr;
    info->range_lo = P.R0;
    info->range_step = P.dR;
    for (int d = P.F; d <= P.S && d < 16; ++d) info->level_points[d] = P.depth_points[d];
    info->leaf_pairs = P.leaf_pairs;
    info->merge_pairs = P.merge_pairs;
    info->final_pairs = P.final_pairs;
    info->plan_seconds = P.plan_seconds;
    info->storage = P.cfg.storage;
    info->device_bytes = (int64_t)P.device_bytes;
    info->model_ms = 1e3 * P.model_s;
    info->final_bricks = P.n_bricks;
    info->final_boxed = P.n_tiled;
    info->ws_scales_offset = (int64_t)P.ws_scales;
    info->root_grid = P.F == 0 ? 1 : 0;
    for (int d = 0; d < (int)P.merge_pairs_depth.size() && d < 16; ++d)
        info->merge_pairs_depth[d] = P.merge_pairs_depth[d];
    for (int d = 0; d < (int)P.level_estimate.size() && d < 16; ++d)
        info->level_estimate[d] = P.level_estimate[d];
    // the choice the range-compression launch makes for aligned echoes
    const bool k16 = (2 * P.cfg.n_freq) % 16 == 0;
    if (P.cfg.range_fused)
        info->range_gemm_form = HHFFBP_GEMM_FORM_FUSED;
    else if (P.cfg.storage != HHFFBP_C64 || (P.dev.Bx == nullptr && P.Bx.empty()))
        info->range_gemm_form = HHFFBP_GEMM_FORM_F32;
    else if (k16 && P.gemm_br_spx > 0)
        info->range_gemm_form = HHFFBP_GEMM_FORM_SPLIT_BRES;
    else if (k16 && P.gemm_dma)
        info->range_gemm_form = HHFFBP_GEMM_FORM_SPLIT_DMA;
    else
        info->range_gemm_form = HHFFBP_GEMM_FORM_SPLIT_REG;
    return HHFFBP_OK;
}

static const hh::HostNode *find_node(const hh::Plan &P, int32_t depth, int32_t index)
{
    if (depth < P.F || depth > P.S) return nullptr;
    if (index < 0 || index >= (int32_t)P.levels[depth].size()) return nullptr;
    return &P.levels[depth][index];
}

hhffbp_status hhffbp_node_layout(hhffbp_plan_t plan, int32_t depth, int32_t index,
                                 int32_t dims[4], int64_t *npoints, int64_t *ws_offset,
                                 int32_t *l_lo, int32_t *l_hi, int64_t *col_off)
{
    if (!plan || !dims || !npoints || !ws_offset)
        return fail(HHFFBP_E_INVALID, "hhffbp_node_layout: NULL argument");
    const hh::Plan &P = plan->plan;
    const hh::HostNode *n = find_node(P, depth, index);
    if (!n) return fail(HHFFBP_E_INVALID, "hhffbp_node_layout: no such node");
    const hh::HostLattice &L = n->lat;
    dims[0] = L.i0;
    dims[1] = L.j0;
    dims[2] = L.ni;
    dims[3] = L.nj;
    *npoints = n->empty() ? 0 : L.npts;
    int64_t base = 0;
    for (int32_t ti : P.compact_to_tree[depth]) {
        if (ti == index) break;
        base += P.levels[depth][ti].lat.npts;
    }
    const int64_t csz = (P.cfg.storage == HHFFBP_C64) ? 8 : 4;
    *ws_offset = (int64_t)P.ws_vals[depth] + csz * base;
    const int64_t nc = (int64_t)L.ni * L.nj;
    for (int64_t c = 0; c < nc; ++c) {
        if (l_lo) l_lo[c] = L.lo[c];
        if (l_hi) l_hi[c] = L.hi[c];
        if (col_off) col_off[c] = L.off[c];
    }
    return HHFFBP_OK;
}

hhffbp_status hhffbp_node_points(hhffbp_plan_t plan, int32_t depth, int32_t index, double *xyz)
{
    if (!plan || !xyz) return fail(HHFFBP_E_INVALID, "hhffbp_node_points: NULL argument");
    const hh::HostNode *n = find_node(plan->plan, depth, index);
    if (!n) return fail(HHFFBP_E_INVALID, "hhffbp_node_points: no such node");
    if (!n->lat.xyz.empty()) std::memcpy(xyz, n->lat.xyz.data(), n->lat.xyz.size() * sizeof(double));
    return HHFFBP_OK;
}

static void destroy_events(hh::Plan &P)
{
    for (hipEvent_t e : P.prof_events) (void)hipEventDestroy(e);
    P.prof_events.clear();
    P.prof_max_calls = P.prof_calls = 0;
}

hhffbp_status hhffbp_profile_begin(hhffbp_plan_t plan, int32_t max_calls)
{
    if (!plan || max_calls < 1) return fail(HHFFBP_E_INVALID, "hhffbp_profile_begin: bad argument");
    hh::Plan &P = plan->plan;
    if (P.cfg.device < 0) return fail(HHFFBP_E_DEVICE, "hhffbp_profile_begin: host-only plan");
    destroy_events(P);
    const size_t per = P.stage_names().size() + 1;
    P.prof_events.assign((size_t)max_calls * per, nullptr);
    for (auto &e : P.prof_events) {
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            destroy_events(P);
            return fail(HHFFBP_E_DEVICE, "hipEventCreate failed");
        }
    }
    P.prof_max_calls = max_calls;
    P.prof_calls = 0;
    return HHFFBP_OK;
}

hhffbp_status hhffbp_profile_end(hhffbp_plan_t plan, double *stage_ms, int32_t max_stages,
                                 int32_t *n_stages, int32_t *n_calls)
{
    if (!plan || !n_stages || !n_calls) return fail(HHFFBP_E_INVALID, "hhffbp_profile_end: NULL");
    hh::Plan &P = plan->plan;
    const int ns = (int)P.stage_names().size();
    *n_stages = ns;
    *n_calls = P.prof_calls;
    if (stage_ms) {
        for (int k = 0; k < std::min(ns, (int)max_stages); ++k) stage_ms[k] = 0.0;
        for (int c = 0; c < P.prof_calls; ++c) {
            hipEvent_t *ev = &P.prof_events[(size_t)c * (ns + 1)];
            if (hipEventSynchronize(ev[ns]) != hipSuccess) {
                destroy_events(P);
                return fail(HHFFBP_E_DEVICE, "hipEventSynchronize failed");
            }
            for (int k = 0; k < std::min(ns, (int)max_stages); ++k) {
                float ms = 0.0f;
                if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) == hipSuccess) stage_ms[k] += ms;
            }
        }
    }
    destroy_events(P);
    return HHFFBP_OK;
}

const char *hhffbp_stage_name(hhffbp_plan_t plan, int32_t i)
{
    static thread_local std::string name;
    if (!plan) return "";
    auto n = plan->plan.stage_names();
    name = (i >= 0 && i < (int32_t)n.size()) ? n[i] : std::string();
    return name.c_str();
}

hhffbp_status hhffbp_stats_workspace_bytes(size_t *bytes)
{
    if (!bytes) return fail(HHFFBP_E_INVALID, "hhffbp_stats_workspace_bytes: NULL argument");
    *bytes = hh::stats_workspace_bytes();
    return HHFFBP_OK;
}

hhffbp_status hhffbp_image_stats(const void *image, const void *reference, int64_t n,
                                 double *stats, void *workspace, size_t ws_bytes, void *stream)
{
    if (n < 0) return fail(HHFFBP_E_INVALID, "hhffbp_image_stats: n < 0");
    if (!stats || (n > 0 && !image))
        return fail(HHFFBP_E_INVALID, "hhffbp_image_stats: NULL argument");
    if (!workspace || ws_bytes < hh::stats_workspace_bytes())
        return fail(HHFFBP_E_WORKSPACE, "hhffbp_image_stats: workspace missing or smaller than " +
                                            std::to_string(hh::stats_workspace_bytes()) + " bytes");
    if (reinterpret_cast<uintptr_t>(workspace) % 8 != 0)
        return fail(HHFFBP_E_WORKSPACE, "hhffbp_image_stats: workspace must be 8-byte aligned");
    const hipError_t e = hh::launch_image_stats(image, reference, n, stats, workspace,
                                                (hipStream_t)stream);
    if (e != hipSuccess)
        return fail(HHFFBP_E_DEVICE, std::string("hhffbp_image_stats: ") + hipGetErrorString(e));
    return HHFFBP_OK;
}

hhffbp_status hhffbp_loss_grad(const void *image, const void *clean, int64_t n,
                               const double *stats, double w_entropy, double w_l2, double *loss,
                               void *grad, void *stream)
{
    if (n < 0) return fail(HHFFBP_E_INVALID, "hhffbp_loss_grad: n < 0");
    if (!stats || (grad && n > 0 && !image))
        return fail(HHFFBP_E_INVALID, "hhffbp_loss_grad: NULL argument");
    if (!std::isfinite(w_entropy) || !std::isfinite(w_l2))
        return fail(HHFFBP_E_INVALID, "hhffbp_loss_grad: weights must be finite");
    const hipError_t e = hh::launch_loss_grad(image, clean, n, stats, w_entropy, w_l2, loss, grad,
                                              (hipStream_t)stream);
    if (e != hipSuccess)
        return fail(HHFFBP_E_DEVICE, std::string("hhffbp_loss_grad: ") + hipGetErrorString(e));
    return HHFFBP_OK;
}

hhffbp_status hhffbp_box_peaks(const void *image, const int64_t dims[3], int32_t n_boxes,
                               const int32_t *boxes, int64_t *peaks, void *stream)
{
    if (!dims || n_boxes < 0 || (n_boxes > 0 && (!image || !boxes || !peaks)))
        return fail(HHFFBP_E_INVALID, "hhffbp_box_peaks: bad argument");
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1)
        return fail(HHFFBP_E_INVALID, "hhffbp_box_peaks: dims must be positive");
    const hipError_t e = hh::launch_box_peaks(image, dims, n_boxes, boxes, peaks,
                                              (hipStream_t)stream);
    if (e != hipSuccess)
        return fail(HHFFBP_E_DEVICE, std::string("hhffbp_box_peaks: ") + hipGetErrorString(e));
    return HHFFBP_OK;
}

const char *hhffbp_status_string(hhffbp_status s)
{
    switch (s) {
    case HHFFBP_OK: return "ok";
    case HHFFBP_E_INVALID: return "invalid argument";
    case HHFFBP_E_UNSUPPORTED: return "unsupported";
    case HHFFBP_E_NOMEM: return "out of memory";
    case HHFFBP_E_DEVICE: return "device error";
    case HHFFBP_E_WORKSPACE: return "workspace too small";
    case HHFFBP_E_NUMERIC: return "numerical failure";
    }
    return "unknown status";
}

const char *hhffbp_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
