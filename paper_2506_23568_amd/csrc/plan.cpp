// Host-side plan of the HHFFBPA library (float64): subarray tree, sampling
// grids, grid preimages, range window and range-compression matrix.
//
// Section references are to the paper (Sec. III: analytic SDC and LLT,
// Sec. IV-A: implementation).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <thread>

#include "hhffbp_internal.hpp"

namespace hh {
namespace {

// ---------------------------------------------------------------------------
// Small thread pool helper: run fn(begin, end) over [0, n) in chunks.
void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)> &fn)
{
    if (n <= 0) return;
    unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    int64_t nchunks = (n + grain - 1) / grain;
    if (hw == 1 || nchunks == 1) {
        fn(0, n);
        return;
    }
    std::atomic<int64_t> next{0};
    auto worker = [&]() {
        for (;;) {
            int64_t c = next.fetch_add(1);
            if (c >= nchunks) break;
            int64_t b = c * grain;
            fn(b, std::min(n, b + grain));
        }
    };
    std::vector<std::thread> th;
    unsigned nt = (unsigned)std::min<int64_t>(hw, nchunks);
    for (unsigned t = 1; t < nt; ++t) th.emplace_back(worker);
    worker();
    for (auto &t : th) t.join();
}

// ---------------------------------------------------------------------------
// Spectrum-compression maps of one subarray (Sec. III).  For a point p the
// focal points of u are (x'_min, y'_0, 0) and (x'_max, y'_0, 0), those of v are
// (x'_0, y'_min, 0) and (x'_0, y'_max, 0), with (x'_0, y'_0) the clamp of
// (x, y) onto the rectangle; r sums the distances to the four vertices.
//   u = kmax/pi (|p-Fu-| - |p-Fu+|),  v = kmax/pi (|p-Fv-| - |p-Fv+|)
//   n = (kmax sqrt(r^2 - D^2) - kmin r) / 4pi,   Phi = (kmax sqrt(r^2-D^2) + kmin r) / 4
struct SubarrayMap {
    double x0, x1, y0, y1, d2, kmin, kmax;

    SubarrayMap(const Rect &r, double kmn, double kmx)
        : x0(r.x0), x1(r.x1), y0(r.y0), y1(r.y1), kmin(kmn), kmax(kmx)
    {
        d2 = 4.0 * (x1 - x0) * (x1 - x0) + 4.0 * (y1 - y0) * (y1 - y0);
    }

    // w = (u, v, n); optional Jacobian rows (grad u, grad v, grad n).
    void eval(const double *p, double *w, double *phi, double *jac) const
    {
        const double x = p[0], y = p[1], z = p[2], zz = z * z;
        const double cx = std::min(std::max(x, x0), x1);
        const double cy = std::min(std::max(y, y0), y1);
        const double dx0 = x - x0, dx1 = x - x1, dy0 = y - y0, dy1 = y - y1;
        const double ex = x - cx, ey = y - cy;
        const double ru0 = std::sqrt(dx0 * dx0 + ey * ey + zz);
        const double ru1 = std::sqrt(dx1 * dx1 + ey * ey + zz);
        const double rv0 = std::sqrt(ex * ex + dy0 * dy0 + zz);
        const double rv1 = std::sqrt(ex * ex + dy1 * dy1 + zz);
        const double q00 = std::sqrt(dx0 * dx0 + dy0 * dy0 + zz);
        const double q01 = std::sqrt(dx0 * dx0 + dy1 * dy1 + zz);
        const double q10 = std::sqrt(dx1 * dx1 + dy0 * dy0 + zz);
        const double q11 = std::sqrt(dx1 * dx1 + dy1 * dy1 + zz);
        const double r = q00 + q01 + q10 + q11;
        const double s = std::sqrt(r * r - d2);
        const double cu = kmax / kPi;
        w[0] = cu * (ru0 - ru1);
        w[1] = cu * (rv0 - rv1);
        w[2] = (kmax * s - kmin * r) / (4.0 * kPi);
        if (phi) *phi = 0.25 * (kmax * s + kmin * r);
        if (jac) {
            // grad |p - a| = (p - a) / |p - a|; the clamped coordinates add nothing.
            jac[0] = cu * (dx0 / ru0 - dx1 / ru1);
            jac[1] = cu * (ey / ru0 - ey / ru1);
            jac[2] = cu * (z / ru0 - z / ru1);
            jac[3] = cu * (ex / rv0 - ex / rv1);
            jac[4] = cu * (dy0 / rv0 - dy1 / rv1);
            jac[5] = cu * (z / rv0 - z / rv1);
            const double grx = dx0 / q00 + dx0 / q01 + dx1 / q10 + dx1 / q11;
            const double gry = dy0 / q00 + dy1 / q01 + dy0 / q10 + dy1 / q11;
            const double grz = z * (1.0 / q00 + 1.0 / q01 + 1.0 / q10 + 1.0 / q11);
            const double a = (kmax * r / s - kmin) / (4.0 * kPi);
            jac[6] = a * grx;
            jac[7] = a * gry;
            jac[8] = a * grz;
        }
    }
};

bool solve3(const double *J, const double *f, double *x)
{
    const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                       J[2] * (J[3] * J[7] - J[4] * J[6]);
    if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
    const double id = 1.0 / det;
    x[0] = id * (f[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (f[1] * J[8] - J[5] * f[2]) +
                 J[2] * (f[1] * J[7] - J[4] * f[2]));
    x[1] = id * (J[0] * (f[1] * J[8] - J[5] * f[2]) - f[0] * (J[3] * J[8] - J[5] * J[6]) +
                 J[2] * (J[3] * f[2] - f[1] * J[6]));
    x[2] = id * (J[0] * (J[4] * f[2] - f[1] * J[7]) - J[1] * (J[3] * f[2] - f[1] * J[6]) +
                 f[0] * (J[3] * J[7] - J[4] * J[6]));
    return true;
}

double norm3(const double *a) { return std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }

// Newton with backtracking on |uvn(p) - target|; p holds the start on entry.
bool newton_invert(const SubarrayMap &m, const double *target, double *p)
{
    double w[3], F[3], J[9], dp[3], pn[3], Fn[3];
    m.eval(p, w, nullptr, J);
    for (int a = 0; a < 3; ++a) F[a] = w[a] - target[a];
    double nf = norm3(F);
    for (int it = 0; it < 80; ++it) {
        if (!solve3(J, F, dp)) return false;
        const double ndp = norm3(dp);
        double lam = 1.0;
        double nfn = 0.0;
        for (int bt = 0; bt < 50; ++bt) {
            for (int a = 0; a < 3; ++a) pn[a] = p[a] - lam * dp[a];
            if (pn[2] < 1e-4) pn[2] = 1e-4;
            m.eval(pn, w, nullptr, nullptr);
            for (int a = 0; a < 3; ++a) Fn[a] = w[a] - target[a];
            nfn = norm3(Fn);
            if (nfn < nf || lam * ndp < 1e-13) break;
            lam *= 0.5;
        }
        std::memcpy(p, pn, sizeof(pn));
        std::memcpy(F, Fn, sizeof(Fn));
        nf = nfn;
        if (lam * ndp < 1e-12) return nf < 1e-8;
        m.eval(p, w, nullptr, J);
    }
    return false;
}

// Starting point for the first grid point of a pencil: n is close to
// (kmax - kmin) / pi times the distance to the subarray centre, and u, v are
// close to kmax L / pi times the direction cosines along x and y.
void pencil_start(const SubarrayMap &m, const double *target, double *p)
{
    const double lx = m.x1 - m.x0, ly = m.y1 - m.y0;
    double rho = kPi * target[2] / (m.kmax - m.kmin);
    // refine rho on the boresight axis, where n(rho) = (kmax rho - kmin sqrt(h^2 + rho^2)) / pi
    const double h2 = 0.25 * (lx * lx + ly * ly);
    for (int it = 0; it < 20; ++it) {
        const double s = std::sqrt(h2 + rho * rho);
        const double f = (m.kmax * rho - m.kmin * s) / kPi - target[2];
        const double df = (m.kmax - m.kmin * rho / s) / kPi;
        rho -= f / df;
        if (rho < 1e-3) rho = 1e-3;
    }
    double ax = kPi * target[0] / (m.kmax * lx);
    double ay = kPi * target[1] / (m.kmax * ly);
    ax = std::max(-0.7, std::min(0.7, ax));
    ay = std::max(-0.7, std::min(0.7, ay));
    const double c = std::sqrt(std::max(0.1, 1.0 - ax * ax - ay * ay));
    const double R = rho / c;
    p[0] = 0.5 * (m.x0 + m.x1) + R * ax;
    p[1] = 0.5 * (m.y0 + m.y1) + R * ay;
    p[2] = R * c;
}

// ---------------------------------------------------------------------------
void partition(Plan &P)
{
    const int64_t n = P.cfg.n_pos;
    const double *pos = P.positions.data();
    double xa = pos[0], xb = pos[0], ya = pos[1], yb = pos[1];
    for (int64_t i = 1; i < n; ++i) {
        xa = std::min(xa, pos[3 * i]);
        xb = std::max(xb, pos[3 * i]);
        ya = std::min(ya, pos[3 * i + 1]);
        yb = std::max(yb, pos[3 * i + 1]);
    }
    if (P.S > 0 && !(xb > xa && yb > ya))
        throw Error{HHFFBP_E_INVALID, "aperture has zero extent along x' or y'"};
    const int first_axis = (xb - xa) >= (yb - ya) ? 0 : 1;
    P.levels.assign(P.S + 1, {});
    HostNode root;
    root.depth = 0;
    root.rect = {xa, xb, ya, yb};
    root.members.resize(n);
    for (int64_t i = 0; i < n; ++i) root.members[i] = (int32_t)i;
    P.levels[0].push_back(std::move(root));
    for (int d = 0; d < P.S; ++d) {
        auto &cur = P.levels[d];
        auto &nxt = P.levels[d + 1];
        for (size_t pi = 0; pi < cur.size(); ++pi) {
            const Rect rc = cur[pi].rect;
            // (rectangle, predicate on (x', y')) for each child, in a fixed order
            std::vector<Rect> rects;
            std::vector<std::function<bool(double, double)>> take;
            if (P.Q == 4) {
                const double xm = 0.5 * (rc.x0 + rc.x1), ym = 0.5 * (rc.y0 + rc.y1);
                rects = {{rc.x0, xm, rc.y0, ym}, {rc.x0, xm, ym, rc.y1},
                         {xm, rc.x1, rc.y0, ym}, {xm, rc.x1, ym, rc.y1}};
                take = {[=](double x, double y) { return x < xm && y < ym; },
                        [=](double x, double y) { return x < xm && y >= ym; },
                        [=](double x, double y) { return x >= xm && y < ym; },
                        [=](double x, double y) { return x >= xm && y >= ym; }};
            } else if ((first_axis + d) % 2 == 0) {
                const double xm = 0.5 * (rc.x0 + rc.x1);
                rects = {{rc.x0, xm, rc.y0, rc.y1}, {xm, rc.x1, rc.y0, rc.y1}};
                take = {[=](double x, double) { return x < xm; },
                        [=](double x, double) { return x >= xm; }};
            } else {
                const double ym = 0.5 * (rc.y0 + rc.y1);
                rects = {{rc.x0, rc.x1, rc.y0, ym}, {rc.x0, rc.x1, ym, rc.y1}};
                take = {[=](double, double y) { return y < ym; },
                        [=](double, double y) { return y >= ym; }};
            }
            for (size_t c = 0; c < rects.size(); ++c) {
                HostNode ch;
                ch.depth = d + 1;
                ch.rect = rects[c];
                ch.parent = (int32_t)pi;
                for (int32_t m : cur[pi].members)
                    if (take[c](pos[3 * m], pos[3 * m + 1])) ch.members.push_back(m);
                cur[pi].children.push_back((int32_t)nxt.size());
                nxt.push_back(std::move(ch));
            }
        }
    }
}

// Grid of `node`: every Lagrange stencil its parent's points need, closed into
// one pencil per (i, j) column (Sec. IV-A, grids G_{m,n}).
void build_lattice(Plan &P, HostNode &node, const std::vector<double> &parent_all)
{
    const SubarrayMap map(node.rect, P.kmin, P.kmax);
    const double *gam = P.gamma_of(node.depth);
    // absent parent points (no preimage) need no children
    std::vector<double> parent_xyz;
    parent_xyz.reserve(parent_all.size());
    for (size_t q = 0; q + 2 < parent_all.size(); q += 3)
        if (std::isfinite(parent_all[q + 2]))
            parent_xyz.insert(parent_xyz.end(), &parent_all[q], &parent_all[q] + 3);
    const int64_t np = (int64_t)parent_xyz.size() / 3;
    if (np == 0) throw Error{HHFFBP_E_NUMERIC, "a subarray's parent grid has no valid point"};
    const int T = P.T;
    const int margin = 0;
    const int slo = -(T / 2) + 1 - margin, shi = T / 2 + margin;
    std::vector<int32_t> base(3 * np);
    parallel_for(np, 4096, [&](int64_t b, int64_t e) {
        double w[3];
        for (int64_t q = b; q < e; ++q) {
            map.eval(&parent_xyz[3 * q], w, nullptr, nullptr);
            for (int a = 0; a < 3; ++a)
                base[3 * q + a] = (int32_t)std::floor(gam[a] * w[a] + kStencilEps);
        }
    });
    int32_t imin = INT32_MAX, imax = INT32_MIN, jmin = INT32_MAX, jmax = INT32_MIN;
    for (int64_t q = 0; q < np; ++q) {
        imin = std::min(imin, base[3 * q]);
        imax = std::max(imax, base[3 * q]);
        jmin = std::min(jmin, base[3 * q + 1]);
        jmax = std::max(jmax, base[3 * q + 1]);
    }
    HostLattice &L = node.lat;
    for (int a = 0; a < 3; ++a) L.gamma[a] = gam[a];
    L.i0 = imin + slo;
    L.j0 = jmin + slo;
    L.ni = imax - imin + (shi - slo) + 1;
    L.nj = jmax - jmin + (shi - slo) + 1;
    const int64_t ncol = (int64_t)L.ni * L.nj;
    L.lo.assign(ncol, INT32_MAX);
    L.hi.assign(ncol, INT32_MIN);
    for (int64_t q = 0; q < np; ++q) {
        const int32_t bi = base[3 * q], bj = base[3 * q + 1], bl = base[3 * q + 2];
        for (int a = slo; a <= shi; ++a) {
            const int64_t ci = bi + a - L.i0;
            for (int b = slo; b <= shi; ++b) {
                const int64_t c = ci * L.nj + (bj + b - L.j0);
                L.lo[c] = std::min(L.lo[c], bl + slo);
                L.hi[c] = std::max(L.hi[c], bl + shi);
            }
        }
    }
    L.off.assign(ncol, 0);
    int64_t tot = 0;
    for (int64_t c = 0; c < ncol; ++c) {
        if (L.hi[c] < L.lo[c]) {
            L.lo[c] = 0;
            L.hi[c] = -1;
        }
        L.off[c] = tot;
        tot += (int64_t)L.hi[c] - L.lo[c] + 1;
    }
    L.npts = tot;
    L.xyz.assign(3 * tot, std::numeric_limits<double>::quiet_NaN());
    std::atomic<int64_t> absent{0};
    const double zv = P.z_valid;
    parallel_for(ncol, 64, [&](int64_t b, int64_t e) {
        for (int64_t c = b; c < e; ++c) {
            if (L.hi[c] < L.lo[c]) continue;
            const int32_t i = L.i0 + (int32_t)(c / L.nj), j = L.j0 + (int32_t)(c % L.nj);
            double p[3], prev[3];
            bool have_prev = false;
            for (int32_t l = L.lo[c]; l <= L.hi[c]; ++l) {
                const double target[3] = {i / gam[0], j / gam[1], l / gam[2]};
                if (have_prev) {
                    std::memcpy(p, prev, sizeof(p));
                } else {
                    pencil_start(map, target, p);
                }
                bool ok = newton_invert(map, target, p) && p[2] >= zv;
                if (!ok && have_prev) {
                    pencil_start(map, target, p);
                    ok = newton_invert(map, target, p) && p[2] >= zv;
                }
                if (!ok) {
                    // beyond the (u, v, n) image of the scene half-space: absent
                    absent.fetch_add(1);
                    have_prev = false;
                    continue;
                }
                std::memcpy(&L.xyz[3 * (L.off[c] + (l - L.lo[c]))], p, sizeof(p));
                std::memcpy(prev, p, sizeof(p));
                have_prev = true;
            }
        }
    });
    L.n_absent = absent.load();
}

// Final-stage boxes: per voxel brick and node of depth F, the bounding box of the
// stencils (base floor(gamma w + eps) - T/2 + 1 .. + T/2) of the brick's voxels,
// widened by one index for rounding (the kernel evaluates w in float64 with a
// ~2e-14 relative square root) and clipped to the node's columns.
// The box [lo, hi] (inclusive lattice indices per axis) with its LDS column
// length and the reciprocals that split a box index.  Exact integer quotients:
// for x < 2^11 and d < 2^11, x * ceil(2^22 / d) >> 22 errs by < x / 2^22 < 1 / d.
TileBox make_box(const int32_t *lo, const int32_t *hi)
{
    const int32_t ni = hi[0] - lo[0] + 1, nj = hi[1] - lo[1] + 1, nl = hi[2] - lo[2] + 1;
    int32_t lsh = 0;
    while ((1 << lsh) < nl) ++lsh;
    // LDS column stride: the least cs >= nl with cs = 24 (mod 32) float2.  LDS
    // has 64 four-byte banks, 32 float2; columns j, j + 1, j + 2, j + 3 then
    // start 0, 24, 16, 8 float2 apart modulo 32, so a wave's lanes, whose
    // stencils span a few columns and up to ~8 points along n, read disjoint
    // banks (measured: 0.136 -> 0.132 ms on the large final stage against
    // 2^lsh + 1).  A box too large at that stride takes 2^lsh + 1.
    static_assert(kFinalCS == 24, "the stride rule below is cs = 24 (mod 32)");
    TileBox b{lo[0], lo[1], lo[2], ni, nj, nl, lsh, ((1 << 22) + nj - 1) / nj, ((1 << 22) + nl - 1) / nl,
              nl + ((kFinalCS - nl) % 32 + 32) % 32};
    if (b.ni * b.nj * b.cs > kTileCap + kTileCap / 4) b.cs = (1 << lsh) + 1;
    return b;
}

// A box the final stage can stage: at most kTileCap values at 2^lsh per column,
// and its columns at stride cs within the kernel's kTileCap + kTileCap / 4 LDS
// values.
bool box_fits(const TileBox &b)
{
    return (b.ni * b.nj << b.lsh) <= kTileCap && b.ni * b.nj * b.cs <= kTileCap + kTileCap / 4;
}

void build_final_tiles(Plan &P)
{
    const hhffbp_config &c = P.cfg;
    const int64_t nx = c.grid_dims[0], ny = c.grid_dims[1], nz = c.grid_dims[2];
    const int64_t bx = (nx + kBrickX - 1) / kBrickX, by = (ny + kBrickY - 1) / kBrickY,
                  bz = (nz + kBrickZ - 1) / kBrickZ;
    const std::vector<int32_t> &d1 = P.compact_to_tree[P.F];
    const int64_t nc = (int64_t)d1.size();
    P.n_bricks = bx * by * bz;
    P.final_tiles.assign(P.n_bricks * nc, TileBox{0, 0, 0, 0, 0, 0, 0, 0, 0, 0});
    P.n_tiled = 0;
    if (!c.final_staging) return;
    std::vector<SubarrayMap> maps;
    for (int32_t ti : d1) maps.emplace_back(P.levels[P.F][ti].rect, P.kmin, P.kmax);
    const int T = P.T, slo = -(T / 2) + 1 - 1, shi = T / 2 + 1;
    std::atomic<int64_t> tiled{0};
    parallel_for(P.n_bricks, 16, [&](int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b) {
            const int64_t kx = b / (by * bz), ky = (b / bz) % by, kz = b % bz;
            for (int64_t ch = 0; ch < nc; ++ch) {
                const HostLattice &L = P.levels[P.F][d1[ch]].lat;
                int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
                for (int64_t ix = kx * kBrickX; ix < std::min(nx, (kx + 1) * kBrickX); ++ix)
                    for (int64_t iy = ky * kBrickY; iy < std::min(ny, (ky + 1) * kBrickY); ++iy)
                        for (int64_t iz = kz * kBrickZ; iz < std::min(nz, (kz + 1) * kBrickZ); ++iz) {
                            const double p[3] = {c.grid_origin[0] + ix * c.grid_pitch[0],
                                                 c.grid_origin[1] + iy * c.grid_pitch[1],
                                                 c.grid_origin[2] + iz * c.grid_pitch[2]};
                            double w[3];
                            maps[ch].eval(p, w, nullptr, nullptr);
                            for (int a = 0; a < 3; ++a) {
                                const int32_t t = (int32_t)std::floor(L.gamma[a] * w[a] + kStencilEps);
                                lo[a] = std::min(lo[a], t + slo);
                                hi[a] = std::max(hi[a], t + shi);
                            }
                        }
                lo[0] = std::max(lo[0], L.i0);
                hi[0] = std::min(hi[0], L.i0 + L.ni - 1);
                lo[1] = std::max(lo[1], L.j0);
                hi[1] = std::min(hi[1], L.j0 + L.nj - 1);
                const TileBox box = make_box(lo, hi);
                if (box.ni < T || box.nj < T || box.nl < T || !box_fits(box)) continue;
                P.final_tiles[b * nc + ch] = box;
                tiled.fetch_add(1);
            }
        }
    });
    P.n_tiled = tiled.load();
}

// Merge bricks of depth d: per node, kMBrickI x kMBrickJ column blocks of its
// grid, each cut into runs of kMBrickL steps over the union of its columns' n ranges.
void build_merge_bricks(Plan &P, int d)
{
    std::vector<MergeBrick> &bricks = P.merge_bricks[d];
    bricks.clear();
    for (int32_t ti : P.compact_to_tree[d]) {
        const HostNode &nd = P.levels[d][ti];
        const HostLattice &L = nd.lat;
        for (int32_t ib = 0; ib < L.ni; ib += kMBrickI)
            for (int32_t jb = 0; jb < L.nj; jb += kMBrickJ) {
                int32_t lmin = INT32_MAX, lmax = INT32_MIN;
                for (int32_t i = ib; i < std::min(L.ni, ib + kMBrickI); ++i)
                    for (int32_t j = jb; j < std::min(L.nj, jb + kMBrickJ); ++j) {
                        const int64_t cidx = (int64_t)i * L.nj + j;
                        if (L.hi[cidx] < L.lo[cidx]) continue;
                        lmin = std::min(lmin, L.lo[cidx]);
                        lmax = std::max(lmax, L.hi[cidx]);
                    }
                for (int32_t l = lmin; lmin <= lmax && l <= lmax; l += kMBrickL)
                    bricks.push_back(MergeBrick{nd.compact, L.i0 + ib, L.j0 + jb, l});
            }
    }
}

// Lane order of the forward merge at depth d (a wave takes 64 consecutive
// entries).  At d >= 2: storage order, runs along the pencils.  Onto the root's
// own lattice (d = 0) and onto depth 1: the points grouped in bricks of 2 x 8 x 4
// (d = 0) or 1 x 4 x 16 (d = 1) lattice steps (i, j, l), bricks in (i, j, l)
// order, points within a brick in (i, j, l) order.  There the children's frames are tilted most against the parent's
// (their centres are a quarter aperture off), so a run along one parent pencil
// crosses many child columns, and a compact group of points reaches fewer L1
// lines per gather instruction (measured on the large workload: 0.129 ms in
// storage order, 0.103 in 2 x 4 x 8 bricks, 0.100 in 2 x 8 x 4, the best of
// eleven shapes of 64 and 128 points).  Onto depth 1, 1 x 4 x 16 bricks: 0.098 ->
// 0.094 ms; at depths 2 and 3 the same shapes ran 1-2% slower than storage order.
void build_merge_order(Plan &P, int d)
{
    const int kBi = d == 0 ? 2 : 1, kBj = d == 0 ? 8 : 4, kBl = d == 0 ? 4 : 16;
    const std::vector<int32_t> &nodes = P.compact_to_tree[d];
    auto &out = P.merge_order[d];
    out.assign(nodes.size(), {});
    parallel_for((int64_t)nodes.size(), 1, [&](int64_t n0, int64_t n1) {
        for (int64_t n = n0; n < n1; ++n) {
            const HostLattice &L = P.levels[d][nodes[n]].lat;
            std::vector<int32_t> &o = out[n];
            o.resize((size_t)L.npts);
            if (d > 1) {
                for (int64_t k = 0; k < L.npts; ++k) o[k] = (int32_t)k;
                continue;
            }
            struct Key {
                int64_t k;
                int32_t p;
            };
            std::vector<Key> keys;
            keys.reserve((size_t)L.npts);
            int32_t lmin = INT32_MAX, lmax = INT32_MIN;
            for (size_t c = 0; c < L.lo.size(); ++c)
                if (L.hi[c] >= L.lo[c]) {
                    lmin = std::min(lmin, L.lo[c]);
                    lmax = std::max(lmax, L.hi[c]);
                }
            const int64_t nbj = (L.nj + kBj - 1) / kBj, nbl = (int64_t)(lmax - lmin) / kBl + 1;
            for (int32_t i = 0; i < L.ni; ++i)
                for (int32_t j = 0; j < L.nj; ++j) {
                    const int64_t c = (int64_t)i * L.nj + j;
                    for (int32_t l = L.lo[c]; l <= L.hi[c]; ++l) {
                        const int64_t dl = l - lmin;
                        const int64_t brick = ((int64_t)(i / kBi) * nbj + j / kBj) * nbl + dl / kBl;
                        const int64_t inner = ((i % kBi) * kBj + j % kBj) * kBl + dl % kBl;
                        keys.push_back(Key{brick * (kBi * kBj * kBl) + inner,
                                           (int32_t)(L.off[c] + (l - L.lo[c]))});
                    }
                }
            std::sort(keys.begin(), keys.end(), [](const Key &a, const Key &b) { return a.k < b.k; });
            if (keys.size() != o.size())
                throw Error{HHFFBP_E_NUMERIC, "merge order does not cover the node's points"};
            for (size_t k = 0; k < keys.size(); ++k) o[k] = keys[k].p;
        }
    });
}

// Fourier transform of the truncated ES kernel phi(t) = exp(beta (sqrt(1 - (2t/W)^2) - 1))
// on |t| <= W/2, at angular frequency theta (rad per bin); composite Simpson.
double es_hat(double theta, int W, double beta)
{
    const int n = 8000;
    const double a = 0.5 * W, h = a / n;
    double s = 0.0;
    for (int i = 0; i <= n; ++i) {
        const double t = i * h;
        const double z = t / a;
        const double v = std::exp(beta * (std::sqrt(std::max(0.0, 1.0 - z * z)) - 1.0)) *
                         std::cos(theta * t);
        const double wgt = (i == 0 || i == n) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
        s += wgt * v;
    }
    return 2.0 * s * h / 3.0;
}

double linear_hat(double theta)
{
    if (std::fabs(theta) < 1e-12) return 1.0;
    const double s = std::sin(0.5 * theta) / (0.5 * theta);
    return s * s;
}

// Range window and the pre-corrected DFT matrix of eq. (2) onto it.

// bfloat16 of x, rounded to nearest even (finite x), and back.
uint16_t bf16_rne(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

float bf16_value(uint16_t h)
{
    const uint32_t u = (uint32_t)h << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}

// The range-compression matrix for the split-bfloat16 GEMM: each entry split
// into three bfloat16 parts (x1 = rne(x), x2 = rne(x - x1), x3 = rne(x - x1 -
// x2)), in MFMA fragment order [k16 step][32-column tile][part][lane][8]: lane
// l holds column 32 tile + l mod 32 at k = 16 step + 8 (l div 32) + e, rows past
// K zero.
void split_gemm_matrix(Plan &P, int K, int N)
{
    const int KS = (K + 15) / 16, NT = N / 32;
    P.gemm_nt = NT;
    P.Bx.assign((size_t)KS * NT * 3 * 64 * 8, 0);
    for (int ks = 0; ks < KS; ++ks)
        for (int ct = 0; ct < NT; ++ct)
            for (int l = 0; l < 64; ++l)
                for (int e = 0; e < 8; ++e) {
                    const int k = 16 * ks + 8 * (l >> 5) + e, n = 32 * ct + (l & 31);
                    const float x = k < K ? P.Bmat[(size_t)k * N + n] : 0.0f;
                    const uint16_t h1 = bf16_rne(x);
                    const float r1 = x - bf16_value(h1);
                    const uint16_t h2 = bf16_rne(r1);
                    const uint16_t h3 = bf16_rne(r1 - bf16_value(h2));
                    const uint16_t h[3] = {h1, h2, h3};
                    for (int q = 0; q < 3; ++q)
                        P.Bx[((((size_t)ks * NT + ct) * 3 + q) * 64 + l) * 8 + e] = h[q];
                }
}

void range_setup(Plan &P, double rmin, double rmax)
{
    const double dk = P.kmax - P.kmin;
    P.dR = kPi / (P.U * dk);
    const int W = P.W;
    const double pad = (0.5 * W + 2.0) * P.dR;
    // the grid is anchored at R = 0 (samples at R_b = b dR), so the sampled
    // profile does not depend on how far the window reaches
    P.R0 = std::floor((rmin - pad) / P.dR) * P.dR;
    int64_t nr = (int64_t)std::ceil((rmax + pad - P.R0) / P.dR) + 1;
    nr = (nr + 31) / 32 * 32;
    P.Nr = nr;
    const int64_t nf = P.cfg.n_freq;
    P.Bmat.assign((size_t)(2 * nf) * (size_t)(2 * nr), 0.0f);
    P.Bdmat.assign((size_t)(2 * nf) * (size_t)(2 * nr), 0.0f);
    P.Badjmat.assign((size_t)(2 * nr) * (size_t)(2 * nf), 0.0f);
    for (int64_t f = 0; f < nf; ++f) {
        const double om = 2.0 * (P.k[f] - P.kc);
        const double corr = (P.kernel == HHFFBP_RANGE_ES) ? es_hat(om * P.dR, W, P.beta)
                                                         : linear_hat(om * P.dR);
        for (int64_t r = 0; r < nr; ++r) {
            const double ph = om * (P.R0 + r * P.dR);
            const double wr = std::cos(ph) / corr, wi = std::sin(ph) / corr;
            // block-real form of a complex matrix M acting on interleaved rows:
            // out.re += in.re M.re - in.im M.im, out.im += in.re M.im + in.im M.re
            auto put = [](std::vector<float> &B, int64_t ncol, int64_t a, int64_t b, double mr,
                          double mi) {
                B[(size_t)(2 * a) * ncol + 2 * b] = (float)mr;
                B[(size_t)(2 * a) * ncol + 2 * b + 1] = (float)mi;
                B[(size_t)(2 * a + 1) * ncol + 2 * b] = (float)(-mi);
                B[(size_t)(2 * a + 1) * ncol + 2 * b + 1] = (float)mr;
            };
            put(P.Bmat, 2 * nr, f, r, wr, wi);
            // range derivative of the compressed data: rows scaled by j 2 k_f
            const double s2k = 2.0 * P.k[f];
            put(P.Bdmat, 2 * nr, f, r, -s2k * wi, s2k * wr);
            // adjoint: grad_s[f] = sum_r conj(W[f][r]) gprof[r]
            put(P.Badjmat, 2 * nf, r, f, wr, -wi);
        }
    }
    if (P.cfg.storage == HHFFBP_C64 && P.cfg.range_gemm == HHFFBP_GEMM_SPLIT_BF16 && !P.cfg.range_fused)
        split_gemm_matrix(P, (int)(2 * nf), (int)(2 * nr));
}

// ---- band-limited interpolation weights -----------------------------------
// For signals band-limited to |omega| <= W per grid step, the weights w_a of
// the taps o_a = a - T/2 + 1 that minimise the squared error at offset x,
// integrated over the band, solve G w = b with
//   G_ab = int_{-W}^{W} cos(omega (o_a - o_b)) d omega,
//   b_a  = int_{-W}^{W} cos(omega (o_a - x)) d omega.
double band_integral(double W, double d)
{
    return std::fabs(d) < 1e-12 ? 2.0 * W : 2.0 * std::sin(W * d) / d;
}

void bandlimited_weights(int T, double W, double x, double *w)
{
    double L[kMaxTaps][kMaxTaps] = {}, y[kMaxTaps];
    // Cholesky factor of the (symmetric positive definite) Gram matrix
    for (int i = 0; i < T; ++i)
        for (int j = 0; j <= i; ++j) {
            double v = band_integral(W, (double)(i - j));
            for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(v > 0.0)) throw Error{HHFFBP_E_NUMERIC, "interpolation Gram matrix not positive"};
                L[i][i] = std::sqrt(v);
            } else {
                L[i][j] = v / L[j][j];
            }
        }
    for (int i = 0; i < T; ++i) {
        double v = band_integral(W, (double)(i - T / 2 + 1) - x);
        for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
        y[i] = v / L[i][i];
    }
    for (int i = T - 1; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < T; ++k) v -= L[k][i] * w[k];
        w[i] = v / L[i][i];
    }
}

// Weight of tap t at offset x from the fitted polynomials (mirror symmetry
// for the taps t >= T/2).
double interp_poly_weight(const InterpPoly &ip, int a, int T, int t, double x)
{
    const int s = (t < T / 2) ? t : T - 1 - t;
    const double y = (t < T / 2) ? x - 0.5 : 0.5 - x;
    double v = 0.0;
    for (int d = kPolyDeg; d >= 0; --d) v = v * y + (double)ip.c[a][s][d];
    return v;
}

// Degree-kPolyDeg least-squares polynomials in y = x - 1/2 (modified
// Gram-Schmidt QR at 40 Chebyshev nodes of [0, 1]) for the weights of the
// first T/2 taps of every axis; the mirror tap is the same polynomial at -y.
// Each fit, with its coefficients rounded to float, is checked against the
// exact weights at 257 offsets.
void fit_interp_poly(const Plan &P, const double *gamma, InterpPoly &ip)
{
    std::memset(&ip, 0, sizeof(ip));
    ip.kind = P.cfg.interp_kernel;
    if (ip.kind != HHFFBP_INTERP_BANDLIMITED) return;
    constexpr int K = 40, D = kPolyDeg + 1;
    const int T = P.T;
    double xk[K], V[K][D], R[D][D] = {};
    for (int k = 0; k < K; ++k) {
        xk[k] = 0.5 - 0.5 * std::cos(kPi * (k + 0.5) / K);
        double p = 1.0;
        for (int d = 0; d < D; ++d, p *= xk[k] - 0.5) V[k][d] = p;
    }
    for (int d = 0; d < D; ++d) {  // V = Q R, Q stored in V
        for (int e = 0; e < d; ++e) {
            double r = 0.0;
            for (int k = 0; k < K; ++k) r += V[k][e] * V[k][d];
            R[e][d] = r;
            for (int k = 0; k < K; ++k) V[k][d] -= r * V[k][e];
        }
        double nrm = 0.0;
        for (int k = 0; k < K; ++k) nrm += V[k][d] * V[k][d];
        R[d][d] = std::sqrt(nrm);
        for (int k = 0; k < K; ++k) V[k][d] /= R[d][d];
    }
    for (int a = 0; a < 3; ++a) {
        const double W = kPi / gamma[a];
        double wk[K][kMaxTaps];
        for (int k = 0; k < K; ++k) bandlimited_weights(T, W, xk[k], wk[k]);
        for (int t = 0; t < T / 2; ++t) {
            double qy[D], c[D];
            for (int d = 0; d < D; ++d) {
                qy[d] = 0.0;
                for (int k = 0; k < K; ++k) qy[d] += V[k][d] * wk[k][t];
            }
            for (int d = D - 1; d >= 0; --d) {
                double v = qy[d];
                for (int e = d + 1; e < D; ++e) v -= R[d][e] * c[e];
                c[d] = v / R[d][d];
            }
            for (int d = 0; d < D; ++d) ip.c[a][t][d] = (float)c[d];
        }
        for (int i = 0; i <= 256; ++i) {
            const double x = i / 256.0;
            double w[kMaxTaps];
            bandlimited_weights(T, W, x, w);
            for (int t = 0; t < T; ++t) {
                const double v = interp_poly_weight(ip, a, T, t, x);
                if (std::fabs(v - w[t]) > 1e-6)
                    throw Error{HHFFBP_E_NUMERIC, "band-limited weight fit above 1e-6"};
            }
        }
    }
}

// Distance range from points to a box (for the range window).
void box_dist(const double *q, const double *lo, const double *hi, double *dmin, double *dmax)
{
    double s0 = 0, s1 = 0;
    for (int a = 0; a < 3; ++a) {
        const double c = std::min(std::max(q[a], lo[a]), hi[a]);
        s0 += (q[a] - c) * (q[a] - c);
        const double f = std::max(std::fabs(q[a] - lo[a]), std::fabs(q[a] - hi[a]));
        s1 += f * f;
    }
    *dmin = std::sqrt(s0);
    *dmax = std::sqrt(s1);
}

// Per depth: gamma_u gamma_v gamma_n times the integral of |det J| over the
// voxel box, summed over the depth's non-empty nodes (Sec. IV-B's sample count
// of a subimage grid, eq. 4_subimgsmppresimp), by the midpoint rule on cells of
// s_a voxels per axis (at most 32 cells per axis).
void level_estimates(Plan &P)
{
    const hhffbp_config &c = P.cfg;
    P.level_estimate.assign(P.S + 1, 0.0);
    int64_t st[3], nc[3];
    for (int a = 0; a < 3; ++a) {
        st[a] = std::max<int64_t>(1, (c.grid_dims[a] + 31) / 32);
        nc[a] = (c.grid_dims[a] + st[a] - 1) / st[a];
    }
    std::vector<std::pair<int, int32_t>> nodes;  // (depth, tree index) of the non-empty nodes
    for (int d = 0; d <= P.S; ++d)
        for (int32_t ti = 0; ti < (int32_t)P.levels[d].size(); ++ti)
            if (!P.levels[d][ti].empty()) nodes.emplace_back(d, ti);
    std::vector<double> part(nodes.size(), 0.0);
    parallel_for((int64_t)nodes.size(), 1, [&](int64_t b0, int64_t b1) {
        for (int64_t q = b0; q < b1; ++q) {
            const SubarrayMap map(P.levels[nodes[q].first][nodes[q].second].rect, P.kmin, P.kmax);
            double acc = 0.0;
            for (int64_t i = 0; i < nc[0]; ++i)
                for (int64_t j = 0; j < nc[1]; ++j)
                    for (int64_t k = 0; k < nc[2]; ++k) {
                        // the cell [i s, min((i + 1) s, n)) along each axis, at its centre
                        const int64_t lo[3] = {i * st[0], j * st[1], k * st[2]};
                        double p[3], vol = 1.0;
                        for (int a = 0; a < 3; ++a) {
                            const int64_t n = std::min(st[a], c.grid_dims[a] - lo[a]);
                            p[a] = c.grid_origin[a] +
                                   ((double)lo[a] + 0.5 * (double)(n - 1)) * c.grid_pitch[a];
                            vol *= (double)n * c.grid_pitch[a];
                        }
                        double w[3], J[9];
                        map.eval(p, w, nullptr, J);
                        const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) -
                                           J[1] * (J[3] * J[8] - J[5] * J[6]) +
                                           J[2] * (J[3] * J[7] - J[4] * J[6]);
                        acc += std::fabs(det) * vol;
                    }
            part[(size_t)q] = acc;
        }
    });
    for (size_t q = 0; q < nodes.size(); ++q) {
        const double *g = P.gamma_of(nodes[q].first);
        P.level_estimate[nodes[q].first] += g[0] * g[1] * g[2] * part[q];
    }
}

void validate(const hhffbp_config &c)
{
    auto bad = [](const std::string &m) { throw Error{HHFFBP_E_INVALID, m}; };
    if (c.n_pos < 1) bad("n_pos must be >= 1");
    if (c.n_freq < 2) bad("n_freq must be >= 2");
    if (!c.positions || !c.freqs_hz) bad("positions and freqs_hz must be non-NULL");
    if (c.n_pos > (int64_t)INT32_MAX / 2) bad("n_pos too large");
    for (int a = 0; a < 3; ++a) {
        if (c.grid_dims[a] < 1) bad("grid_dims must be >= 1");
        if (!(c.grid_pitch[a] > 0) || !std::isfinite(c.grid_pitch[a])) bad("grid_pitch must be > 0");
        if (!std::isfinite(c.grid_origin[a])) bad("grid_origin must be finite");
        if (!(c.oversample[a] >= 1.0 && c.oversample[a] <= 8.0)) bad("oversample must be in [1, 8]");
        if (!(c.oversample_leaf[a] == 0.0 || (c.oversample_leaf[a] >= 1.0 && c.oversample_leaf[a] <= 8.0)))
            bad("oversample_leaf must be 0 or in [1, 8]");
    }
    if ((c.oversample_leaf[0] != 0.0 || c.oversample_leaf[1] != 0.0 || c.oversample_leaf[2] != 0.0) &&
        (c.oversample_leaf[0] == 0.0 || c.oversample_leaf[1] == 0.0 || c.oversample_leaf[2] == 0.0))
        bad("oversample_leaf: set all three axes or none");
    if (c.range_gemm != HHFFBP_GEMM_SPLIT_BF16 && c.range_gemm != HHFFBP_GEMM_F32)
        bad("range_gemm must be HHFFBP_GEMM_SPLIT_BF16 or HHFFBP_GEMM_F32");
    if (c.grid_dims[0] * c.grid_dims[1] * c.grid_dims[2] > ((int64_t)1 << 31))
        bad("grid too large");
    if (c.mode != HHFFBP_FACTORIZED && c.mode != HHFFBP_DIRECT_RC && c.mode != HHFFBP_DIRECT_EXACT)
        bad("unknown mode");
    if (c.stages < -8 || c.stages > 8) bad("stages must be in [-8, 8]");
    if (c.stages < 0 && c.mode != HHFFBP_FACTORIZED) bad("automatic stages need the factorised mode");
    if (c.merge_factor != 2 && c.merge_factor != 4) bad("merge_factor must be 2 or 4");
    if (c.interp_taps != 4 && c.interp_taps != 6) bad("interp_taps must be 4 or 6");
    if (c.final_staging != 0 && c.final_staging != 1) bad("final_staging must be 0 or 1");
    if (c.root_grid != 0 && c.root_grid != 1) bad("root_grid must be 0 or 1");
    if (c.range_fused != 0 && c.range_fused != 1) bad("range_fused must be 0 or 1");
    if (c.range_fused && (c.mode != HHFFBP_FACTORIZED || c.stages == 0 ||
                          c.range_kernel != HHFFBP_RANGE_LINEAR || c.storage != HHFFBP_C64))
        bad("range_fused needs the factorised mode with stages != 0, the linear range kernel "
            "and C64 storage");
    if (c.root_grid && (c.mode != HHFFBP_FACTORIZED || c.stages == 0))
        bad("a root grid needs the factorised mode with stages != 0");
    if (c.interp_kernel != HHFFBP_INTERP_LAGRANGE && c.interp_kernel != HHFFBP_INTERP_BANDLIMITED)
        bad("unknown interpolation kernel");
    if (c.range_kernel == HHFFBP_RANGE_ES) {
        if (c.range_taps < 4 || c.range_taps > 8) bad("range_taps must be in [4, 8]");
    } else if (c.range_kernel != HHFFBP_RANGE_LINEAR) {
        bad("unknown range_kernel");
    }
    if (!(c.range_oversample >= 1.5 && c.range_oversample <= 16.0))
        bad("range_oversample must be in [1.5, 16]");
    if (!(c.position_slack >= 0.0 && c.position_slack < 0.1)) bad("position_slack must be in [0, 0.1)");
    if (c.storage != HHFFBP_C64 && c.storage != HHFFBP_F16 && c.storage != HHFFBP_BF16)
        bad("unknown storage type");
    double zmax = -1e300;
    for (int64_t i = 0; i < 3 * c.n_pos; ++i)
        if (!std::isfinite(c.positions[i])) bad("positions must be finite");
    if (c.weights)
        for (int64_t i = 0; i < c.n_pos; ++i)
            if (!std::isfinite(c.weights[i])) bad("weights must be finite");
    for (int64_t i = 0; i < c.n_pos; ++i) zmax = std::max(zmax, c.positions[3 * i + 2]);
    for (int64_t f = 0; f < c.n_freq; ++f)
        if (!(c.freqs_hz[f] > 0) || !std::isfinite(c.freqs_hz[f])) bad("freqs_hz must be finite and > 0");
    if (!(c.grid_origin[2] > zmax + c.position_slack))
        bad("the voxel grid must lie in front of the aperture (z > max z' + slack)");
    if (c.mode == HHFFBP_FACTORIZED && c.stages > 0 && c.grid_origin[2] <= 0.0)
        bad("factorised imaging needs the grid at z > 0");
}

// Interpolation record of the pair (point p, child with map mc and grid Lc), with
// the parent's SDC phase phi_parent (0 in the final stage).  The lattice
// coordinates and stencil base are those build_lattice used to build Lc, so
// every stencil lies inside Lc's pencils; that is checked here.
void pair_record(const Plan &P, const SubarrayMap &mc, const HostLattice &Lc, const double *p,
                 double phi_parent, InterpIdx &ix, InterpGeo &g)
{
    double w[3], phic;
    mc.eval(p, w, &phic, nullptr);
    int32_t base[3];
    float frac[3];
    for (int a = 0; a < 3; ++a) {
        const double t = Lc.gamma[a] * w[a];
        const double b = std::floor(t + kStencilEps);
        base[a] = (int32_t)b;
        frac[a] = (float)(t - b);
    }
    const int h = P.T / 2 - 1;
    const int32_t ci0 = base[0] - h - Lc.i0, cj0 = base[1] - h - Lc.j0, l0 = base[2] - h;
    bool ok = ci0 >= 0 && ci0 + P.T <= Lc.ni && cj0 >= 0 && cj0 + P.T <= Lc.nj && Lc.ni < 65536 &&
              Lc.nj < 65536;
    for (int a = 0; ok && a < P.T; ++a)
        for (int b = 0; ok && b < P.T; ++b) {
            const int64_t c = (int64_t)(ci0 + a) * Lc.nj + (cj0 + b);
            ok = Lc.lo[c] <= l0 && l0 + P.T - 1 <= Lc.hi[c];
        }
    if (!ok) throw Error{HHFFBP_E_NUMERIC, "an interpolation stencil reaches outside its grid"};
    double turns = (phic - phi_parent) * (0.5 / kPi);
    turns -= std::rint(turns);
    ix.cij = (uint32_t)ci0 | ((uint32_t)cj0 << 16);
    ix.l0 = l0;
    g = InterpGeo{frac[0], frac[1], frac[2], (float)turns};
}

}  // namespace

// Records of the forward merge at depth d, in the order of its lanes: block k
// of `blocks` (a node's lane slots from `start`), thread t: wave t / 64 takes
// child (t / 64) mod Q of the point in slot start + (t / 64) / Q * 64 + t mod 64
// of the node's merge order.
void merge_records(const Plan &P, int d, const std::vector<BlockItem> &blocks,
                   std::vector<InterpIdx> &idx, std::vector<InterpGeo> &geo)
{
    const int nb = (int)blocks.size();
    idx.assign((size_t)nb * kBlockThreads, InterpIdx{kNoPair, 0});
    geo.assign((size_t)nb * kBlockThreads, InterpGeo{0, 0, 0, 0});
    std::vector<SubarrayMap> maps_c;
    std::vector<const HostLattice *> lats_c;
    for (int32_t ti : P.compact_to_tree[d + 1]) {
        maps_c.emplace_back(P.levels[d + 1][ti].rect, P.kmin, P.kmax);
        lats_c.push_back(&P.levels[d + 1][ti].lat);
    }
    parallel_for(nb, 16, [&](int64_t b0, int64_t b1) {
        for (int64_t k = b0; k < b1; ++k) {
            const BlockItem bk = blocks[k];
            const HostNode &hn = P.levels[d][P.compact_to_tree[d][bk.node]];
            const SubarrayMap mp(hn.rect, P.kmin, P.kmax);
            std::vector<int32_t> ch;  // compact indices of the non-empty children, in order
            for (int32_t c : hn.children)
                if (!P.levels[d + 1][c].empty()) ch.push_back(P.levels[d + 1][c].compact);
            const std::vector<int32_t> &ord = P.merge_order[d][bk.node];
            for (int t = 0; t < kBlockThreads; ++t) {
                const int wave = t / 64, c = wave % P.Q;
                const int64_t slot = bk.start + (int64_t)(wave / P.Q) * 64 + t % 64;
                if (slot >= hn.lat.npts || c >= (int)ch.size()) continue;
                const int64_t p = ord[slot];
                const double *x = &hn.lat.xyz[3 * p];
                if (!std::isfinite(x[2])) continue;  // absent parent point: value 0
                double w[3], phip;
                mp.eval(x, w, &phip, nullptr);
                pair_record(P, maps_c[ch[c]], *lats_c[ch[c]], x, phip, idx[k * kBlockThreads + t],
                            geo[k * kBlockThreads + t]);
            }
        }
    });
}

// Records of the final stage: brick b (as the final kernel numbers them), node c
// of depth F, lane t: voxel (kx 4 + t / 64, ky 8 + (t / 8) mod 8, kz 8 + t mod 8).
// With final-stage staging on, every (brick, node) box becomes the hull of the
// stencils its records use (also where the margin box was too large to stage);
// a box no record uses is dropped, and one that would exceed kTileCap keeps no
// box (its lanes gather from the pencils).
void tighten_final_tiles(Plan &P, const std::vector<InterpIdx> &ridx, int64_t nc)
{
    if (!P.cfg.final_staging) return;
    const int T = P.T;
    std::atomic<int64_t> tiled{0};
    parallel_for(P.n_bricks * nc, 64, [&](int64_t b0, int64_t b1) {
        for (int64_t bc = b0; bc < b1; ++bc) {
            TileBox &tb = P.final_tiles[bc];
            const HostLattice &Lc = P.levels[P.F][P.compact_to_tree[P.F][bc % nc]].lat;
            int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
            for (int t = 0; t < kBlockThreads; ++t) {
                const InterpIdx ix = ridx[(size_t)bc * kBlockThreads + t];
                if (ix.cij == kNoPair) continue;
                const int32_t s0[3] = {(int32_t)(ix.cij & 0xffffu) + Lc.i0, (int32_t)(ix.cij >> 16) + Lc.j0,
                                       ix.l0};
                for (int a = 0; a < 3; ++a) {
                    lo[a] = std::min(lo[a], s0[a]);
                    hi[a] = std::max(hi[a], s0[a] + T - 1);
                }
            }
            if (lo[0] > hi[0]) {
                tb = TileBox{0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
                continue;
            }
            const TileBox nb = make_box(lo, hi);
            if (!box_fits(nb)) {
                tb = TileBox{0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
                continue;
            }
            tb = nb;
            tiled.fetch_add(1);
        }
    });
    P.n_tiled = tiled.load();
}

void final_records(const Plan &P, std::vector<InterpIdx> &idx, std::vector<InterpGeo> &geo)
{
    const hhffbp_config &c = P.cfg;
    const int64_t nx = c.grid_dims[0], ny = c.grid_dims[1], nz = c.grid_dims[2];
    const int64_t by = (ny + kBrickY - 1) / kBrickY, bz = (nz + kBrickZ - 1) / kBrickZ;
    const std::vector<int32_t> &nodes = P.compact_to_tree[P.F];
    const int64_t nc = (int64_t)nodes.size();
    idx.assign((size_t)(P.n_bricks * nc) * kBlockThreads, InterpIdx{kNoPair, 0});
    geo.assign((size_t)(P.n_bricks * nc) * kBlockThreads, InterpGeo{0, 0, 0, 0});
    std::vector<SubarrayMap> maps;
    for (int32_t ti : nodes) maps.emplace_back(P.levels[P.F][ti].rect, P.kmin, P.kmax);
    parallel_for(P.n_bricks, 16, [&](int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b) {
            const int64_t kx = b / (by * bz), ky = (b / bz) % by, kz = b % bz;
            for (int t = 0; t < kBlockThreads; ++t) {
                const int64_t ix = kx * kBrickX + t / (kBrickY * kBrickZ),
                              iy = ky * kBrickY + (t / kBrickZ) % kBrickY, iz = kz * kBrickZ + t % kBrickZ;
                if (ix >= nx || iy >= ny || iz >= nz) continue;
                const double p[3] = {c.grid_origin[0] + ix * c.grid_pitch[0],
                                     c.grid_origin[1] + iy * c.grid_pitch[1],
                                     c.grid_origin[2] + iz * c.grid_pitch[2]};
                for (int64_t ch = 0; ch < nc; ++ch) {
                    const size_t r = (size_t)((b * nc + ch) * kBlockThreads + t);
                    pair_record(P, maps[ch], P.levels[P.F][nodes[ch]].lat, p, 0.0, idx[r], geo[r]);
                }
            }
        }
    });
}

// ---------------------------------------------------------------------------
// Sec. IV-B counts the operations of HHFFBPA as C1 N_A N_f log N_f (range
// compression) + C2 sum_n N_SA,n N_s,n (level-1 BP) + 2 C3 sum_m,n N_s,m,n
// (interpolation) and leaves the number of levels to a trade between cost and
// interpolation error.  With stages = -K the plan takes the S in 1..K that
// minimises that count on each candidate's exact pair counts (the range
// compression term does not depend on S), with per-pair costs measured on
// MI355X with this build (large workload, S = 4 with a root grid, band-limited
// weights, complex64): level-1 BP 0.71 ps (linear range kernel) or 2.24 ps (ES);
// interpolation per (point, child) pair, merges and final stage alike, 20.2 ps
// (T = 4) or 56.6 ps (T = 6).
double model_seconds(const Plan &P)
{
    const double c2 = (P.kernel == HHFFBP_RANGE_ES) ? 2.24e-12 : 0.71e-12;
    const double c3 = (P.T == 4) ? 20.2e-12 : 56.6e-12;
    return c2 * (double)P.leaf_pairs + c3 * (double)(P.merge_pairs + P.final_pairs);
}

void choose_stages(hhffbp_config &c)
{
    if (c.stages >= 0) return;
    validate(c);
    const int kmax = -c.stages;
    int best = 1;
    double best_cost = 0.0;
    for (int s = 1; s <= kmax; ++s) {
        Plan t;
        t.cfg = c;
        t.cfg.stages = s;
        t.cfg.device = -1;
        build_plan_host(t);
        const double cost = model_seconds(t);
        if (s == 1 || cost < best_cost) {
            best = s;
            best_cost = cost;
        }
    }
    c.stages = best;
}

void build_plan_host(Plan &P)
{
    auto t0 = std::chrono::steady_clock::now();
    const hhffbp_config &c = P.cfg;
    validate(c);
    P.S = (c.mode == HHFFBP_FACTORIZED) ? c.stages : 0;
    P.F = (c.root_grid && P.S > 0) ? 0 : 1;
    P.Q = c.merge_factor;
    P.T = c.interp_taps;
    for (int a = 0; a < 3; ++a) {
        P.gamma[a] = c.oversample[a];
        P.gamma_leaf[a] = c.oversample_leaf[a] > 0.0 ? c.oversample_leaf[a] : c.oversample[a];
    }
    P.kernel = c.range_kernel;
    P.W = (c.range_kernel == HHFFBP_RANGE_ES) ? c.range_taps : 2;
    P.U = c.range_oversample;
    P.beta = kPi * P.W * (1.0 - 1.0 / (2.0 * P.U)) * 0.98;
    fit_interp_poly(P, P.gamma, P.ipoly);
    fit_interp_poly(P, P.gamma_leaf, P.ipoly_leaf);
    P.positions.assign(c.positions, c.positions + 3 * c.n_pos);
    P.weights.clear();
    if (c.weights) P.weights.assign(c.weights, c.weights + c.n_pos);
    P.k.resize(c.n_freq);
    for (int64_t f = 0; f < c.n_freq; ++f) P.k[f] = 2.0 * kPi * c.freqs_hz[f] / kLight;
    P.kmin = *std::min_element(P.k.begin(), P.k.end());
    P.kmax = *std::max_element(P.k.begin(), P.k.end());
    if (!(P.kmax > P.kmin)) throw Error{HHFFBP_E_INVALID, "need at least two distinct frequencies"};
    P.kc = 0.5 * (P.kmin + P.kmax);
    {
        const int64_t nf = c.n_freq;
        P.k0 = P.k[0];
        P.dk = (P.k[nf - 1] - P.k[0]) / (double)(nf - 1);
        P.k_equispaced = P.dk != 0.0;
        for (int64_t f = 0; f < nf && P.k_equispaced; ++f)
            P.k_equispaced = std::fabs(P.k[f] - (P.k0 + (double)f * P.dk)) <= 1e-9 * std::fabs(P.dk);
    }

    partition(P);
    const int S = P.S;

    // voxel centres, float64
    const int64_t nx = c.grid_dims[0], ny = c.grid_dims[1], nz = c.grid_dims[2];
    std::vector<double> vox;
    if (S > 0) {
        vox.resize(3 * P.n_vox());
        for (int64_t ix = 0; ix < nx; ++ix)
            for (int64_t iy = 0; iy < ny; ++iy)
                for (int64_t iz = 0; iz < nz; ++iz) {
                    const int64_t v = (ix * ny + iy) * nz + iz;
                    vox[3 * v] = c.grid_origin[0] + ix * c.grid_pitch[0];
                    vox[3 * v + 1] = c.grid_origin[1] + iy * c.grid_pitch[1];
                    vox[3 * v + 2] = c.grid_origin[2] + iz * c.grid_pitch[2];
                }
    }
    // grid points whose preimage lies below half the lowest voxel plane are absent
    P.z_valid = 0.5 * c.grid_origin[2];
    // grids, top-down: depth d needs the points of depth d - 1, depth F the voxels
    for (int d = P.F; d <= S; ++d) {
        for (auto &node : P.levels[d]) {
            if (node.empty()) continue;
            const std::vector<double> &ppts =
                (d == P.F) ? vox : P.levels[d - 1][node.parent].lat.xyz;
            build_lattice(P, node, ppts);
        }
    }
    // compact indices, leaf-sorted positions
    P.compact_to_tree.assign(S + 1, {});
    P.depth_points.assign(S + 1, 0);
    for (int d = 0; d <= S; ++d) {
        for (size_t i = 0; i < P.levels[d].size(); ++i) {
            HostNode &nd = P.levels[d][i];
            if (nd.empty()) continue;
            nd.compact = (int32_t)P.compact_to_tree[d].size();
            P.compact_to_tree[d].push_back((int32_t)i);
            P.depth_points[d] += nd.lat.npts;
        }
    }
    P.perm.clear();
    P.leaf_of_sorted.clear();
    P.leaf_centre.clear();
    P.leaf_reach = 0.0;
    for (int32_t ti : P.compact_to_tree[S]) {
        const HostNode &lf = P.levels[S][ti];
        const double xc = 0.5 * (lf.rect.x0 + lf.rect.x1), yc = 0.5 * (lf.rect.y0 + lf.rect.y1);
        for (int32_t m : lf.members) {
            P.perm.push_back(m);
            P.leaf_of_sorted.push_back(lf.compact);
            const double *pm = &P.positions[3 * m];
            P.leaf_reach = std::max(P.leaf_reach, std::sqrt((pm[0] - xc) * (pm[0] - xc) +
                                                            (pm[1] - yc) * (pm[1] - yc) + pm[2] * pm[2]));
        }
        P.leaf_centre.push_back(xc);
        P.leaf_centre.push_back(yc);
    }
    // a member moved by up to the slack per axis stays within this distance of its leaf centre
    P.leaf_reach += std::sqrt(3.0) * c.position_slack;

    // range window: all (point, position) distances the backprojection uses
    double rmin = std::numeric_limits<double>::max(), rmax = 0.0;
    const double slack = c.position_slack;
    auto member_box = [&](const HostNode &nd, double *lo, double *hi) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = 1e300;
            hi[a] = -1e300;
        }
        for (int32_t m : nd.members)
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], P.positions[3 * m + a] - slack);
                hi[a] = std::max(hi[a], P.positions[3 * m + a] + slack);
            }
    };
    if (S == 0) {
        double lo[3], hi[3];
        member_box(P.levels[0][0], lo, hi);
        // the voxel box's extreme distances to the position box
        for (int cx = 0; cx < 2; ++cx)
            for (int cy = 0; cy < 2; ++cy)
                for (int cz = 0; cz < 2; ++cz) {
                    const double q[3] = {c.grid_origin[0] + cx * (nx - 1) * c.grid_pitch[0],
                                         c.grid_origin[1] + cy * (ny - 1) * c.grid_pitch[1],
                                         c.grid_origin[2] + cz * (nz - 1) * c.grid_pitch[2]};
                    double dmn, dmx;
                    box_dist(q, lo, hi, &dmn, &dmx);
                    rmax = std::max(rmax, dmx);
                }
        // nearest approach: the grid's lowest plane to the position box
        const double zg = c.grid_origin[2];
        double s0 = std::max(0.0, zg - hi[2]);
        double gx0 = c.grid_origin[0], gx1 = gx0 + (nx - 1) * c.grid_pitch[0];
        double gy0 = c.grid_origin[1], gy1 = gy0 + (ny - 1) * c.grid_pitch[1];
        double ddx = std::max(0.0, std::max(lo[0] - gx1, gx0 - hi[0]));
        double ddy = std::max(0.0, std::max(lo[1] - gy1, gy0 - hi[1]));
        rmin = std::sqrt(s0 * s0 + ddx * ddx + ddy * ddy);
    } else {
        for (int32_t ti : P.compact_to_tree[S]) {
            const HostNode &lf = P.levels[S][ti];
            double lo[3], hi[3];
            member_box(lf, lo, hi);
            for (int64_t q = 0; q < lf.lat.npts; ++q) {
                if (!std::isfinite(lf.lat.xyz[3 * q + 2])) continue;
                double dmn, dmx;
                box_dist(&lf.lat.xyz[3 * q], lo, hi, &dmn, &dmx);
                rmin = std::min(rmin, dmn);
                rmax = std::max(rmax, dmx);
            }
        }
    }
    range_setup(P, rmin, rmax);

    // work accounting
    P.leaf_pairs = 0;
    P.merge_pairs = 0;
    P.final_pairs = 0;
    if (S == 0) {
        P.leaf_pairs = P.n_vox() * c.n_pos;
    } else {
        for (int32_t ti : P.compact_to_tree[S]) {
            const HostNode &lf = P.levels[S][ti];
            P.leaf_pairs += lf.lat.npts * (int64_t)lf.members.size();
        }
        P.merge_pairs_depth.assign(S + 1, 0);
        for (int d = P.F; d < S; ++d)
            for (int32_t ti : P.compact_to_tree[d]) {
                const HostNode &nd = P.levels[d][ti];
                int nch = 0;
                for (int32_t ch : nd.children) nch += P.levels[d + 1][ch].empty() ? 0 : 1;
                P.merge_pairs += nd.lat.npts * nch;
                P.merge_pairs_depth[d] += nd.lat.npts * nch;
            }
        level_estimates(P);
        P.final_pairs = P.n_vox() * (int64_t)P.compact_to_tree[P.F].size();
    }
    P.model_s = model_seconds(P);
    if (S > 0) build_final_tiles(P);  // with final_staging = 0 every box is left empty
    P.merge_bricks.assign(S + 1, {});
    for (int d = P.F; d < S; ++d) build_merge_bricks(P, d);
    P.merge_order.assign(S + 1, {});
    for (int d = P.F; d < S; ++d) build_merge_order(P, d);

    // workspace layout; profiles and subimages in the storage type
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t csz = (c.storage == HHFFBP_C64) ? 8 : 4;
    size_t off = 0;
    P.ws_prof = off;
    if (!c.range_fused)  // the fused level-1 BP keeps its profiles in LDS
        off += al((size_t)c.n_pos * P.Nr * 8);  // also the backward's float32 range-derivative profiles
    P.ws_posoff = off;
    off += al((size_t)c.n_pos * 16);
    P.ws_scales = off;
    off += al(64 * sizeof(float));
    P.ws_amax = off;
    off += al(kAbsmaxParts * sizeof(float));
    P.ws_vals.assign(S + 1, 0);
    for (int d = P.F; d <= S; ++d) {
        P.ws_vals[d] = off;
        off += al((size_t)P.depth_points[d] * csz);
    }
    P.ws_total = off;
    P.ws_gvals.assign(S + 1, 0);
    for (int d = P.F; d <= S; ++d) {
        P.ws_gvals[d] = off;
        off += al((size_t)P.depth_points[d] * 8);
    }
    P.ws_gprof = off;
    off += al((size_t)c.n_pos * P.Nr * 8);
    P.ws_gpos = off;
    off += al((size_t)c.n_pos * 16);
    P.ws_gmax = off;
    off += al((size_t)std::max<size_t>(1, P.compact_to_tree[S].size()) * sizeof(float));
    P.ws_total_bwd = off;

    // worst-case gain from the echoes to each stage (half-precision scales):
    // profiles <= sqrt(2) Nf max|W| max|w_i| max|s| (w_i the aperture weights); a leaf sums <= members x W taps of
    // them; a merge sums <= children x L_u L_v L_n (L_a the interpolation
    // kernel's largest absolute weight sum on [0, 1) along axis a: 1.25 (T = 4)
    // and 1.3906 (T = 6) for Lagrange; sampled from the fitted polynomials, with
    // a 1% margin, for the band-limited weights).
    {
        double wmax = 0.0;
        for (size_t i = 0; i < P.Bmat.size(); ++i) wmax = std::max(wmax, (double)std::fabs(P.Bmat[i]));
        // L_u L_v L_n of the weights that interpolate from grids with these polynomials
        auto weight_sums = [&](const InterpPoly &ip) {
            double lt = 1.0;
            for (int a = 0; a < 3; ++a) {
                double la = (P.T == 4) ? 1.25 : 1.40;
                if (ip.kind == HHFFBP_INTERP_BANDLIMITED) {
                    la = 0.0;
                    for (int i = 0; i <= 256; ++i) {
                        const double x = i / 256.0;
                        double sum = 0.0;
                        for (int t = 0; t < P.T; ++t) sum += std::fabs(interp_poly_weight(ip, a, P.T, t, x));
                        la = std::max(la, sum);
                    }
                    la *= 1.01;
                }
                lt *= la;
            }
            return lt;
        };
        P.scale_mult.assign(P.n_scales(), 0.0f);
        // the aperture weights scale each echo row before the range compression
        double wt = P.weights.empty() ? 1.0 : 0.0;
        for (float v : P.weights) wt = std::max(wt, (double)std::fabs(v));
        const double m0 = std::sqrt(2.0) * (double)c.n_freq * wmax * wt;
        P.scale_mult[0] = (float)m0;
        if (S > 0) {
            size_t mem_max = 0;
            for (int32_t ti : P.compact_to_tree[S]) mem_max = std::max(mem_max, P.levels[S][ti].members.size());
            double m = m0 * (double)mem_max * (double)P.W;
            P.scale_mult[S] = (float)m;
            for (int d = S - 1; d >= P.F; --d) {
                size_t nch = 0;
                for (int32_t ti : P.compact_to_tree[d]) nch = std::max(nch, P.levels[d][ti].children.size());
                m *= (double)nch * weight_sums(P.ipoly_for(d + 1));
                P.scale_mult[P.scale_slot(d)] = (float)m;
            }
        }
    }
    P.plan_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace hh

namespace hh {

// ---------------------------------------------------------------------------
namespace {

template <class T>
void upload_vec(size_t &total, void **dst, const std::vector<T> &v)
{
    *dst = nullptr;
    if (v.empty()) return;
    total += v.size() * sizeof(T);
    if (hipMalloc(dst, v.size() * sizeof(T)) != hipSuccess) {
        *dst = nullptr;
        throw Error{HHFFBP_E_NOMEM, "hipMalloc failed during plan upload"};
    }
    if (hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        throw Error{HHFFBP_E_DEVICE, "hipMemcpy failed during plan upload"};
}

// Workgroup -> leaf block of the level-1 BP.  The dispatcher deals workgroup b
// to XCD b mod 8; every block of one leaf is placed on one XCD, so the leaf's
// range profiles come from HBM once and from that XCD's L2 for its other
// blocks.  Leaves go to XCDs largest first, each to the least loaded one (work =
// blocks x positions); slots an XCD does not fill hold -1 (the workgroup exits).
std::vector<int32_t> leaf_block_order(const std::vector<BlockItem> &blocks,
                                      const std::vector<NodeDev> &leaves)
{
    constexpr int kXcds = 8;
    struct Run {
        int32_t first, count;
        double work;
    };
    std::vector<Run> runs;
    for (int32_t b = 0; b < (int32_t)blocks.size(); ++b) {
        if (b == 0 || blocks[b].node != blocks[b - 1].node) runs.push_back(Run{b, 0, 0.0});
        ++runs.back().count;
    }
    for (Run &r : runs) {
        const NodeDev &nd = leaves[blocks[r.first].node];
        r.work = (double)r.count * (double)std::max(1, nd.pos_end - nd.pos_begin);
    }
    std::stable_sort(runs.begin(), runs.end(), [](const Run &a, const Run &b) { return a.work > b.work; });
    std::vector<std::vector<int32_t>> lists(kXcds);
    std::vector<double> load(kXcds, 0.0);
    for (const Run &r : runs) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[x] += r.work;
        for (int32_t k = 0; k < r.count; ++k) lists[x].push_back(r.first + k);
    }
    size_t slots = 0;
    for (const auto &l : lists) slots = std::max(slots, l.size());
    std::vector<int32_t> order(slots * kXcds, -1);
    for (int x = 0; x < kXcds; ++x)
        for (size_t s = 0; s < lists[x].size(); ++s) order[s * kXcds + x] = lists[x][s];
    return order;
}

}  // namespace

void upload_plan(Plan &P)
{
    const int S = P.S;
    P.dev.nodes.assign(S + 1, nullptr);
    P.dev.cols.assign(S + 1, nullptr);
    P.dev.colbase.assign(S + 1, nullptr);
    P.dev.merge_blocks.assign(S + 1, nullptr);
    P.dev.merge_blocks_fwd.assign(S + 1, nullptr);
    P.dev.merge_bricks.assign(S + 1, nullptr);
    P.dev.merge_order.assign(S + 1, nullptr);
    P.dev.merge_rank.assign(S + 1, nullptr);
    P.dev.merge_idx.assign(S + 1, nullptr);
    P.dev.merge_geo.assign(S + 1, nullptr);
    P.n_blocks_merge.assign(S + 1, 0);
    P.n_blocks_merge_fwd.assign(S + 1, 0);
    P.device_bytes = 0;
    if (P.cfg.device < 0) return;  // host-only plan: geometry and sizes, no device tables
    if (hipSetDevice(P.cfg.device) != hipSuccess)
        throw Error{HHFFBP_E_DEVICE, "hipSetDevice failed"};
    DeviceBuffers &D = P.dev;
    upload_vec(P.device_bytes, &D.B, P.Bmat);
    if (!P.Bx.empty()) upload_vec(P.device_bytes, &D.Bx, P.Bx);
    upload_vec(P.device_bytes, &D.Bd, P.Bdmat);
    upload_vec(P.device_bytes, &D.Badj, P.Badjmat);
    upload_vec(P.device_bytes, &D.scale_mult, P.scale_mult);
    upload_vec(P.device_bytes, &D.perm, P.perm);
    upload_vec(P.device_bytes, &D.leaf_of_sorted, P.leaf_of_sorted);
    upload_vec(P.device_bytes, &D.leaf_centre, P.leaf_centre);
    upload_vec(P.device_bytes, &D.pos64, P.positions);
    upload_vec(P.device_bytes, &D.check_counts,
               std::vector<int32_t>((size_t)((P.cfg.n_pos + kBlockThreads - 1) / kBlockThreads), 0));
    if (!P.weights.empty()) upload_vec(P.device_bytes, &D.weights, P.weights);
    if (P.cfg.mode == HHFFBP_DIRECT_EXACT) {
        std::vector<float> kt(P.k.size());
        for (size_t f = 0; f < P.k.size(); ++f) kt[f] = (float)(P.k[f] / kPi);
        upload_vec(P.device_bytes, &D.kf, P.k);
        upload_vec(P.device_bytes, &D.kf_turns, kt);
    }
    // the range-compression GEMM's forms, for every mode that range-compresses
    if (prepare_forward(P) != hipSuccess)
        throw Error{HHFFBP_E_DEVICE, "split GEMM LDS opt-in failed"};
    if (S == 0) return;
    int32_t pos_cursor = 0;
    for (int d = P.F; d <= S; ++d) {
        std::vector<NodeDev> nodes;
        std::vector<ColEntry> cols;
        std::vector<int32_t> colbase;
        std::vector<BlockItem> blocks, blocks_fwd;
        std::vector<LeafPoint> lpts;
        std::vector<BinWindow> wins, fused_wins;
        std::vector<BlockItem> fused_blocks;
        int32_t vbase = 0, cbase = 0;
        for (int32_t ti : P.compact_to_tree[d]) {
            const HostNode &hn = P.levels[d][ti];
            const HostLattice &L = hn.lat;
            NodeDev nd{};
            nd.x0 = hn.rect.x0;
            nd.x1 = hn.rect.x1;
            nd.y0 = hn.rect.y0;
            nd.y1 = hn.rect.y1;
            nd.d2 = 4.0 * (nd.x1 - nd.x0) * (nd.x1 - nd.x0) + 4.0 * (nd.y1 - nd.y0) * (nd.y1 - nd.y0);
            nd.i0 = L.i0;
            nd.j0 = L.j0;
            nd.ni = L.ni;
            nd.nj = L.nj;
            nd.col_base = cbase;
            nd.val_base = vbase;
            nd.npts = (int32_t)L.npts;
            nd.nchild = 0;
            for (int a = 0; a < 4; ++a) nd.child[a] = -1;
            if (d < S) {
                for (int32_t ch : hn.children) {
                    const HostNode &cn = P.levels[d + 1][ch];
                    if (!cn.empty()) nd.child[nd.nchild++] = cn.compact;
                }
            }
            nd.pos_begin = nd.pos_end = 0;
            if (d == S) {
                nd.pos_begin = pos_cursor;
                pos_cursor += (int32_t)hn.members.size();
                nd.pos_end = pos_cursor;
            }
            for (int64_t c = 0; c < (int64_t)L.ni * L.nj; ++c)
            {
                cols.push_back(ColEntry{(int32_t)L.off[c], L.lo[c], L.hi[c], 0});
                colbase.push_back((int32_t)L.off[c] - L.lo[c]);
            }
            for (int32_t st = 0; st < nd.npts; st += 256) blocks.push_back(BlockItem{hn.compact, st});
            // the forward merge runs one lane per (point, child): 256 / Q points a block
            nd.fwd_block0 = (int32_t)blocks_fwd.size();
            for (int32_t st = 0; st < nd.npts; st += 256 / P.Q)
                blocks_fwd.push_back(BlockItem{hn.compact, st});
            if (d == S) {
                const SubarrayMap map(hn.rect, P.kmin, P.kmax);
                const double xc = 0.5 * (hn.rect.x0 + hn.rect.x1), yc = 0.5 * (hn.rect.y0 + hn.rect.y1);
                for (int64_t q = 0; q < L.npts; ++q) {
                    const double *pq = &L.xyz[3 * q];
                    if (!std::isfinite(pq[2])) {
                        // absent point: contributes nothing, evaluates to exactly 0
                        lpts.push_back(LeafPoint{0.0f, 0.0f, 1.0f, 0, 0.0f, 0.0f, 0.0f, 0});
                        continue;
                    }
                    const double dx = pq[0] - xc, dy = pq[1] - yc, dz = pq[2];
                    const double rc = std::sqrt(dx * dx + dy * dy + dz * dz);
                    const double t = (rc - P.R0) / P.dR;
                    const double fb = std::floor(t);
                    double w[3], phi;
                    map.eval(pq, w, &phi, nullptr);
                    const double ph = 2.0 * P.kc * rc - phi;
                    LeafPoint lp;
                    lp.dx = (float)dx;
                    lp.dy = (float)dy;
                    lp.dz = (float)dz;
                    lp.bin = (int32_t)fb;
                    lp.frac = (float)(t - fb);
                    lp.pre_re = (float)std::cos(ph);
                    lp.pre_im = (float)std::sin(ph);
                    lp.pad = 0;
                    lpts.push_back(lp);
                }
                // per block of 256 points: the bins its taps can reach.  With
                // |Delta R| <= reach (the leaf's largest |p' - c| plus slack), tau =
                // Delta R / dR + frac - W/2 lies in [-reach/dR - W/2, reach/dR + 1 - W/2)
                // and a point with bin b reads b + 1 + floor(tau) .. + W - 1.  One more
                // bin on each side covers float32 rounding of tau, so the level-1 BP
                // reads its taps without clamping tau (positions are clamped to the
                // slack box before).
                double reach = 0.0;
                for (int32_t m : hn.members) {
                    const double *pm = &P.positions[3 * m];
                    reach = std::max(reach, std::sqrt((pm[0] - xc) * (pm[0] - xc) +
                                                      (pm[1] - yc) * (pm[1] - yc) + pm[2] * pm[2]));
                }
                reach += std::sqrt(3.0) * P.cfg.position_slack;
                const int32_t mlo = (int32_t)std::floor(-reach / P.dR - 0.5 * P.W) - 1;
                const int32_t mhi = (int32_t)std::floor(reach / P.dR + 1.0 - 0.5 * P.W) + P.W;
                const int32_t Nr = (int32_t)P.Nr;
                // the window of the block of points [st, st + len)
                auto window = [&](int32_t st, int32_t len) {
                    int32_t blo = INT32_MAX, bhi = INT32_MIN;
                    for (int32_t q = st; q < std::min(nd.npts, st + len); ++q) {
                        if (!std::isfinite(L.xyz[3 * q + 2])) continue;
                        const int32_t b1 = lpts[vbase + q].bin + 1;
                        blo = std::min(blo, b1 + mlo);
                        bhi = std::max(bhi, b1 + mhi);
                    }
                    if (blo > bhi) {  // only absent points: any W bins
                        blo = 0;
                        bhi = P.W - 1;
                    }
                    blo = std::max(blo, 0);
                    bhi = std::min(bhi, Nr - 1);
                    if (bhi - blo + 1 < P.W) {
                        blo = std::max(0, std::min(blo, Nr - P.W));
                        bhi = blo + P.W - 1;
                    }
                    return BinWindow{blo, bhi - blo + 1};
                };
                // level-1 windows start at an even bin and span an even count (a
                // superset; Nr is even, so it stays within the profile): the kernel
                // stages complex64 bins two at a time in 16-byte loads
                for (int32_t st = 0; st < nd.npts; st += 256) {
                    BinWindow wv = window(st, 256);
                    const int32_t lo2 = wv.lo & ~1, hi2 = (wv.lo + wv.n - 1) | 1;
                    wins.push_back(BinWindow{lo2, hi2 - lo2 + 1});
                }
                if (P.cfg.range_fused)
                    for (int32_t st = 0; st < nd.npts; st += kFusedPoints) {
                        fused_blocks.push_back(BlockItem{hn.compact, st});
                        fused_wins.push_back(window(st, kFusedPoints));
                    }
            }
            vbase += nd.npts;
            cbase += L.ni * L.nj;
            nodes.push_back(nd);
        }
        upload_vec(P.device_bytes, &D.nodes[d], nodes);
        upload_vec(P.device_bytes, &D.cols[d], cols);
        upload_vec(P.device_bytes, &D.colbase[d], colbase);
        if (d < S) {
            upload_vec(P.device_bytes, &D.merge_blocks[d], blocks);
            P.n_blocks_merge[d] = (int64_t)blocks.size();
            upload_vec(P.device_bytes, &D.merge_blocks_fwd[d], blocks_fwd);
            upload_vec(P.device_bytes, &D.merge_bricks[d], P.merge_bricks[d]);
            {
                std::vector<int32_t> order, rank;
                for (const std::vector<int32_t> &o : P.merge_order[d]) {
                    const int32_t base = (int32_t)order.size();
                    order.insert(order.end(), o.begin(), o.end());
                    rank.resize(order.size());
                    for (size_t k = 0; k < o.size(); ++k) rank[base + o[k]] = (int32_t)k;
                }
                if ((int64_t)order.size() != P.depth_points[d])
                    throw Error{HHFFBP_E_NUMERIC, "merge order does not cover the depth's points"};
                upload_vec(P.device_bytes, &D.merge_order[d], order);
                upload_vec(P.device_bytes, &D.merge_rank[d], rank);
            }
            P.n_blocks_merge_fwd[d] = (int64_t)blocks_fwd.size();
            std::vector<InterpIdx> ridx;
            std::vector<InterpGeo> rgeo;
            merge_records(P, d, blocks_fwd, ridx, rgeo);
            upload_vec(P.device_bytes, &D.merge_idx[d], ridx);
            upload_vec(P.device_bytes, &D.merge_geo[d], rgeo);
        } else {
            upload_vec(P.device_bytes, &D.leafpts, lpts);
            upload_vec(P.device_bytes, &D.leaf_blocks, blocks);
            upload_vec(P.device_bytes, &D.leaf_wins, wins);
            upload_vec(P.device_bytes, &D.fused_blocks, fused_blocks);
            upload_vec(P.device_bytes, &D.fused_wins, fused_wins);
            P.n_blocks_fused = (int64_t)fused_blocks.size();
            P.fused_win_max = 0;
            for (const BinWindow &wv : fused_wins) P.fused_win_max = std::max(P.fused_win_max, wv.n);
            // the fused kernel's LDS: 16 echo rows of 2 Nf (rounded up to 4), 16
            // profiles over the widest window, 16 position offsets
            const size_t kp = (size_t)((2 * P.cfg.n_freq + 3) / 4 * 4);
            if (P.cfg.range_fused &&
                (kp * 16 + 16 * 2 * (size_t)P.fused_win_max) * 4 + 16 * 16 > 65536)
                throw Error{HHFFBP_E_UNSUPPORTED,
                            "range_fused: the echo rows and profile window exceed 64 KB of LDS"};
            P.n_blocks_leaf = (int64_t)blocks.size();
            const std::vector<int32_t> order = leaf_block_order(blocks, nodes);
            upload_vec(P.device_bytes, &D.leaf_order, order);
            P.n_blocks_leaf_phys = (int64_t)order.size();
            P.leaf_win_max = 0;
            for (const BinWindow &wv : wins) P.leaf_win_max = std::max(P.leaf_win_max, wv.n);
            // adjoint work items: each leaf's positions in groups of kAdjPos
            std::vector<BlockItem> ab;
            for (size_t li = 0; li < nodes.size(); ++li)
                for (int32_t p0 = nodes[li].pos_begin; p0 < nodes[li].pos_end; p0 += kAdjPos)
                    ab.push_back(BlockItem{(int32_t)li, p0});
            upload_vec(P.device_bytes, &D.adj_blocks, ab);
            P.n_blocks_adj = (int64_t)ab.size();
        }
    }
    {
        std::vector<InterpIdx> ridx;
        std::vector<InterpGeo> rgeo;
        final_records(P, ridx, rgeo);
        const int64_t nc = (int64_t)P.compact_to_tree[P.F].size();
        tighten_final_tiles(P, ridx, nc);
        // every pair's stencil inside its brick's LDS box: the final stage then
        // runs without the pencil path (fewer registers, no per-lane test)
        bool box_only = true;
        for (int64_t bc = 0; box_only && bc < P.n_bricks * nc; ++bc) {
            const TileBox &tb = P.final_tiles[bc];
            const int64_t c = bc % nc;
            const HostLattice &Lc = P.levels[P.F][P.compact_to_tree[P.F][c]].lat;
            for (int t = 0; t < kBlockThreads; ++t) {
                const InterpIdx ix = ridx[(size_t)bc * kBlockThreads + t];
                if (ix.cij == kNoPair) continue;
                const int64_t ti = (int64_t)(ix.cij & 0xffffu) + Lc.i0 - tb.i0,
                              tj = (int64_t)(ix.cij >> 16) + Lc.j0 - tb.j0, tl = (int64_t)ix.l0 - tb.l0;
                if (tb.ni <= 0 || ti < 0 || ti > tb.ni - P.T || tj < 0 || tj > tb.nj - P.T || tl < 0 ||
                    tl > tb.nl - P.T) {
                    box_only = false;
                    break;
                }
            }
        }
        P.final_box_only = box_only;
        P.final_cs = -1;
        P.final_box_vals = P.final_box_cols = 0;
        for (const TileBox &tb : P.final_tiles) {
            if (tb.ni <= 0) continue;
            if (P.final_cs < 0) P.final_cs = tb.cs;
            if (tb.cs != P.final_cs) P.final_cs = 0;
            P.final_box_vals = std::max(P.final_box_vals, (int64_t)tb.ni * tb.nj * tb.cs);
            P.final_box_cols = std::max(P.final_box_cols, (int64_t)tb.ni * tb.nj);
        }
        if (P.final_cs < 0) P.final_cs = 0;
        upload_vec(P.device_bytes, &D.final_tiles, P.final_tiles);
        upload_vec(P.device_bytes, &D.final_idx, ridx);
        upload_vec(P.device_bytes, &D.final_geo, rgeo);
    }
    // images at the plan's own positions read their leaf offsets from the plan,
    // formed once here by the same kernel that forms them for other positions
    upload_vec(P.device_bytes, &D.unit_scales, std::vector<float>((size_t)P.n_scales(), 1.0f));
    {
        const size_t bytes = (size_t)P.cfg.n_pos * sizeof(float4);
        if (hipMalloc(&D.posoff, bytes) != hipSuccess) {
            D.posoff = nullptr;
            throw Error{HHFFBP_E_NOMEM, "hipMalloc failed during plan upload"};
        }
        P.device_bytes += bytes;
        if (launch_prep(P, (const double *)D.pos64, (float4 *)D.posoff, nullptr) != hipSuccess ||
            hipStreamSynchronize(nullptr) != hipSuccess)
            throw Error{HHFFBP_E_DEVICE, "position offsets failed during plan upload"};
    }
    if (prepare_backward(P) != hipSuccess)
        throw Error{HHFFBP_E_DEVICE, "setting the level-1 adjoint's LDS limit failed"};
}

void release_plan(Plan &P)
{
    DeviceBuffers &D = P.dev;
    auto fr = [](void *&p) {
        if (p) (void)hipFree(p);
        p = nullptr;
    };
    fr(D.B);
    fr(D.Bx);
    fr(D.perm);
    fr(D.leaf_of_sorted);
    fr(D.leaf_centre);
    fr(D.pos64);
    fr(D.check_counts);
    fr(D.posoff);
    fr(D.unit_scales);
    fr(D.weights);
    fr(D.kf);
    fr(D.kf_turns);
    fr(D.leafpts);
    fr(D.leaf_blocks);
    fr(D.leaf_wins);
    fr(D.leaf_order);
    fr(D.fused_blocks);
    fr(D.fused_wins);
    fr(D.final_tiles);
    fr(D.adj_blocks);
    fr(D.Bd);
    fr(D.Badj);
    fr(D.scale_mult);
    fr(D.final_idx);
    fr(D.final_geo);
    for (auto *v : {&D.nodes, &D.cols, &D.colbase, &D.merge_blocks, &D.merge_blocks_fwd,
                    &D.merge_bricks, &D.merge_idx, &D.merge_geo, &D.merge_order, &D.merge_rank})
        for (auto &p : *v) fr(p);
}

}  // namespace hh
