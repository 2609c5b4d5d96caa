"""Oracle HHFFBPA (Sec. IV-A, Fig. algimp), float64, steps in the paper's order.

Test infrastructure (oracle).

1. Level-1 subimages: BPA of each leaf subarray on its grid G_{1,n}; the BPA
   value is the eq. (4) sum over the leaf's positions and all frequencies.
2. SDC (eq. sdc_mul): f' = f exp(-j Phi) with Phi of eq. sdc_phi.
3. Merge: the compressed child subimages are interpolated at the (u, v, n)
   coordinates of the parent's grid points, the SDC is reverted by
   exp(+j Phi_child), and the children are summed coherently
   (f_{m,n} = sum of its children, Fig. pcsffbp).  A parent below the root is
   compressed again with its own Phi before the next merge.
4. The root's grid is the user voxel grid; its sum is the image.  With the
   plan's root grid the root is merged onto its own compressed lattice like any
   other parent, and the image is that lattice interpolated at the voxels with
   the root's SDC reverted (one child, the root).

The level-1 sum is eq. (4) itself, or (``range_u``) the fast form: range
profiles sampled every dR = pi / (U (k_max - k_min)) on the grid R_b = b dR,
pre-corrected for the linear kernel, and read by linear interpolation.

The interpolation kernel (the paper does not name one) is separable over the
stencil b - T/2 + 1 .. b + T/2 on each axis, b = floor(t + 1e-9): the T-tap
Lagrange polynomial, or the least-squares weights for the grid's band
(``bandlimited_weights``).  With S = 0 the root is the single subarray and step 1 alone
gives eq. (4) on the voxels.
"""
from __future__ import annotations

import numpy as np

from . import geometry as G
from . import native
from .plan import lagrange_offsets, stencil_base


def lagrange_weights(x, T):
    """(N, T) weights of the T-point Lagrange interpolant at fractional x in [0, 1)."""
    nodes = lagrange_offsets(T).astype(float)
    w = np.ones((x.shape[0], T))
    for a in range(T):
        for m in range(T):
            if m != a:
                w[:, a] *= (x - nodes[m]) / (nodes[a] - nodes[m])
    return w


def bandlimited_weights(x, T, gamma):
    """(N, T) least-squares weights for signals band-limited to |omega| <= pi / gamma
    per lattice step: the compressed subimages have unit spectral support per
    LLT unit (Sec. III) and a grid with gamma points per unit.  For each x they
    minimise  int_{-W}^{W} |sum_a w_a e^{j omega a} - e^{j omega x}|^2 d omega,
    W = pi / gamma, over the taps a = -T/2+1 .. T/2: the normal equations
    G w = b with G_ab = int cos(omega (a - b)), b_a = int cos(omega (a - x))."""
    W = np.pi / float(gamma)
    o = lagrange_offsets(T).astype(float)

    def integral(d):  # int_{-W}^{W} cos(omega d) d omega
        d = np.asarray(d, float)
        small = np.abs(d) < 1e-12
        return np.where(small, 2 * W, 2 * np.sin(W * d) / np.where(small, 1.0, d))

    G = integral(o[:, None] - o[None, :])
    b = integral(o[None, :] - np.asarray(x, float)[:, None])
    return np.linalg.solve(G, b.T).T


def axis_weights(x, T, kernel, gamma):
    """Interpolation weights of one axis: "lagrange" or "bandlimited"."""
    if kernel == "lagrange":
        return lagrange_weights(x, T)
    if kernel == "bandlimited":
        return bandlimited_weights(x, T, gamma)
    raise ValueError(f"unknown interpolation kernel {kernel}")


def interpolate(lat, vals, t, T, chunk=1 << 17, kernel="lagrange", gamma=(3.0, 3.0, 3.5)):
    """Separable T^3-tap interpolation (Lagrange, or band-limited least squares
    with the grid's oversampling ``gamma`` per axis) of lattice values at t.

    Raises if a stencil reaches a point that the lattice does not hold (the
    grids are built so that this cannot happen); absent points hold 0.
    """
    out = np.zeros(t.shape[0], np.complex128)
    offs = lagrange_offsets(T)
    for c0 in range(0, t.shape[0], chunk):
        tc = t[c0:c0 + chunk]
        base = stencil_base(tc).astype(np.int64)
        frac = tc - base
        wu, wv, wn = (axis_weights(frac[:, a], T, kernel, gamma[a]) for a in range(3))
        acc = np.zeros(tc.shape[0], np.complex128)
        missing = np.zeros(tc.shape[0], bool)
        for a, da in enumerate(offs):
            ci = base[:, 0] + da - lat.i0
            for b, db in enumerate(offs):
                cj = base[:, 1] + db - lat.j0
                inside = (ci >= 0) & (ci < lat.ni) & (cj >= 0) & (cj < lat.nj)
                cic, cjc = np.where(inside, ci, 0), np.where(inside, cj, 0)
                lo, hi, of = lat.l_lo[cic, cjc], lat.l_hi[cic, cjc], lat.off[cic, cjc]
                for c, dc in enumerate(offs):
                    ll = base[:, 2] + dc
                    ok = inside & (ll >= lo) & (ll <= hi)
                    missing |= ~ok
                    idx = np.where(ok, of + ll - lo, 0)
                    acc += np.where(ok, wu[:, a] * wv[:, b] * wn[:, c] * vals[idx], 0.0)
        if missing.any():
            raise RuntimeError(f"{missing.sum()} interpolation stencils reach outside the grid")
        out[c0:c0 + tc.shape[0]] = acc
    return out


def range_step(kmin, kmax, U):
    """Range-sample spacing dR = pi / (U (k_max - k_min)): U-fold oversampling of
    the range profile's band (eq. 2)."""
    return np.pi / (U * (kmax - kmin))


def _bp(plan, positions, echoes, q, range_u):
    """The level-1 backprojection sum at points q: eq. (4) itself, or with
    ``range_u`` its range-compressed form with linear interpolation at U-fold
    oversampling (native.bp_rc_linear)."""
    if range_u is None:
        return native.bp_eq4(positions, plan.k, echoes, q)
    return native.bp_rc_linear(positions, plan.k, echoes, q,
                               range_step(plan.kmin, plan.kmax, range_u))


def leaf_bp(plan, node, echoes, positions, range_u=None):
    """Compressed level-1 subimage f'(q) = exp(-j Phi(q)) * eq.(4) over the leaf's positions."""
    lat = node.lattice
    q = lat.xyz[lat.valid]
    f = _bp(plan, positions[node.members], echoes[node.members], q, range_u)
    out = np.zeros(lat.size, np.complex128)
    out[lat.valid] = f * np.exp(-1j * G.phi(q, node.rect, plan.kmin, plan.kmax))
    return out


def leaf_bp_at(plan, node, echoes, positions, point_index, range_u=None):
    """The leaf subimage of ``leaf_bp`` at selected lattice points only (for
    sampled checks at sizes where whole subimages are too slow); absent points
    give 0."""
    lat = node.lattice
    sel = np.asarray(point_index, np.int64)
    out = np.zeros(sel.size, np.complex128)
    ok = lat.valid[sel]
    q = lat.xyz[sel[ok]]
    f = _bp(plan, positions[node.members], echoes[node.members], q, range_u)
    out[ok] = f * np.exp(-1j * G.phi(q, node.rect, plan.kmin, plan.kmax))
    return out


def resample(plan, node, vals, points):
    """exp(+j Phi_node) I_node((u, v, n)_node(points)): a node's compressed
    subimage, interpolated at ``points`` and with its SDC reverted."""
    g = plan.gamma_at(node.depth)
    t = g * G.uvn(points, node.rect, plan.kmin, plan.kmax)
    val = interpolate(node.lattice, vals, t, plan.taps, kernel=plan.kernel, gamma=g)
    return val * np.exp(1j * G.phi(points, node.rect, plan.kmin, plan.kmax))


def merge_at(plan, node, child_vals, points):
    """f_node(points) = sum_c exp(+j Phi_c) I_c((u, v, n)_c(points)) (uncompressed)."""
    d = node.depth
    acc = np.zeros(points.shape[0], np.complex128)
    for ci in node.children:
        child = plan.levels[d + 1][ci]
        if child.empty:
            continue
        acc += resample(plan, child, child_vals[(d + 1, ci)], points)
    return acc


def weighted(echoes, weights):
    """Echoes under the aperture measure of eq. (4): with weights w_i the
    integral over p' becomes sum_i w_i (...), the same as scaling s_i by w_i."""
    echoes = np.asarray(echoes, np.complex128)
    if weights is None:
        return echoes
    return echoes * np.asarray(weights, float)[:, None]


def image(plan, echoes, positions=None, keep=False, range_u=None, weights=None):
    """HHFFBPA image on the voxel grid, (nx, ny, nz) complex128.

    ``positions`` are the antenna positions used for backprojection (the plan's
    tree and grids stay as built).  With ``keep`` the compressed subimages of
    every node are returned as well, keyed by (depth, index).  ``range_u``
    selects the range-compressed, linearly interpolated level-1 sum (see ``_bp``).
    ``weights`` are the aperture weights of eq. (4) (None: 1).
    """
    levels = plan.levels
    if positions is None:
        raise ValueError("positions are required")
    positions = np.asarray(positions, float)
    echoes = weighted(echoes, weights)
    S = len(levels) - 1
    if S == 0:
        img = _bp(plan, positions, echoes, plan.voxels, range_u)
        return (img.reshape(plan.dims), {}) if keep else img.reshape(plan.dims)
    vals = {}
    for idx, node in enumerate(levels[S]):
        if not node.empty:
            vals[(S, idx)] = leaf_bp(plan, node, echoes, positions, range_u)
    for d in range(S - 1, -1 if plan.root_grid else 0, -1):
        for idx, node in enumerate(levels[d]):
            if node.empty:
                continue
            lat = node.lattice
            pts = lat.xyz[lat.valid]
            f = merge_at(plan, node, vals, pts)
            out = np.zeros(lat.size, np.complex128)
            out[lat.valid] = f * np.exp(-1j * G.phi(pts, node.rect, plan.kmin, plan.kmax))
            vals[(d, idx)] = out
    if plan.root_grid:
        img = resample(plan, levels[0][0], vals[(0, 0)], plan.voxels).reshape(plan.dims)
    else:
        img = merge_at(plan, levels[0][0], vals, plan.voxels).reshape(plan.dims)
    return (img, vals) if keep else img


def stencil_points(lat, t, T):
    """Point indices (unique, ascending) of every tap of the T^3 stencils around
    the lattice coordinates t (N, 3); raises if a tap lies outside the lattice."""
    base = stencil_base(t).astype(np.int64)
    offs = lagrange_offsets(T)
    out = []
    for da in offs:
        ci = base[:, 0] + da - lat.i0
        for db in offs:
            cj = base[:, 1] + db - lat.j0
            inside = (ci >= 0) & (ci < lat.ni) & (cj >= 0) & (cj < lat.nj)
            if not inside.all():
                raise RuntimeError("a stencil reaches outside the grid's columns")
            lo, hi, of = lat.l_lo[ci, cj], lat.l_hi[ci, cj], lat.off[ci, cj]
            for dc in offs:
                ll = base[:, 2] + dc
                if np.any((ll < lo) | (ll > hi)):
                    raise RuntimeError("a stencil reaches outside a grid pencil")
                out.append(of + ll - lo)
    return np.unique(np.concatenate(out)) if out else np.zeros(0, np.int64)


def image_at(plan, echoes, positions, voxel_index, range_u=None, weights=None, keep=False):
    """The HHFFBPA image of ``image`` at the voxels ``voxel_index`` (linear, z
    fastest) only.  The same steps in the same order, restricted to the grid
    points those voxels need: at each depth, from the root down, the points of
    every stencil that the needed points of the depth above reach (for depth 1,
    or the root's own grid, the voxels' stencils); then leaf sums at the
    needed leaf points, and merges at the needed points of each depth, from the
    leaves up.  Values no needed point reads are never formed (NaN in the work
    arrays, so that reading one would show in the result).  With ``keep`` also
    returns {(depth, node): (point indices, compressed values)} of every depth."""
    levels = plan.levels
    positions = np.asarray(positions, float)
    echoes = weighted(echoes, weights)
    S = len(levels) - 1
    vi = np.asarray(voxel_index, np.int64)
    vox = plan.voxels[vi]
    if S == 0:
        return _bp(plan, positions, echoes, vox, range_u)
    top = 0 if plan.root_grid else 1

    def coords(node, pts):
        return plan.gamma_at(node.depth) * G.uvn(pts, node.rect, plan.kmin, plan.kmax)

    need = {}
    for d in range(top, S + 1):
        for idx, node in enumerate(levels[d]):
            if node.empty:
                continue
            if d == top:
                pts = vox
            else:
                par = levels[d - 1][node.parent]
                sel = need[(d - 1, node.parent)]
                sel = sel[par.lattice.valid[sel]]
                pts = par.lattice.xyz[sel]
            need[(d, idx)] = stencil_points(node.lattice, coords(node, pts), plan.taps)

    def work_array(node, sel, values):
        lat = node.lattice
        a = np.where(lat.valid, np.nan, 0.0).astype(np.complex128)
        a[sel] = values
        return a

    vals = {}
    for idx, node in enumerate(levels[S]):
        if not node.empty:
            sel = need[(S, idx)]
            vals[(S, idx)] = work_array(node, sel,
                                        leaf_bp_at(plan, node, echoes, positions, sel, range_u))
    for d in range(S - 1, top - 1, -1):
        for idx, node in enumerate(levels[d]):
            if node.empty:
                continue
            lat = node.lattice
            sel = need[(d, idx)]
            ok = lat.valid[sel]
            pts = lat.xyz[sel[ok]]
            f = np.zeros(sel.size, np.complex128)
            f[ok] = merge_at(plan, node, vals, pts) * np.exp(
                -1j * G.phi(pts, node.rect, plan.kmin, plan.kmax))
            vals[(d, idx)] = work_array(node, sel, f)
    if plan.root_grid:
        img = resample(plan, levels[0][0], vals[(0, 0)], vox)
    else:
        img = merge_at(plan, levels[0][0], vals, vox)
    if not np.all(np.isfinite(img)):
        raise RuntimeError("a stencil read a grid value that was not formed")
    if keep:
        return img, {key: (sel, vals[key][sel]) for key, sel in need.items()}
    return img


def direct_bp(positions, freqs_hz, echoes, points, weights=None):
    """Plain eq. (4) at arbitrary points (float64), aperture weights w_i (None: 1)."""
    k = 2.0 * np.pi * np.asarray(freqs_hz, float) / 299792458.0
    return native.bp_eq4(positions, k, weighted(echoes, weights), points)


def direct_bp_linear(positions, freqs_hz, echoes, points, U):
    """Eq. (4) through range compression with linear interpolation at U-fold
    range oversampling (float64)."""
    k = 2.0 * np.pi * np.asarray(freqs_hz, float) / 299792458.0
    return native.bp_rc_linear(positions, k, echoes, points, range_step(k.min(), k.max(), U))


def nrmse(a, ref):
    a, ref = np.asarray(a).ravel(), np.asarray(ref).ravel()
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))
