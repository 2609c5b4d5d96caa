"""Oracle adjoint and trajectory gradient of HHFFBPA, float64 (test infrastructure).

The image is linear in the echoes, f = A s (Sec. IV-A: leaf BP, SDC, merges).
For a real loss L and the complex-gradient convention g = dL/dRe f + j dL/dIm f:

* echo gradient      grad_s = A^H g: the literal transpose of the oracle's steps,
                     in reverse order (final stage, merges, leaf BP);
* position gradient  dL/dp'_i = Re sum_q conj(G(q)) d f'(q)/d p'_i, where G is
                     the cotangent of the compressed leaf subimage f' and only the
                     leaf BP depends on p' (the tree and grids stay as planned).

For a leaf, f'(q) = exp(-j Phi(q)) sum_i sum_f s_if exp(j 2 k_f |q - p'_i|), so
both gradients of a leaf are eq. (4)'s adjoint and position derivative with the
weights w(q) = G(q) exp(+j Phi(q)).
"""
import numpy as np

from . import geometry as G
from . import native
from .hhffbp import axis_weights
from .plan import lagrange_offsets, stencil_base


def scatter_transpose(lat, t, T, coef, out, kernel="lagrange", gamma=(3.0, 3.0, 3.5)):
    """Transpose of ``hhffbp.interpolate``: out[tap] += w(tap) * coef for each point."""
    offs = lagrange_offsets(T)
    base = stencil_base(t).astype(np.int64)
    frac = t - base
    wu, wv, wn = (axis_weights(frac[:, a], T, kernel, gamma[a]) for a in range(3))
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
                if not ok.all():
                    raise RuntimeError("a stencil reaches outside the grid")
                idx = of + ll - lo
                np.add.at(out, idx, wu[:, a] * wv[:, b] * wn[:, c] * coef)


def _split_to_children(plan, node, points, cot, phi_parent, child_cot):
    """Cotangent of f_node at `points` (uncompressed sum over children) -> children."""
    d = node.depth
    for ci in node.children:
        child = plan.levels[d + 1][ci]
        if child.empty:
            continue
        g = plan.gamma_at(d + 1)
        t = g * G.uvn(points, child.rect, plan.kmin, plan.kmax)
        ph = G.phi(points, child.rect, plan.kmin, plan.kmax) - phi_parent
        acc = child_cot.setdefault((d + 1, ci), np.zeros(child.lattice.size, np.complex128))
        scatter_transpose(child.lattice, t, plan.taps, np.exp(-1j * ph) * cot, acc,
                          kernel=plan.kernel, gamma=g)


def leaf_cotangents(plan, grad_image):
    """Cotangents G of every node's compressed subimage, from the image cotangent."""
    levels = plan.levels
    S = len(levels) - 1
    g = np.asarray(grad_image, np.complex128).ravel()
    cot = {}
    if S == 0:
        return cot
    if plan.root_grid:
        # transpose of the last resample: image = exp(+j Phi_root) I_root(voxels)
        root = levels[0][0]
        g0 = plan.gamma_at(0)
        t = g0 * G.uvn(plan.voxels, root.rect, plan.kmin, plan.kmax)
        ph = G.phi(plan.voxels, root.rect, plan.kmin, plan.kmax)
        cot[(0, 0)] = np.zeros(root.lattice.size, np.complex128)
        scatter_transpose(root.lattice, t, plan.taps, np.exp(-1j * ph) * g, cot[(0, 0)],
                          kernel=plan.kernel, gamma=g0)
        first = 0
    else:
        _split_to_children(plan, levels[0][0], plan.voxels, g, 0.0, cot)
        first = 1
    for d in range(first, S):
        for idx, node in enumerate(levels[d]):
            if node.empty:
                continue
            lat = node.lattice
            c = cot.get((d, idx), np.zeros(lat.size, np.complex128))
            v = lat.valid
            pts = lat.xyz[v]
            # f'_P = exp(-j Phi_P) f_P: the cotangent of f_P is exp(+j Phi_P) * cot(f'_P);
            # children see exp(-j Phi_c) of that, i.e. exp(-j (Phi_c - Phi_P)) cot(f'_P)
            _split_to_children(plan, node, pts, c[v], G.phi(pts, node.rect, plan.kmin, plan.kmax),
                               cot)
    return cot


def echo_gradient(plan, grad_image, positions, weights=None):
    """grad_s = A^H g, (n_pos, n_f) complex128; with aperture weights w_i row i
    of A carries w_i, so row i of the result does too."""
    g = _echo_gradient(plan, grad_image, positions)
    return g if weights is None else g * np.asarray(weights, float)[:, None]


def _echo_gradient(plan, grad_image, positions):
    positions = np.asarray(positions, float)
    n_pos, n_f = positions.shape[0], plan.k.shape[0]
    S = len(plan.levels) - 1
    out = np.zeros((n_pos, n_f), np.complex128)
    if S == 0:
        return native.bp_eq4_adjoint(positions, plan.k, plan.voxels, grad_image)
    cot = leaf_cotangents(plan, grad_image)
    for idx, node in enumerate(plan.levels[S]):
        if node.empty or (S, idx) not in cot:
            continue
        lat = node.lattice
        v = lat.valid
        q = lat.xyz[v]
        w = cot[(S, idx)][v] * np.exp(1j * G.phi(q, node.rect, plan.kmin, plan.kmax))
        out[node.members] = native.bp_eq4_adjoint(positions[node.members], plan.k, q, w)
    return out


def position_gradient(plan, echoes, positions, grad_image, weights=None):
    """dL/dp' for L with image cotangent g, (n_pos, 3) float64 (aperture
    weights w_i scale position i's terms, as they scale its echoes)."""
    positions = np.asarray(positions, float)
    echoes = np.asarray(echoes, np.complex128)
    if weights is not None:
        echoes = echoes * np.asarray(weights, float)[:, None]
    S = len(plan.levels) - 1
    if S == 0:
        return native.bp_eq4_dpos(positions, plan.k, echoes, plan.voxels, grad_image)
    out = np.zeros_like(positions)
    cot = leaf_cotangents(plan, grad_image)
    for idx, node in enumerate(plan.levels[S]):
        if node.empty or (S, idx) not in cot:
            continue
        lat = node.lattice
        v = lat.valid
        q = lat.xyz[v]
        w = cot[(S, idx)][v] * np.exp(1j * G.phi(q, node.rect, plan.kmin, plan.kmax))
        m = node.members
        out[m] = native.bp_eq4_dpos(positions[m], plan.k, echoes[m], q, w)
    return out
