"""Oracle plan for HHFFBPA: subarray tree, sampling grids G_{m,n}, preimages.

Test infrastructure (oracle), float64 throughout.

Readings of what the paper leaves open (Sec. IV-A and Fig. pcsffbp):

* Partition.  The aperture's (x', y') bounding box is bisected at its midpoint,
  one x and one y split per stage for merge factor Q = 4 (two of the paper's
  binary levels fused), alternating axes starting with the longer one for
  Q = 2.  A position with x' >= mid goes to the upper cell.  A node's rectangle
  is its cell; a node without positions has a zero subimage and no grid.
* Grid G_{m,n}.  Uniform in (u, v, n) with spacing 1/gamma per axis; the point
  (i, j, l) sits at (u, v, n) = (i, j, l) / gamma.  The grid of a node holds
  exactly the points its parent needs: for every point of the parent's grid
  (for the root: every user voxel) the T-tap interpolation stencil around the
  point's (u, v, n) in the child, optionally widened by ``margin`` points on
  every side, then closed along n into one contiguous pencil per (i, j) column.
  Built from the root downwards, so no stencil ever reaches a missing point.
  The spacing may differ per axis: (u, v, n) = (i/gamma_u, j/gamma_v, l/gamma_n).
* Root grid (optional).  The root's grid is the user voxel grid.  With
  ``root_grid`` the root gets a compressed lattice of its own, built like every
  other grid (the stencils of the voxels in the root's (u, v, n), i.e. with the
  full aperture's rectangle), the depth-1 grids are built from its points, and
  one more single-child resample carries it to the voxels.  Where the voxel
  grid is finer than the full aperture's band needs, that lattice has fewer
  points than the voxels, so the last merge does fewer interpolations.
* Conversion (u, v, n) -> (x, y, z).  Newton's method with the analytic
  Jacobian of eq. uvw_xyz, to 1e-12 m, from a boresight starting point.  A
  stencil of a point seen at a grazing angle can reach (u, v, n) beyond the
  image of the scene half-space; a grid point whose preimage is not found at
  z >= half the lowest voxel z is absent: it holds the value 0 (the paper's
  grids are silent on this; absent samples are read as zero).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import geometry as G

C0 = 299792458.0


@dataclasses.dataclass
class Lattice:
    i0: int
    j0: int
    l_lo: np.ndarray     # (ni, nj) int64; an empty column has l_hi < l_lo
    l_hi: np.ndarray     # (ni, nj) int64
    off: np.ndarray      # (ni, nj) int64, start of each column in point order
    ijl: np.ndarray      # (M, 3) int64 lattice indices, columns i-major, then j, then l
    xyz: np.ndarray      # (M, 3) float64 preimages (NaN where absent)
    valid: np.ndarray    # (M,) bool: the point has a preimage and holds a value

    @property
    def ni(self):
        return self.l_lo.shape[0]

    @property
    def nj(self):
        return self.l_lo.shape[1]

    @property
    def size(self):
        return self.ijl.shape[0]


@dataclasses.dataclass
class Node:
    depth: int                 # 0 = full aperture (final image); S = leaves
    rect: tuple                # (x0, x1, y0, y1) cell rectangle
    members: np.ndarray        # position indices
    children: list             # indices into the next depth's node list
    parent: int                # index into the previous depth's list (-1 for the root)
    lattice: Lattice | None = None

    @property
    def empty(self):
        return self.members.size == 0


def partition(positions, stages, merge_factor):
    """Subarray tree as a list of levels; levels[d] holds the nodes at depth d."""
    if merge_factor not in (2, 4):
        raise ValueError("merge factor must be 2 or 4")
    xy = np.asarray(positions, float)[:, :2]
    x0, y0 = xy.min(0)
    x1, y1 = xy.max(0)
    if not (x1 > x0 and y1 > y0):
        raise ValueError("aperture has zero extent along x' or y'")
    first_axis = 0 if (x1 - x0) >= (y1 - y0) else 1
    levels = [[Node(0, (x0, x1, y0, y1), np.arange(xy.shape[0]), [], -1)]]
    for d in range(stages):
        nxt = []
        for pi, node in enumerate(levels[d]):
            a0, a1, b0, b1 = node.rect
            m = node.members
            if merge_factor == 4:
                xm, ym = 0.5 * (a0 + a1), 0.5 * (b0 + b1)
                up_x, up_y = xy[m, 0] >= xm, xy[m, 1] >= ym
                parts = [((a0, xm, b0, ym), ~up_x & ~up_y), ((a0, xm, ym, b1), ~up_x & up_y),
                         ((xm, a1, b0, ym), up_x & ~up_y), ((xm, a1, ym, b1), up_x & up_y)]
            else:
                axis = (first_axis + d) % 2
                if axis == 0:
                    xm = 0.5 * (a0 + a1)
                    up = xy[m, 0] >= xm
                    parts = [((a0, xm, b0, b1), ~up), ((xm, a1, b0, b1), up)]
                else:
                    ym = 0.5 * (b0 + b1)
                    up = xy[m, 1] >= ym
                    parts = [((a0, a1, b0, ym), ~up), ((a0, a1, ym, b1), up)]
            for rect, mask in parts:
                node.children.append(len(nxt))
                nxt.append(Node(d + 1, rect, m[mask], [], pi))
        levels.append(nxt)
    return levels


def lagrange_offsets(T):
    """Stencil offsets relative to the base index: -T/2+1 .. T/2."""
    return np.arange(-(T // 2) + 1, T // 2 + 1)


# Coordinates of a parent point in a child that shares an edge with it (Q = 2)
# fall on child grid nodes up to rounding; the base index is floor(t + EPS) so
# that every implementation picks the same stencil there.
STENCIL_EPS = 1e-9


def stencil_base(t):
    return np.floor(t + STENCIL_EPS)


def required_lattice(t, T, margin):
    """Pencil columns covering every T-tap stencil (plus margin) around the coordinates t.

    ``t`` is (N, 3) in lattice units (gamma * (u, v, n)).
    """
    base = stencil_base(t).astype(np.int64)
    lo = -(T // 2) + 1 - margin
    hi = T // 2 + margin
    bi, bj, bl = base[:, 0], base[:, 1], base[:, 2]
    bi0, bj0 = bi.min(), bj.min()
    nci, ncj = bi.max() - bi0 + 1, bj.max() - bj0 + 1
    big = np.iinfo(np.int64).max // 4
    cmin = np.full((nci, ncj), big, np.int64)
    cmax = np.full((nci, ncj), -big, np.int64)
    np.minimum.at(cmin, (bi - bi0, bj - bj0), bl)
    np.maximum.at(cmax, (bi - bi0, bj - bj0), bl)
    w = hi - lo
    lmin = np.full((nci + w, ncj + w), big, np.int64)
    lmax = np.full((nci + w, ncj + w), -big, np.int64)
    for di in range(w + 1):
        for dj in range(w + 1):
            sl = (slice(di, di + nci), slice(dj, dj + ncj))
            lmin[sl] = np.minimum(lmin[sl], cmin)
            lmax[sl] = np.maximum(lmax[sl], cmax)
    filled = lmin < big
    l_lo = np.where(filled, lmin + lo, 0)
    l_hi = np.where(filled, lmax + hi, -1)
    return int(bi0 + lo), int(bj0 + lo), l_lo, l_hi


def enumerate_points(i0, j0, l_lo, l_hi):
    cnt = np.maximum(l_hi - l_lo + 1, 0)
    off = np.concatenate([[0], np.cumsum(cnt.ravel())])[:-1].reshape(cnt.shape)
    ii, jj = np.meshgrid(np.arange(cnt.shape[0]), np.arange(cnt.shape[1]), indexing="ij")
    ci = np.repeat(ii.ravel(), cnt.ravel())
    cj = np.repeat(jj.ravel(), cnt.ravel())
    start = np.repeat(off.ravel(), cnt.ravel())
    ll = np.arange(ci.size) - start + np.repeat(l_lo.ravel(), cnt.ravel())
    ijl = np.stack([ci + i0, cj + j0, ll], axis=1).astype(np.int64)
    return off.astype(np.int64), ijl


def boresight_guess(w, rect, kmin, kmax):
    """Starting point for Newton: range from the boresight relation for n,
    direction cosines from u and v in the far-field approximation."""
    x0, x1, y0, y1 = rect
    xc, yc = 0.5 * (x0 + x1), 0.5 * (y0 + y1)
    lx, ly = x1 - x0, y1 - y0
    h2 = 0.25 * (lx * lx + ly * ly)
    pn = math.pi * w[:, 2]
    # kmax z - pi n = kmin sqrt(h^2 + z^2)  ->  quadratic in z
    a = kmax * kmax - kmin * kmin
    b = -2.0 * pn * kmax
    c = pn * pn - kmin * kmin * h2
    z = (-b + np.sqrt(np.maximum(b * b - 4 * a * c, 0.0))) / (2 * a)
    z = np.maximum(z, 1e-3)
    ax = np.clip(math.pi * w[:, 0] / (kmax * lx), -0.7, 0.7)
    ay = np.clip(math.pi * w[:, 1] / (kmax * ly), -0.7, 0.7)
    s = np.sqrt(np.maximum(1.0 - ax * ax - ay * ay, 0.1))
    R = z / s
    return np.stack([xc + R * ax, yc + R * ay, R * s], axis=1)


def invert_uvn(w, rect, kmin, kmax, z_valid, tol=1e-12, maxit=100):
    """Solve uvn(p) = w for p by damped Newton (float64).

    Returns (p, ok).  ``ok`` is False where no preimage with z >= z_valid was
    found; such grid points lie beyond the edge of the (u, v, n) image of the
    half-space in front of the aperture and hold no subimage value.
    """
    p = boresight_guess(w, rect, kmin, kmax)
    F = G.uvn(p, rect, kmin, kmax) - w
    nf = np.linalg.norm(F, axis=1)
    active = np.ones(w.shape[0], bool)
    for _ in range(maxit):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        J = G.jacobian(p[idx], rect, kmin, kmax)
        with np.errstate(all="ignore"):
            dp = np.linalg.solve(J, F[idx][:, :, None])[:, :, 0]
        dp = np.where(np.isfinite(dp), dp, 0.0)
        step = np.ones(idx.size)
        pn = p[idx] - dp
        for _ in range(40):
            pn = p[idx] - step[:, None] * dp
            pn[:, 2] = np.maximum(pn[:, 2], 1e-4)
            Fn = G.uvn(pn, rect, kmin, kmax) - w[idx]
            nfn = np.linalg.norm(Fn, axis=1)
            bad = ~(nfn <= nf[idx]) & (step * np.linalg.norm(dp, axis=1) > tol)
            if not bad.any():
                break
            step[bad] *= 0.5
        p[idx] = pn
        F[idx] = Fn
        nf[idx] = nfn
        done = step * np.linalg.norm(dp, axis=1) < tol
        active[idx[done]] = False
    ok = ~active & (nf < 1e-9) & (p[:, 2] >= z_valid)
    p[~ok] = np.nan
    return p, ok


@dataclasses.dataclass
class Plan:
    levels: list
    k: np.ndarray
    kmin: float
    kmax: float
    gamma: np.ndarray           # (3,) oversampling along u, v, n
    taps: int
    margin: int
    voxels: np.ndarray          # (N_vox, 3)
    dims: tuple
    kernel: str = "lagrange"    # interpolation weights: "lagrange" or "bandlimited"
    root_grid: bool = False     # the root holds a compressed lattice (see module notes)
    gamma_leaf: np.ndarray = None  # (3,) oversampling of the level-1 (leaf) grids; None: gamma

    def gamma_at(self, depth):
        """Oversampling of the grids at ``depth``: the leaf grids' own when set."""
        if self.gamma_leaf is not None and depth == len(self.levels) - 1:
            return self.gamma_leaf
        return self.gamma


def build_plan(positions, freqs_hz, origin, pitch, dims, stages, merge_factor,
               gamma=3.0, taps=4, margin=0, kernel="lagrange", root_grid=False, gamma_leaf=None):
    """Oracle plan: tree, top-down grids and their xyz preimages.  ``gamma_leaf``
    (optional) is the oversampling of the level-1 (leaf) grids; the other grids
    use ``gamma``."""
    from workloads import voxel_centres

    k = 2.0 * math.pi * np.asarray(freqs_hz, float) / C0
    kmin, kmax = float(k.min()), float(k.max())
    levels = partition(positions, stages, merge_factor)
    vox = voxel_centres(origin, pitch, dims)
    z_valid = 0.5 * float(vox[:, 2].min())
    gamma = np.broadcast_to(np.asarray(gamma, float), (3,)).copy()
    if kernel not in ("lagrange", "bandlimited"):
        raise ValueError(f"unknown interpolation kernel {kernel}")
    if root_grid and stages < 1:
        raise ValueError("a root grid needs at least one stage")
    if gamma_leaf is not None:
        gamma_leaf = np.broadcast_to(np.asarray(gamma_leaf, float), (3,)).copy()
    plan = Plan(levels, k, kmin, kmax, gamma, int(taps), int(margin), vox, tuple(dims), kernel,
                bool(root_grid), gamma_leaf)
    for d in range(0 if root_grid else 1, len(levels)):
        for node in levels[d]:
            if node.empty:
                continue
            if d == 0 or (d == 1 and not root_grid):
                ppts = vox
            else:
                parent = levels[d - 1][node.parent]
                ppts = parent.lattice.xyz[parent.lattice.valid]
            g = plan.gamma_at(d)
            t = g * G.uvn(ppts, node.rect, kmin, kmax)
            i0, j0, l_lo, l_hi = required_lattice(t, taps, margin)
            off, ijl = enumerate_points(i0, j0, l_lo, l_hi)
            xyz, ok = invert_uvn(ijl / g, node.rect, kmin, kmax, z_valid)
            node.lattice = Lattice(i0, j0, l_lo, l_hi, off, ijl, xyz, ok)
    return plan
