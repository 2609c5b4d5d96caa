"""Pins of the oracle HHFFBPA (CPU only).

HHFFBPA approximates eq. (4); the oracle is pinned to eq. (4) by:
* the special case S = 0 (one subarray whose grid is the voxel grid), which is
  eq. (4) exactly;
* the error bound: <= -30 dB NRMSE against eq. (4) at the default settings;
* convergence: the error falls as the grid oversampling and the taps grow;
* linearity in the echoes and the global-phase identity;
* the Lagrange kernel reproducing polynomials of degree < T;
* the grid construction: every position in exactly one leaf, preimages that
  map back to their (u, v, n), no stencil leaving its grid.
"""
import numpy as np
import pytest

from oracle import geometry as G
from oracle import hhffbp as OH
from oracle import plan as OP
from workloads import voxel_centres


def _plan(w, S, gamma=3.0, T=4, Q=4):
    return OP.build_plan(w.positions, w.freqs_hz, w.grid_origin, w.grid_pitch, w.grid_dims,
                         S, Q, gamma, T)


@pytest.fixture(scope="module")
def direct_small(small):
    vox = voxel_centres(small.grid_origin, small.grid_pitch, small.grid_dims)
    return OH.direct_bp(small.positions, small.freqs_hz, small.echoes, vox).reshape(small.grid_dims)


def test_lagrange_reproduces_polynomials():
    x = np.linspace(0, 0.999, 37)
    for T in (4, 6):
        w = OH.lagrange_weights(x, T)
        nodes = OP.lagrange_offsets(T)
        for deg in range(T):
            poly = w @ (nodes.astype(float) ** deg)
            assert np.max(np.abs(poly - x ** deg)) < 1e-12
        # exact at the node x = 0
        w0 = OH.lagrange_weights(np.array([0.0]), T)[0]
        assert abs(w0[T // 2 - 1] - 1) < 1e-15 and np.sum(np.abs(w0)) - 1 < 1e-15


def test_stage_zero_is_eq4(small, direct_small):
    img = OH.image(_plan(small, 0), small.echoes, small.positions)
    assert np.max(np.abs(img - direct_small)) <= 1e-12 * np.max(np.abs(direct_small))


@pytest.mark.parametrize("S", [1, 2])
def test_error_bound_against_eq4(small, direct_small, S):
    img = OH.image(_plan(small, S), small.echoes, small.positions)
    e = OH.nrmse(img, direct_small)
    assert 20 * np.log10(e) <= -30.0


def test_binary_merges(small, direct_small):
    """Q = 2: the paper's binary, alternating-axis merges (two stages = one Q=4 stage)."""
    img = OH.image(_plan(small, 2, Q=2), small.echoes, small.positions)
    assert 20 * np.log10(OH.nrmse(img, direct_small)) <= -30.0


def test_convergence_with_oversampling_and_taps(small, direct_small):
    errs = {}
    for gamma, T in ((2.0, 4), (3.0, 4), (3.0, 6)):
        img = OH.image(_plan(small, 1, gamma, T), small.echoes, small.positions)
        errs[(gamma, T)] = OH.nrmse(img, direct_small)
    assert errs[(3.0, 4)] < 0.5 * errs[(2.0, 4)]
    assert errs[(3.0, 6)] < 0.5 * errs[(3.0, 4)]


def test_linearity_and_global_phase(small):
    pl = _plan(small, 1)
    rng = np.random.default_rng(0)
    s2 = rng.standard_normal(small.echoes.shape) + 1j * rng.standard_normal(small.echoes.shape)
    a, b = 0.3 + 1j, -2.0
    f1 = OH.image(pl, small.echoes, small.positions)
    f2 = OH.image(pl, s2, small.positions)
    f12 = OH.image(pl, a * small.echoes + b * s2, small.positions)
    assert np.max(np.abs(f12 - a * f1 - b * f2)) <= 1e-11 * np.max(np.abs(f12))
    fp = OH.image(pl, small.echoes * np.exp(0.7j), small.positions)
    assert np.max(np.abs(fp - f1 * np.exp(0.7j))) <= 1e-11 * np.max(np.abs(f1))


def test_partition_and_grids(small):
    pl = _plan(small, 2)
    S = len(pl.levels) - 1
    members = np.concatenate([n.members for n in pl.levels[S]])
    assert np.array_equal(np.sort(members), np.arange(small.n_pos))
    for d in range(1, S + 1):
        for node in pl.levels[d]:
            x0, x1, y0, y1 = node.rect
            xy = small.positions[node.members, :2]
            assert np.all((xy[:, 0] >= x0) & (xy[:, 0] <= x1) & (xy[:, 1] >= y0) & (xy[:, 1] <= y1))
            if node.empty:
                assert node.lattice is None
                continue
            L = node.lattice
            ok = L.valid
            back = G.uvn(L.xyz[ok], node.rect, pl.kmin, pl.kmax) * pl.gamma
            assert np.max(np.abs(back - L.ijl[ok])) < 1e-8
    # config 0 has an empty leaf: it must be skipped, not fail
    assert any(n.empty for n in pl.levels[S])


def test_fast_range_mode(small, direct_small):
    """Level-1 sums through linearly interpolated range profiles: the image
    stays within -30 dB of eq. (4) at U = 8, its distance to the eq. (4)-leaf
    HHFFBPA falls 3-8x per doubling of U (second order or better), and S = 0 reduces to the direct sum
    of the same form."""
    pl = _plan(small, 2, gamma=(3.0, 3.0, 3.5))
    ref = OH.image(pl, small.echoes, small.positions)
    d = []
    for U in (8, 16):
        img = OH.image(pl, small.echoes, small.positions, range_u=U)
        d.append(OH.nrmse(img, ref))
        if U == 8:
            assert 20 * np.log10(OH.nrmse(img, direct_small)) <= -30.0
    assert 3.0 < d[0] / d[1] < 8.0 and d[0] < 1e-3
    vox = voxel_centres(small.grid_origin, small.grid_pitch, small.grid_dims)
    s0 = OH.image(_plan(small, 0), small.echoes, small.positions, range_u=8)
    lin = OH.direct_bp_linear(small.positions, small.freqs_hz, small.echoes, vox, 8)
    assert np.max(np.abs(s0.ravel() - lin)) <= 1e-12 * np.max(np.abs(lin))


def test_bandlimited_weights():
    """The least-squares weights for |omega| <= pi / gamma: exact at the stencil
    nodes; equal to a brute-force least-squares fit of e^{j omega x} by the taps
    on a dense omega grid (independent of the closed-form normal equations);
    never worse than Lagrange in the integrated error over the band."""
    from oracle.plan import lagrange_offsets
    rng = np.random.default_rng(4)
    for T in (4, 6):
        o = lagrange_offsets(T).astype(float)
        for g in (2.0, 3.0, 3.5):
            W = np.pi / g
            w0 = OH.bandlimited_weights(np.array([0.0]), T, g)[0]
            assert np.max(np.abs(w0 - (o == 0))) < 1e-10      # cond(G) up to ~1e6
            om = np.linspace(-W, W, 4001)
            dw = om[1] - om[0]
            q = np.full(om.size, dw)
            q[[0, -1]] *= 0.5                       # trapezoid weights
            x = rng.uniform(0, 1, 5)
            w_ls = OH.bandlimited_weights(x, T, g)
            w_lg = OH.lagrange_weights(x, T)
            for i, xi in enumerate(x):
                A = np.exp(1j * om[:, None] * o[None, :]) * np.sqrt(q)[:, None]
                y = np.exp(1j * om * xi) * np.sqrt(q)
                Ar = np.vstack([A.real, A.imag])
                yr = np.concatenate([y.real, y.imag])
                w_bf = np.linalg.lstsq(Ar, yr, rcond=None)[0]
                assert np.max(np.abs(w_bf - w_ls[i])) < 1e-6
                J = lambda w: np.sum(np.abs(A @ w - y) ** 2)
                assert J(w_ls[i]) <= J(w_lg[i]) * (1 + 1e-9)


def test_bandlimited_kernel_accuracy(small, direct_small):
    """The same grids interpolated with the band-limited weights are more
    accurate than with Lagrange's (S = 2, gamma = (2, 2, 2.5): within -35 dB of
    eq. (4), at least 8 dB better)."""
    from oracle import plan as OP
    g = (2.0, 2.0, 2.5)
    e = {}
    for kern in ("lagrange", "bandlimited"):
        pl = OP.build_plan(small.positions, small.freqs_hz, small.grid_origin, small.grid_pitch,
                           small.grid_dims, 2, 4, g, 4, kernel=kern)
        e[kern] = 20 * np.log10(OH.nrmse(OH.image(pl, small.echoes, small.positions), direct_small))
    assert e["bandlimited"] <= -35.0
    assert e["bandlimited"] <= e["lagrange"] - 8.0


def test_root_grid(small, direct_small):
    """A compressed lattice at the root (the full-aperture grid) plus one
    resample to the voxels: its points map back to their (u, v, n) in the full
    aperture's frame; their values are eq. (4) over every position, compressed
    with the root's Phi (within the merge error); the image stays within -30 dB
    of eq. (4) for S = 1, 2 and Q = 2, and its error falls by more than half with
    T = 6 taps."""
    for S, Q in ((1, 4), (2, 4), (2, 2)):
        pl = OP.build_plan(small.positions, small.freqs_hz, small.grid_origin, small.grid_pitch,
                           small.grid_dims, S, Q, 3.0, 4, root_grid=True)
        img, vals = OH.image(pl, small.echoes, small.positions, keep=True)
        assert 20 * np.log10(OH.nrmse(img, direct_small)) <= -30.0, (S, Q)
        root = pl.levels[0][0]
        L = root.lattice
        ok = L.valid
        back = G.uvn(L.xyz[ok], root.rect, pl.kmin, pl.kmax) * pl.gamma
        assert np.max(np.abs(back - L.ijl[ok])) < 1e-8
        # root values: eq. (4) at the points that lie in the scene box, compressed
        box = np.all((L.xyz[ok] >= small.grid_origin) &
                     (L.xyz[ok] <= small.grid_origin + (np.array(small.grid_dims) - 1) * small.grid_pitch),
                     axis=1)
        q = L.xyz[ok][box]
        ref = OH.direct_bp(small.positions, small.freqs_hz, small.echoes, q) * \
            np.exp(-1j * G.phi(q, root.rect, pl.kmin, pl.kmax))
        assert 20 * np.log10(OH.nrmse(vals[(0, 0)][ok][box], ref)) <= -30.0
        assert not np.any(vals[(0, 0)][~ok])
    e = {}
    for T in (4, 6):
        pl = OP.build_plan(small.positions, small.freqs_hz, small.grid_origin, small.grid_pitch,
                           small.grid_dims, 1, 4, 3.0, T, root_grid=True)
        e[T] = OH.nrmse(OH.image(pl, small.echoes, small.positions), direct_small)
    assert e[6] < 0.5 * e[4]
    with pytest.raises(ValueError):
        OP.build_plan(small.positions, small.freqs_hz, small.grid_origin, small.grid_pitch,
                      small.grid_dims, 0, 4, 3.0, 4, root_grid=True)


def test_leaf_oversampling(small, direct_small):
    """Leaf grids at their own oversampling (gamma_leaf): the grids above the
    leaves are those of the uniform plan, the leaf points map back to their
    (u, v, n) at gamma_leaf, gamma_leaf = gamma reproduces the uniform plan's
    image exactly, coarser leaf grids hold fewer points and lose accuracy
    monotonically, and the image stays within -30 dB of eq. (4)."""
    g = (2.2, 2.2, 2.6)
    args = (small.positions, small.freqs_hz, small.grid_origin, small.grid_pitch, small.grid_dims,
            2, 4, g, 4)
    uni = OP.build_plan(*args, kernel="bandlimited")
    same = OP.build_plan(*args, kernel="bandlimited", gamma_leaf=g)
    img_u = OH.image(uni, small.echoes, small.positions)
    assert np.array_equal(OH.image(same, small.echoes, small.positions), img_u)
    err, npts = [], []
    for gl in ((2.0, 2.0, 2.4), (1.8, 1.8, 2.2), (1.6, 1.6, 2.0)):
        pl = OP.build_plan(*args, kernel="bandlimited", gamma_leaf=gl)
        assert np.allclose(pl.gamma_at(1), g) and np.allclose(pl.gamma_at(2), gl)
        for node_u, node in zip(uni.levels[1], pl.levels[1]):
            if node.empty:
                continue
            assert np.array_equal(node.lattice.ijl, node_u.lattice.ijl)
        n = 0
        for node in pl.levels[2]:
            if node.empty:
                continue
            L = node.lattice
            back = G.uvn(L.xyz[L.valid], node.rect, pl.kmin, pl.kmax) * np.asarray(gl)
            assert np.max(np.abs(back - L.ijl[L.valid])) < 1e-8
            n += L.size
        npts.append(n)
        img = OH.image(pl, small.echoes, small.positions)
        err.append(OH.nrmse(img, direct_small))
        assert 20 * np.log10(err[-1]) <= -30.0, gl
    e_u = OH.nrmse(img_u, direct_small)
    assert npts[0] > npts[1] > npts[2]
    assert e_u <= err[0] <= err[1] <= err[2]
