"""Pins of the oracle's adjoint and trajectory gradient (CPU only).

* the adjoint identity <A s, g> = <s, A^H g> for the factorised operator;
* the position gradient against central finite differences of the oracle
  image (frozen plan), h = 1e-6 m;
* the loss cotangent against finite differences of the loss.
"""
import numpy as np
import pytest

from oracle import adjoint as OA
from oracle import hhffbp as OH
from oracle import loss as OL
from oracle import plan as OP


@pytest.fixture(scope="module")
def tiny():
    """A reduced handheld scan: 192 positions of the small walk, 6x6x4 voxels."""
    from workloads import make_config
    w = make_config(0)
    sel = np.arange(0, w.n_pos, 5)[:192]
    pos, ech = w.positions[sel], w.echoes[sel]
    origin = np.array([-0.005, -0.005, 0.245])
    pitch = np.full(3, 2e-3)
    dims = (6, 6, 4)
    pl = OP.build_plan(pos, w.freqs_hz, origin, pitch, dims, 1, 4, (3.0, 3.0, 3.5), 4)
    return pl, pos, ech


def test_factorised_adjoint_identity(tiny):
    pl, pos, ech = tiny
    rng = np.random.default_rng(0)
    s = rng.standard_normal(ech.shape) + 1j * rng.standard_normal(ech.shape)
    g = rng.standard_normal(pl.dims) + 1j * rng.standard_normal(pl.dims)
    lhs = np.vdot(g.ravel(), OH.image(pl, s, pos).ravel())
    rhs = np.vdot(OA.echo_gradient(pl, g, pos).ravel(), s.ravel())
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_position_gradient_against_central_differences(tiny):
    pl, pos, ech = tiny
    rng = np.random.default_rng(1)
    g = rng.standard_normal(pl.dims) + 1j * rng.standard_normal(pl.dims)

    def L(p):
        return float(np.real(np.vdot(g.ravel(), OH.image(pl, ech, p).ravel())))

    grad = OA.position_gradient(pl, ech, pos, g)
    scale = np.max(np.abs(grad))
    h = 1e-6
    for i, a in [(0, 0), (7, 1), (31, 2), (100, 0), (150, 2), (191, 1)]:
        pp, pm = pos.copy(), pos.copy()
        pp[i, a] += h
        pm[i, a] -= h
        fd = (L(pp) - L(pm)) / (2 * h)
        assert abs(fd - grad[i, a]) <= 1e-5 * scale, (i, a, fd, grad[i, a])


def test_loss_cotangent_against_central_differences():
    rng = np.random.default_rng(2)
    f = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    fc = f + 0.3 * (rng.standard_normal(40) + 1j * rng.standard_normal(40))
    g = OL.loss_cotangent(f, fc)
    h = 1e-7
    for v in range(0, 40, 7):
        e = np.zeros(40)
        e[v] = h
        d_re = (OL.loss(f + e, fc) - OL.loss(f - e, fc)) / (2 * h)
        d_im = (OL.loss(f + 1j * e, fc) - OL.loss(f - 1j * e, fc)) / (2 * h)
        assert abs(d_re - g[v].real) < 1e-7 and abs(d_im - g[v].imag) < 1e-7


def test_factorised_adjoint_identity_bandlimited(tiny):
    """<A s, g> = <s, A^H g> with band-limited interpolation weights."""
    pl, pos, ech = tiny
    from oracle import plan as OP
    from workloads import make_config
    w = make_config(0)
    sel = np.arange(0, w.n_pos, 5)[:192]
    plb = OP.build_plan(w.positions[sel], w.freqs_hz, np.array([-0.005, -0.005, 0.245]),
                        np.full(3, 2e-3), (6, 6, 4), 1, 4, (2.0, 2.0, 2.5), 4, kernel="bandlimited")
    rng = np.random.default_rng(3)
    s = rng.standard_normal(ech.shape) + 1j * rng.standard_normal(ech.shape)
    g = rng.standard_normal(plb.dims) + 1j * rng.standard_normal(plb.dims)
    lhs = np.vdot(g.ravel(), OH.image(plb, s, pos).ravel())
    rhs = np.vdot(OA.echo_gradient(plb, g, pos).ravel(), s.ravel())
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_aperture_weights(tiny):
    """Aperture weights (the measure of dp' in eq. (4)): 0/1 weights give eq. (4)
    over the selected positions alone; a constant weight scales the image; the
    weighted operator and its adjoint satisfy <A_w s, g> = <s, A_w^H g>; the
    weighted position gradient matches central differences of the weighted
    image (frozen plan, h = 1e-6 m)."""
    pl, pos, ech = tiny
    rng = np.random.default_rng(4)
    n = pos.shape[0]
    pts = np.array([[0.0, 0.0, 0.25], [0.003, -0.002, 0.248], [-0.004, 0.001, 0.252]])
    keep = rng.random(n) < 0.4
    from workloads import make_config
    freqs = make_config(0).freqs_hz
    f_w = OH.direct_bp(pos, freqs, ech, pts, weights=keep.astype(float))
    f_sub = OH.direct_bp(pos[keep], freqs, ech[keep], pts)
    assert np.allclose(f_w, f_sub, rtol=0, atol=1e-12 * np.abs(f_sub).max())
    f1 = OH.direct_bp(pos, freqs, ech, pts)
    assert np.allclose(OH.direct_bp(pos, freqs, ech, pts, weights=np.full(n, 2.5)), 2.5 * f1,
                       rtol=1e-14, atol=0)
    w = rng.uniform(0.2, 1.8, n)
    s = rng.standard_normal(ech.shape) + 1j * rng.standard_normal(ech.shape)
    g = rng.standard_normal(pl.dims) + 1j * rng.standard_normal(pl.dims)
    lhs = np.vdot(g.ravel(), OH.image(pl, s, pos, weights=w).ravel())
    rhs = np.vdot(OA.echo_gradient(pl, g, pos, weights=w).ravel(), s.ravel())
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    gp = OA.position_gradient(pl, ech, pos, g, weights=w)
    h = 1e-6
    for i, a in ((3, 0), (77, 1), (150, 2)):
        dp = np.zeros_like(pos)
        dp[i, a] = h
        fp = OH.image(pl, ech, pos + dp, weights=w)
        fm = OH.image(pl, ech, pos - dp, weights=w)
        fd = np.real(np.vdot(g.ravel(), ((fp - fm) / (2 * h)).ravel()))
        assert abs(gp[i, a] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(gp).max())


def test_root_grid_adjoint_and_position_gradient(tiny):
    """With a root grid (one more merge, then one resample to the voxels): the
    adjoint identity <A s, g> = <s, A^H g>, and the position gradient against
    central differences of the image (frozen plan, h = 1e-6 m)."""
    pl, pos, ech = tiny
    from oracle import plan as OP
    from workloads import make_config
    w = make_config(0)
    plr = OP.build_plan(pos, w.freqs_hz, np.array([-0.005, -0.005, 0.245]), np.full(3, 2e-3),
                        (6, 6, 4), 2, 2, (3.0, 3.0, 3.5), 4, root_grid=True)
    assert plr.levels[0][0].lattice is not None
    rng = np.random.default_rng(5)
    s = rng.standard_normal(ech.shape) + 1j * rng.standard_normal(ech.shape)
    g = rng.standard_normal(plr.dims) + 1j * rng.standard_normal(plr.dims)
    lhs = np.vdot(g.ravel(), OH.image(plr, s, pos).ravel())
    rhs = np.vdot(OA.echo_gradient(plr, g, pos).ravel(), s.ravel())
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    gp = OA.position_gradient(plr, ech, pos, g)
    h = 1e-6
    for i, a in ((2, 1), (64, 0), (180, 2)):
        dp = np.zeros_like(pos)
        dp[i, a] = h
        fd = np.real(np.vdot(g.ravel(), ((OH.image(plr, ech, pos + dp) -
                                          OH.image(plr, ech, pos - dp)) / (2 * h)).ravel()))
        assert abs(gp[i, a] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(gp).max())
