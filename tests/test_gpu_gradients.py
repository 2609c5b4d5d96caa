"""GPU gradients: hhffbp_backward (through the C ABI and the autograd Function)
against the float64 oracle.

* the adjoint identity <A s, g> = <s, A^H g> of the GPU forward and backward;
* the echo gradient against the oracle's transposed HHFFBPA (NRMSE <= 1e-5);
* the position gradient against the oracle's analytic gradient (<= 1e-3);
* the grad workload (1024 positions with a smooth 0-3 mm trajectory error):
  entropy + L2-to-clean loss through torch.autograd, position gradients at 64
  seeded coordinates against central differences (h = 1e-6 m) of the float64
  oracle loss with the frozen plan (relative error <= 1e-3).
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

H = pytest.importorskip("paper_2506_23568_amd")
GAMMA = (3.0, 3.0, 3.5)
TAPS = 4


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _args(w, pos=None):
    return (w.positions if pos is None else pos, w.freqs_hz, w.grid_origin, w.grid_pitch,
            w.grid_dims)


def _nrmse(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def test_gpu_adjoint_identity(torch, small):
    pl = H.Plan(*_args(small), stages=2, oversample=GAMMA, interp_taps=TAPS)
    rng = np.random.default_rng(0)
    s = rng.standard_normal(small.echoes.shape) + 1j * rng.standard_normal(small.echoes.shape)
    g = rng.standard_normal(small.grid_dims) + 1j * rng.standard_normal(small.grid_dims)
    st = torch.from_numpy(s.astype(np.complex64)).cuda()
    gt = torch.from_numpy(g.astype(np.complex64)).cuda()
    f = pl.image(st).cpu().numpy().astype(np.complex128)
    ge, _ = pl.backward(None, gt, want_positions=False)
    ge = ge.cpu().numpy().astype(np.complex128)
    lhs = np.vdot(g.astype(np.complex64).astype(np.complex128).ravel(), f.ravel())
    rhs = np.vdot(ge.ravel(), s.astype(np.complex64).astype(np.complex128).ravel())
    _say(f"  <As,g> {lhs:.6e}  <s,A^H g> {rhs:.6e}  rel {abs(lhs - rhs) / abs(lhs):.2e}")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("S,Q", [(2, 4), (2, 2)])
def test_gpu_gradients_vs_oracle(torch, small, S, Q):
    from oracle import adjoint as OA
    from oracle import plan as OP
    op = OP.build_plan(*_args(small), S, Q, GAMMA, TAPS)
    pl = H.Plan(*_args(small), stages=S, merge_factor=Q, oversample=GAMMA, interp_taps=TAPS)
    rng = np.random.default_rng(1)
    g = rng.standard_normal(small.grid_dims) + 1j * rng.standard_normal(small.grid_dims)
    ref_s = OA.echo_gradient(op, g, small.positions)
    ref_p = OA.position_gradient(op, small.echoes, small.positions, g)
    ech = torch.from_numpy(small.echoes.astype(np.complex64)).cuda()
    gt = torch.from_numpy(g.astype(np.complex64)).cuda()
    ge, gp = pl.backward(ech, gt)
    ge = ge.cpu().numpy().astype(np.complex128)
    gp = gp.cpu().numpy()
    es = _nrmse(ge, ref_s)
    ep = float(np.linalg.norm(gp - ref_p) / np.linalg.norm(ref_p))
    _say(f"  S={S} Q={Q}: echo gradient NRMSE {es:.2e}; position gradient rel {ep:.2e}")
    assert es <= 1e-5
    assert ep <= 1e-3


def _torch_loss(torch, f, f_clean):
    """Entropy of |f|^2 plus the relative L2 distance to f_clean (float64)."""
    f = f.to(torch.complex128).reshape(-1)
    fc = f_clean.reshape(-1)
    a = f.real ** 2 + f.imag ** 2
    q = a / a.sum()
    H_ = -(q * torch.log(q)).sum()
    d = f - fc
    return H_ + (d.real ** 2 + d.imag ** 2).sum() / (fc.real ** 2 + fc.imag ** 2).sum()


def test_autofocus_gradient_against_finite_differences(torch):
    from oracle import hhffbp as OH
    from oracle import loss as OL
    from oracle import plan as OP
    from workloads import make_config
    w = make_config(3)
    p_true, p_img = w.positions, w.imager_positions
    _say(f"  trajectory error max {np.abs(p_img - p_true).max() * 1e3:.2f} mm")
    S = 2
    op_true = OP.build_plan(*_args(w, p_true), S, 4, GAMMA, TAPS)
    f_clean = OH.image(op_true, w.echoes, p_true)
    op = OP.build_plan(*_args(w, p_img), S, 4, GAMMA, TAPS)
    pl = H.Plan(*_args(w, p_img), stages=S, oversample=GAMMA, interp_taps=TAPS)
    ech = torch.from_numpy(w.echoes.astype(np.complex64)).cuda()
    pos_t = torch.from_numpy(p_img.copy()).cuda().requires_grad_(True)
    fc_t = torch.from_numpy(f_clean).cuda()
    img = H.hhffbp_image(ech, pos_t, pl)
    L = _torch_loss(torch, img, fc_t)
    L.backward()
    g_gpu = pos_t.grad.cpu().numpy()

    def loss_at(p):
        return OL.loss(OH.image(op, w.echoes, p), f_clean)

    L0 = loss_at(p_img)
    _say(f"  loss: oracle {L0:.6f}, GPU {L.item():.6f}")
    rng = np.random.default_rng(4)
    coords = [(int(rng.integers(w.n_pos)), int(rng.integers(3))) for _ in range(64)]
    h = 1e-6
    fd = np.zeros(len(coords))
    for k, (i, a) in enumerate(coords):
        pp, pm = p_img.copy(), p_img.copy()
        pp[i, a] += h
        pm[i, a] -= h
        fd[k] = (loss_at(pp) - loss_at(pm)) / (2 * h)
        if k % 16 == 15:
            _say(f"  finite differences {k + 1}/64")
    gs = np.array([g_gpu[i, a] for i, a in coords])
    rel = float(np.linalg.norm(gs - fd) / np.linalg.norm(fd))
    worst = float(np.max(np.abs(gs - fd)) / np.max(np.abs(fd)))
    _say(f"  GPU vs FD: rel {rel:.2e}, worst coordinate {worst:.2e} of max |FD|")
    assert abs(L.item() - L0) <= 1e-4 * abs(L0)
    assert rel <= 1e-3
    assert worst <= 1e-2


def test_gpu_gradients_bandlimited(torch, small):
    """The adjoint and position gradient with band-limited interpolation
    weights against the oracle (same bars as with Lagrange's)."""
    from oracle import adjoint as OA
    from oracle import plan as OP
    g3 = (2.0, 2.0, 2.5)
    op = OP.build_plan(*_args(small), 2, 4, g3, TAPS, kernel="bandlimited")
    pl = H.Plan(*_args(small), stages=2, oversample=g3, interp_taps=TAPS,
                interp_kernel="bandlimited")
    rng = np.random.default_rng(2)
    g = rng.standard_normal(small.grid_dims) + 1j * rng.standard_normal(small.grid_dims)
    ref_s = OA.echo_gradient(op, g, small.positions)
    ref_p = OA.position_gradient(op, small.echoes, small.positions, g)
    ge, gp = pl.backward(torch.from_numpy(small.echoes.astype(np.complex64)).cuda(),
                         torch.from_numpy(g.astype(np.complex64)).cuda())
    es = _nrmse(ge.cpu().numpy().astype(np.complex128), ref_s)
    ep = float(np.linalg.norm(gp.cpu().numpy() - ref_p) / np.linalg.norm(ref_p))
    _say(f"  bandlimited: echo gradient NRMSE {es:.2e}; position gradient rel {ep:.2e}")
    assert es <= 1e-5
    assert ep <= 1e-3


def test_gpu_gradients_with_aperture_weights(torch, small):
    """Weighted echo and position gradients against the oracle's (weights scale
    row i of A and position i's terms): echo <= 1e-5, positions <= 1e-3."""
    from oracle import adjoint as OA
    from oracle import plan as OP
    w8 = np.random.default_rng(9).uniform(0.1, 2.0, small.n_pos)
    op = OP.build_plan(*_args(small), 2, 4, GAMMA, TAPS)
    pl = H.Plan(*_args(small), stages=2, oversample=GAMMA, interp_taps=TAPS, weights=w8)
    rng = np.random.default_rng(2)
    g = rng.standard_normal(small.grid_dims) + 1j * rng.standard_normal(small.grid_dims)
    ref_s = OA.echo_gradient(op, g, small.positions, weights=w8)
    ref_p = OA.position_gradient(op, small.echoes, small.positions, g, weights=w8)
    ech = torch.from_numpy(small.echoes.astype(np.complex64)).cuda()
    gt = torch.from_numpy(g.astype(np.complex64)).cuda()
    ge, gp = pl.backward(ech, gt)
    es = _nrmse(ge.cpu().numpy().astype(np.complex128), ref_s)
    gp = gp.cpu().numpy()
    ep = float(np.linalg.norm(gp - ref_p) / np.linalg.norm(ref_p))
    _say(f"  weighted: echo gradient NRMSE {es:.2e}; position gradient rel {ep:.2e}")
    assert es <= 1e-5 and ep <= 1e-3



@pytest.mark.parametrize("U,bound", [(8, 5e-3), (4, 2e-2)])
def test_gpu_gradients_linear_range_mode(torch, small, U, bound):
    """The fast range mode (linear kernel, U-fold range oversampling) in the
    backward.  Echo gradient: the adjoint identity with the same mode's forward
    (<= 1e-5).  Position gradient: the kernels interpolate the range-derivative
    profiles h' (the analytic derivative), so they give the exact gradient to the
    range kernel's accuracy (1/U^2: ~1e-3 at U = 8), checked against the
    oracle's exact position gradient (<= 5e-3 at U = 8, 2e-2 at U = 4); central
    differences of the oracle's own linear form are reported beside it."""
    from oracle import adjoint as OA
    from oracle import hhffbp as OH
    from oracle import plan as OP
    kw = dict(stages=2, oversample=GAMMA, interp_taps=TAPS, range_kernel="linear",
              range_oversample=float(U))
    pl = H.Plan(*_args(small), **kw)
    rng = np.random.default_rng(6)
    s = rng.standard_normal(small.echoes.shape) + 1j * rng.standard_normal(small.echoes.shape)
    g = rng.standard_normal(small.grid_dims) + 1j * rng.standard_normal(small.grid_dims)
    st = torch.from_numpy(s.astype(np.complex64)).cuda()
    gt = torch.from_numpy(g.astype(np.complex64)).cuda()
    f = pl.image(st).cpu().numpy().astype(np.complex128)
    ge, _ = pl.backward(None, gt, want_positions=False)
    ge = ge.cpu().numpy().astype(np.complex128)
    lhs = np.vdot(g.astype(np.complex64).astype(np.complex128).ravel(), f.ravel())
    rhs = np.vdot(ge.ravel(), s.astype(np.complex64).astype(np.complex128).ravel())
    e_adj = abs(lhs - rhs) / abs(lhs)
    ech = torch.from_numpy(small.echoes.astype(np.complex64)).cuda()
    _, gp = pl.backward(ech, gt)
    gp = gp.cpu().numpy()
    op = OP.build_plan(*_args(small), 2, 4, GAMMA, TAPS)
    ref = OA.position_gradient(op, small.echoes, small.positions, g)
    e_p = float(np.linalg.norm(gp - ref) / np.linalg.norm(ref))
    coords = [(int(rng.integers(small.n_pos)), int(rng.integers(3))) for _ in range(8)]
    h = 1e-6
    fd, an = [], []
    for i, a in coords:
        pp, pm = small.positions.copy(), small.positions.copy()
        pp[i, a] += h
        pm[i, a] -= h
        d = OH.image(op, small.echoes, pp, range_u=U) - OH.image(op, small.echoes, pm, range_u=U)
        fd.append(np.real(np.vdot(g.ravel(), d.ravel())) / (2 * h))
        an.append(gp[i, a])
    e_fd = float(np.linalg.norm(np.array(an) - np.array(fd)) / np.linalg.norm(fd))
    _say(f"  U={U}: adjoint identity {e_adj:.2e}; position gradient vs exact {e_p:.2e}, "
         f"vs central differences of the linear form {e_fd:.2e}")
    assert e_adj <= 1e-5
    assert e_p <= bound
