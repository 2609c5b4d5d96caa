"""GPU parity with a compressed root grid (the root merged onto a lattice of its
own in the full aperture's (u, v, n), then one single-child resample to the
voxels): image, every compressed subimage including the root's, storage forms,
the final stage's LDS staging, and the backward, all against the float64
oracle built with the same choice.  Bars as in the parity tests without a root
grid: 1e-5 NRMSE for float32 storage, <= -30 dB against eq. (4)."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

H = pytest.importorskip("paper_2506_23568_amd")
GAMMA = (3.0, 3.0, 3.5)
TAPS = 4
BOUND = {"c64": 1e-5, "f16": 1e-3, "bf16": 1e-2}


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


@pytest.fixture(scope="module")
def eq4_small(small):
    from oracle import hhffbp as OH
    from workloads import voxel_centres
    vox = voxel_centres(small.grid_origin, small.grid_pitch, small.grid_dims)
    return OH.direct_bp(small.positions, small.freqs_hz, small.echoes, vox).reshape(small.grid_dims)


def _args(w):
    return (w.positions, w.freqs_hz, w.grid_origin, w.grid_pitch, w.grid_dims)


def _nrmse(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _echoes(torch, w, storage="c64"):
    if storage == "c64":
        return torch.from_numpy(w.echoes.astype(np.complex64)).cuda()
    return H.Plan.pack_echoes(torch.from_numpy(w.echoes), storage).cuda()


@pytest.mark.parametrize("S,Q,kernel,storage", [
    (1, 4, "lagrange", "c64"), (2, 4, "lagrange", "c64"), (2, 2, "lagrange", "c64"),
    (2, 4, "bandlimited", "c64"), (2, 4, "lagrange", "f16"), (2, 4, "lagrange", "bf16"),
])
def test_root_grid_image_vs_oracle(torch, small, eq4_small, S, Q, kernel, storage):
    from oracle import hhffbp as OH
    from oracle import plan as OP
    _say(f"root grid small S={S} Q={Q} {kernel} {storage}")
    op = OP.build_plan(*_args(small), S, Q, GAMMA, TAPS, kernel=kernel, root_grid=True)
    ref, vals = OH.image(op, small.echoes, small.positions, keep=True)
    assert (0, 0) in vals
    pl = H.Plan(*_args(small), stages=S, merge_factor=Q, oversample=GAMMA, interp_taps=TAPS,
                interp_kernel=kernel, storage=storage, root_grid=True)
    info = pl.info()
    assert info["root_grid"] == 1
    assert info["level_points"][0] == op.levels[0][0].lattice.size
    ws = pl._workspace(torch)
    img = pl.image(_echoes(torch, small, storage), workspace=ws)
    torch.cuda.synchronize()
    img = img.cpu().numpy().astype(np.complex128)
    e = _nrmse(img, ref)
    worst = 0.0
    for (d, i), v in vals.items():
        g = pl.workspace_view(ws, d, i).cpu().numpy().astype(np.complex128)
        worst = max(worst, _nrmse(g, v))
    e_bp = _nrmse(img, eq4_small)
    _say(f"  vs oracle {e:.3e}; worst stage {worst:.3e}; vs eq.4 {20 * np.log10(e_bp):.1f} dB")
    assert e <= BOUND[storage]
    assert worst <= BOUND[storage]
    assert 20 * np.log10(e_bp) <= -30.0


@pytest.mark.parametrize("storage", ["c64", "f16"])
def test_root_grid_final_staging_is_bit_exact(torch, small, storage):
    """The resample from the root grid reads the same taps in the same order
    whether the root's values are staged through LDS or gathered directly."""
    kw = dict(stages=2, oversample=GAMMA, interp_taps=TAPS, storage=storage, root_grid=True)
    on = H.Plan(*_args(small), **kw)
    off = H.Plan(*_args(small), final_staging=False, **kw)
    assert on.info()["final_boxed"] > 0 and off.info()["final_boxed"] == 0
    ech = _echoes(torch, small, storage)
    a = on.image(ech).cpu().numpy()
    b = off.image(ech).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("S,Q", [(2, 4), (2, 2)])
def test_root_grid_gradients_vs_oracle(torch, small, S, Q):
    from oracle import adjoint as OA
    from oracle import plan as OP
    op = OP.build_plan(*_args(small), S, Q, GAMMA, TAPS, root_grid=True)
    pl = H.Plan(*_args(small), stages=S, merge_factor=Q, oversample=GAMMA, interp_taps=TAPS,
                root_grid=True)
    rng = np.random.default_rng(11)
    g = rng.standard_normal(small.grid_dims) + 1j * rng.standard_normal(small.grid_dims)
    ref_s = OA.echo_gradient(op, g, small.positions)
    ref_p = OA.position_gradient(op, small.echoes, small.positions, g)
    ge, gp = pl.backward(_echoes(torch, small), torch.from_numpy(g.astype(np.complex64)).cuda())
    es = _nrmse(ge.cpu().numpy().astype(np.complex128), ref_s)
    ep = float(np.linalg.norm(gp.cpu().numpy() - ref_p) / np.linalg.norm(ref_p))
    _say(f"  root grid S={S} Q={Q}: echo gradient NRMSE {es:.2e}; position gradient rel {ep:.2e}")
    assert es <= 1e-5
    assert ep <= 1e-3


def test_root_grid_adjoint_identity(torch, small):
    pl = H.Plan(*_args(small), stages=2, oversample=GAMMA, interp_taps=TAPS, root_grid=True)
    rng = np.random.default_rng(12)
    s = rng.standard_normal(small.echoes.shape) + 1j * rng.standard_normal(small.echoes.shape)
    g = rng.standard_normal(small.grid_dims) + 1j * rng.standard_normal(small.grid_dims)
    s32 = s.astype(np.complex64)
    g32 = g.astype(np.complex64)
    f = pl.image(torch.from_numpy(s32).cuda()).cpu().numpy().astype(np.complex128)
    ge, _ = pl.backward(None, torch.from_numpy(g32).cuda(), want_positions=False)
    ge = ge.cpu().numpy().astype(np.complex128)
    lhs = np.vdot(g32.astype(np.complex128).ravel(), f.ravel())
    rhs = np.vdot(ge.ravel(), s32.astype(np.complex128).ravel())
    _say(f"  root grid <As,g> {lhs:.6e}  <s,A^H g> {rhs:.6e}")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
