"""GPU parity on shapes the workloads do not produce: voxel grids that fill no
brick or tile evenly (29 x 19 x 13, 5 x 3 x 2, a single voxel), frequencies that
are not equispaced, and apertures of a few positions (most leaves empty, some
holding one position).  Every case against the float64 oracle built with the
same choices: 1e-5 NRMSE for images, subimages and echo gradients, 1e-3 for the
position gradient, as in the parity tests on the workloads."""
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


def _nrmse(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _centred(dims, pitch=2e-3, centre=(0.0, 0.0, 0.25)):
    d = np.asarray(dims)
    return (np.asarray(centre) - 0.5 * (d - 1) * pitch, np.full(3, pitch),
            tuple(int(v) for v in dims))


def _image_and_stages(torch, pl, echoes):
    ws = pl._workspace(torch)
    img = pl.image(torch.from_numpy(echoes.astype(np.complex64)).cuda(), workspace=ws)
    torch.cuda.synchronize()
    return img.cpu().numpy().astype(np.complex128), ws


@pytest.mark.parametrize("dims", [(29, 19, 13), (5, 3, 2), (1, 1, 1)])
@pytest.mark.parametrize("S,root", [(1, False), (2, False), (2, True)])
def test_ragged_grids_vs_oracle(torch, small, dims, S, root):
    from oracle import hhffbp as OH
    from oracle import plan as OP
    o, p, d = _centred(dims)
    args = (small.positions, small.freqs_hz, o, p, d)
    _say(f"ragged grid {d} S={S} root grid {root}")
    op = OP.build_plan(*args, S, 4, GAMMA, TAPS, root_grid=root)
    ref, vals = OH.image(op, small.echoes, small.positions, keep=True)
    pl = H.Plan(*args, stages=S, oversample=GAMMA, interp_taps=TAPS, root_grid=root)
    img, ws = _image_and_stages(torch, pl, small.echoes)
    e = _nrmse(img, ref)
    worst = max(_nrmse(pl.workspace_view(ws, dd, i).cpu().numpy().astype(np.complex128), v)
                for (dd, i), v in vals.items())
    off = H.Plan(*args, stages=S, oversample=GAMMA, interp_taps=TAPS, root_grid=root,
                 final_staging=False)
    img_off, _ = _image_and_stages(torch, off, small.echoes)
    _say(f"  vs oracle {e:.2e}; worst stage {worst:.2e}; staging bit-exact "
         f"{np.array_equal(img, img_off)}")
    assert e <= 1e-5 and worst <= 1e-5
    assert np.array_equal(img, img_off)


@pytest.mark.parametrize("dims", [(29, 19, 13), (1, 1, 1)])
def test_ragged_grids_direct_vs_eq4(torch, small, dims):
    from oracle import hhffbp as OH
    from workloads import voxel_centres
    o, p, d = _centred(dims)
    args = (small.positions, small.freqs_hz, o, p, d)
    ref = OH.direct_bp(small.positions, small.freqs_hz, small.echoes,
                       voxel_centres(o, p, d)).reshape(d)
    ech = torch.from_numpy(small.echoes.astype(np.complex64)).cuda()
    for mode in ("direct_rc", "direct_exact"):
        img = H.Plan(*args, mode=mode).image(ech).cpu().numpy().astype(np.complex128)
        e = _nrmse(img, ref)
        _say(f"  {mode} grid {d}: vs eq.4 {e:.2e}")
        assert e <= 1e-5


def test_ragged_grid_gradients_vs_oracle(torch, small):
    from oracle import adjoint as OA
    from oracle import plan as OP
    o, p, d = _centred((29, 19, 13))
    args = (small.positions, small.freqs_hz, o, p, d)
    op = OP.build_plan(*args, 2, 4, GAMMA, TAPS)
    pl = H.Plan(*args, stages=2, oversample=GAMMA, interp_taps=TAPS)
    rng = np.random.default_rng(21)
    g = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    ref_s = OA.echo_gradient(op, g, small.positions)
    ref_p = OA.position_gradient(op, small.echoes, small.positions, g)
    ge, gp = pl.backward(torch.from_numpy(small.echoes.astype(np.complex64)).cuda(),
                         torch.from_numpy(g.astype(np.complex64)).cuda())
    es = _nrmse(ge.cpu().numpy().astype(np.complex128), ref_s)
    ep = float(np.linalg.norm(gp.cpu().numpy() - ref_p) / np.linalg.norm(ref_p))
    _say(f"  ragged grid gradients: echoes {es:.2e}, positions {ep:.2e}")
    assert es <= 1e-5
    assert ep <= 1e-3


def test_unequal_frequency_steps_hhffbp(torch, small):
    """Frequencies jittered by up to 30% of their step (the range compression is
    a dense DFT, so any spacing is valid): echoes synthesised at those
    frequencies, HHFFBPA against the oracle (<= 1e-5) and eq. (4) (<= -30 dB)."""
    from oracle import hhffbp as OH
    from oracle import plan as OP
    from workloads import synth_echoes, voxel_centres
    rng = np.random.default_rng(6)
    f = np.sort(small.freqs_hz + rng.uniform(-0.3, 0.3, small.freqs_hz.size) *
                (small.freqs_hz[1] - small.freqs_hz[0]))
    ech = synth_echoes(small.positions, f, small.target_pos, small.target_amp)
    args = (small.positions, f, small.grid_origin, small.grid_pitch, small.grid_dims)
    op = OP.build_plan(*args, 2, 4, GAMMA, TAPS)
    ref = OH.image(op, ech, small.positions)
    eq4 = OH.direct_bp(small.positions, f, ech, voxel_centres(*args[2:])).reshape(small.grid_dims)
    pl = H.Plan(*args, stages=2, oversample=GAMMA, interp_taps=TAPS)
    img, _ = _image_and_stages(torch, pl, ech)
    e, e4 = _nrmse(img, ref), _nrmse(img, eq4)
    _say(f"  unequal steps: vs oracle {e:.2e}; vs eq.4 {20 * np.log10(e4):.1f} dB")
    assert e <= 1e-5
    assert 20 * np.log10(e4) <= -30.0


@pytest.mark.parametrize("S", [1, 2])
def test_few_positions(torch, small, S):
    """Seven positions: most leaves are empty (zero subimages, no grid) and the
    others hold one to three positions."""
    from oracle import hhffbp as OH
    from oracle import plan as OP
    idx = np.arange(0, small.positions.shape[0], 150)
    pos, ech = small.positions[idx], small.echoes[idx]
    args = (pos, small.freqs_hz, small.grid_origin, small.grid_pitch, small.grid_dims)
    op = OP.build_plan(*args, S, 4, GAMMA, TAPS)
    assert any(n.empty for n in op.levels[S])
    ref, vals = OH.image(op, ech, pos, keep=True)
    pl = H.Plan(*args, stages=S, oversample=GAMMA, interp_taps=TAPS)
    img, ws = _image_and_stages(torch, pl, ech)
    e = _nrmse(img, ref)
    worst = max(_nrmse(pl.workspace_view(ws, d, i).cpu().numpy().astype(np.complex128), v)
                for (d, i), v in vals.items())
    _say(f"  {idx.size} positions S={S}: {pl.info()['n_leaves']} leaves; vs oracle {e:.2e}; "
         f"worst stage {worst:.2e}")
    assert e <= 1e-5 and worst <= 1e-5
