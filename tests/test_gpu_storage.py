"""Half-precision storage (echoes, range profiles and subimages as IEEE half or
bfloat16 pairs; sums and phases in float32) against the float64 oracle.

Expected rounding error per stored stage: 2^-12 RMS relative for half, 2^-9 for
bfloat16; five stored stages (echoes, profiles, leaf and two merge levels).
Bounds: half <= 1e-3, bfloat16 <= 1e-2 NRMSE against the oracle HHFFBPA; both
within -30 dB of eq. (4).
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

H = pytest.importorskip("paper_2506_23568_amd")
GAMMA = (3.0, 3.0, 3.5)
TAPS = 4
BOUND = {"f16": 1e-3, "bf16": 1e-2}


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _args(w):
    return (w.positions, w.freqs_hz, w.grid_origin, w.grid_pitch, w.grid_dims)


def _nrmse(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _echoes(torch, w, storage):
    return H.Plan.pack_echoes(torch.from_numpy(w.echoes), storage).cuda()


@pytest.fixture(scope="module")
def oracle_small(small):
    from oracle import hhffbp as OH
    from oracle import plan as OP
    from workloads import voxel_centres
    vox = voxel_centres(small.grid_origin, small.grid_pitch, small.grid_dims)
    bp = OH.direct_bp(small.positions, small.freqs_hz, small.echoes, vox).reshape(small.grid_dims)
    op = OP.build_plan(*_args(small), 2, 4, GAMMA, TAPS)
    img, vals = OH.image(op, small.echoes, small.positions, keep=True)
    return bp, img, vals


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_half_storage_small(torch, small, oracle_small, storage):
    bp, ref, vals = oracle_small
    pl = H.Plan(*_args(small), stages=2, oversample=GAMMA, interp_taps=TAPS, storage=storage)
    ws = pl._workspace(torch)
    img = pl.image(_echoes(torch, small, storage), workspace=ws)
    torch.cuda.synchronize()
    img = img.cpu().numpy().astype(np.complex128)
    e = _nrmse(img, ref)
    e_bp = _nrmse(img, bp)
    worst = 0.0
    for (d, i), v in vals.items():
        g = pl.workspace_view(ws, d, i).cpu().numpy().astype(np.complex128)
        worst = max(worst, _nrmse(g, v))
    _say(f"  {storage}: vs oracle HHFFBPA {e:.2e} ({20 * np.log10(e):.1f} dB), worst stage "
         f"{worst:.2e}; vs eq.4 {20 * np.log10(e_bp):.1f} dB")
    assert e <= BOUND[storage]
    assert worst <= BOUND[storage]
    assert 20 * np.log10(e_bp) <= -30.0


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_half_storage_direct(torch, small, oracle_small, storage):
    bp = oracle_small[0]
    pl = H.Plan(*_args(small), mode="direct_rc", storage=storage)
    img = pl.image(_echoes(torch, small, storage))
    torch.cuda.synchronize()
    e = _nrmse(img.cpu().numpy().astype(np.complex128), bp)
    _say(f"  direct {storage}: vs eq.4 {e:.2e}")
    assert e <= BOUND[storage]


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_half_storage_mid(torch, storage):
    """Full-size mid workload: half-precision image against the float32 one and
    the float32 direct BP on the full grid."""
    from workloads import make_config
    w = make_config(1)
    kw = dict(stages=3, oversample=GAMMA, interp_taps=TAPS)
    ref = H.Plan(*_args(w), **kw).image(torch.from_numpy(w.echoes.astype(np.complex64)).cuda())
    d = H.Plan(*_args(w), mode="direct_rc").image(torch.from_numpy(w.echoes.astype(np.complex64)).cuda())
    img = H.Plan(*_args(w), storage=storage, **kw).image(_echoes(torch, w, storage))
    torch.cuda.synchronize()
    e = (torch.linalg.norm(img - ref) / torch.linalg.norm(ref)).item()
    e_d = (torch.linalg.norm(img - d) / torch.linalg.norm(d)).item()
    _say(f"  mid {storage}: vs float32 HHFFBPA {e:.2e}; vs float32 direct {20 * np.log10(e_d):.1f} dB")
    assert e <= 2 * BOUND[storage]
    assert 20 * np.log10(e_d) <= -30.0


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_half_storage_backward(torch, small, storage):
    """Gradients from half echoes against those from float32 echoes."""
    kw = dict(stages=2, oversample=GAMMA, interp_taps=TAPS)
    p32 = H.Plan(*_args(small), **kw)
    ph = H.Plan(*_args(small), storage=storage, **kw)
    rng = np.random.default_rng(5)
    g = rng.standard_normal(small.grid_dims) + 1j * rng.standard_normal(small.grid_dims)
    gt = torch.from_numpy(g.astype(np.complex64)).cuda()
    s32, p_32 = p32.backward(torch.from_numpy(small.echoes.astype(np.complex64)).cuda(), gt)
    sh, p_h = ph.backward(_echoes(torch, small, storage), gt)
    es = (torch.linalg.norm(sh - s32) / torch.linalg.norm(s32)).item()
    ep = (torch.linalg.norm(p_h - p_32) / torch.linalg.norm(p_32)).item()
    _say(f"  backward {storage}: echo gradient {es:.2e}, position gradient {ep:.2e}")
    assert es <= 1e-6          # the echo gradient does not depend on the echoes
    assert ep <= BOUND[storage]


@pytest.mark.parametrize("storage", ["c64", "f16", "bf16"])
def test_poisoned_workspace(torch, small, storage):
    """Every workspace byte that forward or backward reads is written first: a
    workspace filled with NaN bytes gives the same image and gradients as a
    zeroed one."""
    kw = dict(stages=2, oversample=GAMMA, interp_taps=TAPS, storage=storage)
    pl = H.Plan(*_args(small), **kw)
    ech = _echoes(torch, small, storage)
    rng = np.random.default_rng(6)
    g = rng.standard_normal(small.grid_dims) + 1j * rng.standard_normal(small.grid_dims)
    gt = torch.from_numpy(g.astype(np.complex64)).cuda()
    nb = pl.workspace_bytes_backward()
    out = []
    for fill in (0, 255):
        ws = torch.full((nb,), fill, dtype=torch.uint8, device="cuda")
        img = pl.image(ech, workspace=ws)
        ws.fill_(fill)
        ge, gp = pl.backward(ech, gt, workspace=ws)
        torch.cuda.synchronize()
        out.append((img.clone(), ge.clone(), gp.clone()))
    (i0, s0, p0), (i1, s1, p1) = out
    assert torch.isfinite(torch.view_as_real(i1)).all()
    assert torch.isfinite(torch.view_as_real(s1)).all() and torch.isfinite(p1).all()
    assert torch.equal(i0, i1)
    assert (torch.linalg.norm(s1 - s0) / torch.linalg.norm(s0)).item() <= 1e-6
    assert (torch.linalg.norm(p1 - p0) / torch.linalg.norm(p0)).item() <= 1e-6
