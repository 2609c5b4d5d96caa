"""Range compression (eq. 2): the split-bfloat16 GEMM against the float32 MFMA
GEMM, and through direct BP on its profiles against float64 eq. (4).

The split GEMM represents each float32 operand to 2^-27 of itself and keeps every
partial product above 2^-26, so both GEMMs carry float32 accumulation error:
images formed from either set of profiles differ by NRMSE <= 1e-6 and by no single
value above 5e-5 of the RMS (the parity tests' per-value rule: a bright target's
peak stands far above the RMS, and float32 rounding there is ~1e-7 of the peak),
and direct BP on the split profiles stays within the same 1e-5 of eq. (4) as the
float32 ones (ES range kernel, W = 7, U = 2).  The ragged case takes 13
frequencies (K = 26 reals, not a multiple of the 16-deep MFMA step: the register
form) and 1000 positions (not a multiple of the 64-row tile); the direct-load form
(K a multiple of 16) runs with ragged rows and with one, two and four k steps, and
the B-resident form (K a multiple of 64, two or more row tiles a wave) at the large
workload's size, with a ragged last tile and with aperture weights."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

H = pytest.importorskip("paper_2506_23568_amd")
REG, DMA, BRES = 1, 2, 3  # hhffbp_plan_info.range_gemm_form of the split GEMM


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _args(pos, freqs, w):
    return (pos, freqs, w.grid_origin, w.grid_pitch, w.grid_dims)


def _image(torch, plan, echoes):
    ech = torch.from_numpy(np.ascontiguousarray(echoes).astype(np.complex64)).cuda()
    img = plan.image(ech)
    torch.cuda.synchronize()
    return img.cpu().numpy().astype(np.complex128)


def _nrmse(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _max_rel(a, ref):
    return float(np.abs(a - ref).max() / np.sqrt(np.mean(np.abs(ref) ** 2)))


def _compare(torch, pos, freqs, echoes, w, form=None, **kw):
    """Images with either GEMM; `form`: the split GEMM's kernel form the plan must report."""
    imgs = {}
    for g in ("split_bf16", "f32"):
        plan = H.Plan(*_args(pos, freqs, w), range_gemm=g, **kw)
        if g == "split_bf16" and form is not None:
            assert plan.info()["range_gemm_form"] == form
        imgs[g] = _image(torch, plan, echoes)
    e, m = _nrmse(imgs["split_bf16"], imgs["f32"]), _max_rel(imgs["split_bf16"], imgs["f32"])
    _say(f"  split vs f32 GEMM: NRMSE {e:.2e}, max {m:.2e} of the RMS")
    assert e <= 1e-6 and m <= 5e-5
    return imgs


def test_split_gemm_direct_small(torch, small):
    from oracle import hhffbp as OH
    from workloads import voxel_centres
    _say("direct_rc on the small workload, split vs float32 GEMM and vs eq. (4)")
    imgs = _compare(torch, small.positions, small.freqs_hz, small.echoes, small, form=DMA, mode="direct_rc")
    vox = voxel_centres(small.grid_origin, small.grid_pitch, small.grid_dims)
    ref = OH.direct_bp(small.positions, small.freqs_hz, small.echoes, vox).reshape(small.grid_dims)
    e = _nrmse(imgs["split_bf16"], ref)
    _say(f"  split GEMM direct BP vs eq. (4): {e:.2e}")
    assert e <= 1e-5


def test_split_gemm_ragged(torch, small):
    from oracle import hhffbp as OH
    from workloads import voxel_centres
    pos, freqs = small.positions[:1000], small.freqs_hz[:13]
    echoes = small.echoes[:1000, :13]
    _say("direct_rc, 1000 positions x 13 frequencies: split vs float32 GEMM and vs eq. (4)")
    imgs = _compare(torch, pos, freqs, echoes, small, form=REG, mode="direct_rc")
    vox = voxel_centres(small.grid_origin, small.grid_pitch, small.grid_dims)
    ref = OH.direct_bp(pos, freqs, echoes, vox).reshape(small.grid_dims)
    e = _nrmse(imgs["split_bf16"], ref)
    _say(f"  split GEMM direct BP vs eq. (4): {e:.2e}")
    assert e <= 1e-5


def test_split_gemm_weights(torch, small):
    """Aperture weights scale the GEMM's echo rows: the split path applies them
    before splitting, as the float32 path does."""
    w = np.random.default_rng(7).uniform(0.2, 3.0, small.positions.shape[0])
    _say("direct_rc with aperture weights up to 3: split vs float32 GEMM")
    _compare(torch, small.positions, small.freqs_hz, small.echoes, small, form=DMA, mode="direct_rc", weights=w)


def test_split_gemm_hhffbpa_mid(torch):
    """The benchmarked HHFFBPA form on the mid workload with either GEMM."""
    from workloads import make_config
    w = make_config(1, synth_device="cuda")
    _say("HHFFBPA mid (band-limited, S = 3, linear U = 4, leaf grids (1.8, 1.8, 2.2)): split vs float32 GEMM")
    _compare(torch, w.positions, w.freqs_hz, w.echoes, w, form=DMA, stages=3, merge_factor=4, interp_taps=4,
             interp_kernel="bandlimited", oversample=(2.2, 2.2, 2.6), oversample_leaf=(1.8, 1.8, 2.2),
             range_kernel="linear", range_oversample=4.0)


@pytest.mark.parametrize("n_pos,n_f,form", [(1000, 32, 2), (300, 8, 2), (777, 16, 2)])
def test_split_gemm_direct_load_edges(torch, small, n_pos, n_f, form):
    """The direct-load form (K % 16 == 0): row counts that are not a multiple of
    the block's 256 rows, and K of one, two and four 16-deep steps (the ring's
    prologue and last-step waits)."""
    from oracle import hhffbp as OH
    from workloads import voxel_centres
    pos, freqs = small.positions[:n_pos], small.freqs_hz[:n_f]
    echoes = small.echoes[:n_pos, :n_f]
    _say(f"direct_rc, {n_pos} positions x {n_f} frequencies (K = {2 * n_f}): split vs float32 GEMM, eq. (4)")
    imgs = _compare(torch, pos, freqs, echoes, small, form=form, mode="direct_rc")
    vox = voxel_centres(small.grid_origin, small.grid_pitch, small.grid_dims)
    ref = OH.direct_bp(pos, freqs, echoes, vox).reshape(small.grid_dims)
    e = _nrmse(imgs["split_bf16"], ref)
    _say(f"  split GEMM direct BP vs eq. (4): {e:.2e}")
    assert e <= 1e-5


@pytest.fixture(scope="module")
def large_scene():
    from workloads import make_config
    return make_config(2, synth_device="cuda")


@pytest.mark.parametrize("n_pos,n_f,weighted", [(65521, 128, False), (65536, 128, True), (131072, 64, False)])
def test_split_gemm_b_resident_large(torch, large_scene, n_pos, n_f, weighted):
    """The B-resident form, which takes over where every wave gets two or more
    32-row tiles: the large workload's positions (65521: a ragged last tile) on
    its voxel grid (direct BP's range extent at U = 4: N_r = 160, ten column
    tiles in four groups, the last group's two tiles past N clamped), the large
    workload's K = 256 (144 KB of resident fragments), with and without aperture
    weights scaling the finished rows; and the positions taken twice (131072
    rows) with 64 frequencies: K = 128 (two k groups of the prefetch), N_r = 96
    in two column groups, 16 row streams per XCD; split vs float32 GEMM through
    direct BP (linear range kernel, U = 4, the timed form's)."""
    w = large_scene
    reps = -(-n_pos // w.positions.shape[0])
    pos = np.concatenate([w.positions] * reps)[:n_pos]
    echoes = np.concatenate([w.echoes[:, :n_f]] * reps)[:n_pos]
    freqs = w.freqs_hz[:n_f]
    kw = {}
    if weighted:
        kw["weights"] = np.random.default_rng(11).uniform(0.2, 3.0, n_pos)
    _say(f"direct_rc on the large grid, {n_pos} positions x {n_f} frequencies (K = {2 * n_f}), "
         f"weights {weighted}: B-resident split vs float32 GEMM")
    _compare(torch, pos, freqs, echoes, w, form=BRES, mode="direct_rc", range_kernel="linear",
             range_oversample=4.0, **kw)
