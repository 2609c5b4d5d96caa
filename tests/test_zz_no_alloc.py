"""hhffbp_image_noalloc (the library's own per-device workspace) against
hhffbp_image with a caller workspace, through the C ABI: the same image bit for
bit on two calls in a row, the second with a smaller input; a plan that needs
more workspace than the library holds is refused before any launch."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

H = pytest.importorskip("paper_2506_23568_amd")


def _say(msg):
    print(msg, flush=True)


def test_noalloc_matches_image_twice(small):
    import torch

    w = small
    cases = [
        # the small workload's full size, then a smaller input: half the
        # positions and an eighth of the voxels
        (w.positions, w.echoes, w.grid_origin, w.grid_dims),
        (w.positions[:512], w.echoes[:512], w.grid_origin + 8 * w.grid_pitch, (16, 16, 8)),
    ]
    for k, (pos, ech_np, origin, dims) in enumerate(cases):
        _say(f"noalloc call {k}: {pos.shape[0]} positions, grid {dims}")
        pl = H.Plan(pos, w.freqs_hz, origin, w.grid_pitch, dims, stages=2, merge_factor=4,
                    oversample=(2.2, 2.2, 2.6), interp_kernel="bandlimited",
                    range_kernel="linear", range_oversample=4.0)
        assert pl.workspace_bytes() <= H.NOALLOC_WORKSPACE_BYTES
        ech = torch.from_numpy(ech_np.astype(np.complex64)).cuda()
        ref = pl.image(ech)
        got = torch.full(dims, complex(np.nan, np.nan), dtype=torch.complex64, device="cuda")
        pl.image_noalloc(ech, out=got)
        # and at device positions of the caller's (the position pass runs too)
        moved = torch.from_numpy(pos + 1e-4).cuda()
        ref_m = pl.image(ech, positions=moved)
        got_m = pl.image_noalloc(ech, positions=moved)
        torch.cuda.synchronize()
        a, b = got.cpu().numpy(), ref.cpu().numpy()
        _say(f"  max |noalloc - image| {np.abs(a - b).max():.3e}")
        assert np.array_equal(a, b)
        assert np.array_equal(got_m.cpu().numpy(), ref_m.cpu().numpy())


def test_noalloc_refuses_a_plan_beyond_its_workspace(small):
    import torch

    w = small
    # 262144 positions (the small walk repeated with sub-millimetre offsets):
    # the direct mode's range profiles alone need more than 256 MiB
    rep = 256
    pos = np.concatenate([w.positions + 1e-5 * k for k in range(rep)])
    pl = H.Plan(pos, w.freqs_hz, w.grid_origin, w.grid_pitch, w.grid_dims, mode="direct_rc",
                range_kernel="linear", range_oversample=16.0)
    need = pl.workspace_bytes()
    _say(f"workspace {need} bytes, library array {H.NOALLOC_WORKSPACE_BYTES}")
    assert need > H.NOALLOC_WORKSPACE_BYTES
    ech = torch.zeros((pos.shape[0], w.n_f), dtype=torch.complex64, device="cuda")
    out = torch.full(w.grid_dims, 7.0 + 1.0j, dtype=torch.complex64, device="cuda")
    with pytest.raises(H.HHFFBPError) as e:
        pl.image_noalloc(ech, out=out)
    assert e.value.status == -5
    torch.cuda.synchronize()
    assert bool((out == 7.0 + 1.0j).all())
