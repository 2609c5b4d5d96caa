"""GPU image reductions (hhffbp_image_stats / hhffbp_loss_grad / hhffbp_box_peaks)
against the float64 oracle: ragged and empty sizes, ties across blocks, zero
images, with and without a reference; argmax indices bit-exact."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

H = pytest.importorskip("paper_2506_23568_amd")


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _rand(rng, n):
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)


def _cmp_stats(got, ref):
    for k in (0, 1, 2, 3):
        assert abs(got[k] - ref[k]) <= 1e-12 * max(abs(ref[k]), 1e-300), k
    assert got[4] == ref[4] and got[5] == ref[5]
    assert abs(got[6] - ref[6]) <= 1e-12 * max(1.0, abs(ref[6]))
    if np.isnan(ref[7]):
        assert np.isnan(got[7])
    else:
        assert abs(got[7] - ref[7]) <= 1e-12 * ref[7]


@pytest.mark.parametrize("n", [0, 1, 255, 257, 65536, 1000003])
@pytest.mark.parametrize("with_ref", [False, True])
def test_image_stats(torch, n, with_ref):
    from oracle import metrics as OM
    rng = np.random.default_rng(n + 7)
    f = _rand(rng, n)
    r = _rand(rng, n) if with_ref else None
    if n > 300000:
        f[[5, 300000, n - 1]] = 9.0 + 9.0j   # equal maxima in different blocks
    ft = torch.from_numpy(f).cuda()
    rt = torch.from_numpy(r).cuda() if with_ref else None
    got = H.image_stats(ft, rt).cpu().numpy()
    again = H.image_stats(ft, rt).cpu().numpy()
    assert np.array_equal(got, again, equal_nan=True)   # fixed summation order
    ref = OM.stats(f, r)
    print(f"  n={n} ref={with_ref}: H {got[6]:.6f} argmax {int(got[5])}", flush=True)
    _cmp_stats(got, ref)
    if n > 300000:
        assert int(got[5]) == 5


def test_zero_image(torch):
    from oracle import metrics as OM
    f = np.zeros(5000, np.complex64)
    got = H.image_stats(torch.from_numpy(f).cuda()).cpu().numpy()
    _cmp_stats(got, OM.stats(f))
    assert got[6] == 0.0 and got[5] == 0


@pytest.mark.parametrize("with_clean", [False, True])
def test_loss_and_cotangent(torch, with_clean):
    from oracle import loss as OL
    from oracle import metrics as OM
    rng = np.random.default_rng(11)
    n = 70001
    f = _rand(rng, n)
    f[::97] = 0                       # voxels without an entropy term
    c = _rand(rng, n) if with_clean else None
    ft = torch.from_numpy(f).cuda()
    ct = torch.from_numpy(c).cuda() if with_clean else None
    loss, g = H.loss_grad(ft, ct)
    loss = loss.item()
    g = g.cpu().numpy().astype(np.complex128)
    if with_clean:
        ref_l = OL.loss(f, c)
        ref_g = OL.loss_cotangent(f, c)
    else:
        ref_l = OM.entropy(f)
        a = np.abs(f.astype(np.complex128)) ** 2
        S = a.sum()
        lnq = np.zeros(n)
        lnq[a > 0] = np.log(a[a > 0] / S)
        ref_g = np.where(a > 0, -2.0 * (lnq + ref_l) / S, 0.0) * f
    print(f"  loss {loss:.12f} oracle {ref_l:.12f}", flush=True)
    assert abs(loss - ref_l) <= 1e-12 * abs(ref_l)
    assert np.linalg.norm(g - ref_g) <= 1e-6 * np.linalg.norm(ref_g)


def test_box_peaks(torch):
    from oracle import metrics as OM
    rng = np.random.default_rng(13)
    d = (37, 29, 41)
    f = _rand(rng, int(np.prod(d))).reshape(d)
    f[3, 4, 5] = f[3, 4, 30] = f[20, 1, 1] = 12.0       # a three-way tie
    boxes = np.array([[0, 36, 0, 28, 0, 40], [3, 3, 4, 4, 0, 40], [-9, 5, -1, 10, 35, 99],
                      [40, 50, 0, 3, 0, 3], [7, 6, 0, 28, 0, 40], [10, 30, 2, 20, 5, 35],
                      [2, 25, 0, 28, 0, 40]], np.int32)
    got = H.box_peaks(torch.from_numpy(f).cuda(), boxes).cpu().numpy()
    ref = OM.box_peaks(f, boxes)
    print(f"  peaks {got.tolist()}", flush=True)
    assert np.array_equal(got, ref)
    assert got[0] == (3 * 29 + 4) * 41 + 5 and got[3] == -1 and got[4] == -1


def test_weighted_loss(torch):
    """L = w_H H + w_2 ||f - c||^2 / ||c||^2 and its cotangent: the same linear
    combination of the oracle's two terms."""
    from oracle import loss as OL
    from oracle import metrics as OM
    rng = np.random.default_rng(12)
    n = 40000
    f, c = _rand(rng, n), _rand(rng, n)
    wh, w2 = 0.3, 2.5
    loss, g = H.loss_grad(torch.from_numpy(f).cuda(), torch.from_numpy(c).cuda(), w_entropy=wh,
                          w_l2=w2)
    Hf = OM.entropy(f)
    l2 = OL.loss(f, c) - Hf
    g_full = OL.loss_cotangent(f, c)
    fc = f.astype(np.complex128) - c.astype(np.complex128)
    g_l2 = 2 * fc / np.sum(np.abs(c.astype(np.complex128)) ** 2)
    ref_g = wh * (g_full - g_l2) + w2 * g_l2
    assert abs(loss.item() - (wh * Hf + w2 * l2)) <= 1e-12 * abs(wh * Hf + w2 * l2)
    g = g.cpu().numpy().astype(np.complex128)
    assert np.linalg.norm(g - ref_g) <= 1e-6 * np.linalg.norm(ref_g)
