"""Pins of the oracle's image reductions (CPU only): closed forms, a hand-computed
entropy, Parseval through an FFT, and a masked-argmax restatement of the box
peaks."""
import numpy as np

from oracle import metrics as OM


def _rand(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


def test_entropy_closed_forms():
    rng = np.random.default_rng(0)
    n = 1000
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, n))
    assert abs(OM.entropy(3.0 * ph) - np.log(n)) < 1e-12          # uniform magnitude
    one = np.zeros(n, complex)
    one[17] = 2 - 1j
    assert OM.entropy(one) == 0.0                                  # one non-zero voxel
    two = np.zeros(n, complex)
    two[[3, 900]] = [1j, -1.0]
    assert abs(OM.entropy(two) - np.log(2)) < 1e-15
    # |f|^2 = 1, 2, 3, 4: q = 0.1 .. 0.4, H worked out by hand
    f = np.sqrt(np.array([1.0, 2.0, 3.0, 4.0])) * np.exp(1j * np.array([0.3, 1.0, 2.0, 5.0]))
    assert abs(OM.entropy(f) - 1.2798542258336676) < 1e-14
    assert OM.entropy(np.zeros(5, complex)) == 0.0
    g = _rand(rng, 300)
    assert abs(OM.entropy(8.0 * g) - OM.entropy(g)) < 1e-12      # scale invariance (exact scaling)
    assert abs(OM.entropy(7.5 * g.astype(np.complex128)) - OM.entropy(g)) < 1e-12
    assert abs(OM.entropy(g[::-1]) - OM.entropy(g)) < 1e-12      # order invariance


def test_nrmse_and_psnr_closed_forms():
    rng = np.random.default_rng(1)
    r = _rand(rng, (8, 9, 10)).astype(np.complex128)
    assert abs(OM.nrmse(1.25 * r, r) - 0.25) < 1e-14
    f = r.copy()
    f.flat[123] += 0.5j
    assert abs(OM.nrmse(f, r) - 0.5 / np.linalg.norm(r)) < 1e-14
    c = 0.01 * np.exp(0.7j)
    assert abs(OM.psnr_db(r + c, r) - 20 * np.log10(np.abs(r).max() / 0.01)) < 1e-10


def test_stats_definitions():
    rng = np.random.default_rng(2)
    f = _rand(rng, 4097)
    r = _rand(rng, 4097)
    s = OM.stats(f, r)
    # Parseval through the FFT
    assert abs(s[0] - np.sum(np.abs(np.fft.fft(f.astype(np.complex128))) ** 2) / f.size) < 1e-9 * s[0]
    assert abs(s[1] - np.sum(np.abs(np.fft.fft(r.astype(np.complex128))) ** 2) / r.size) < 1e-9 * s[1]
    assert abs(s[7] - np.sqrt(s[2] / s[1])) < 1e-15
    # entropy from the sums: H = ln S - sum a ln a / S
    assert abs(s[6] - (np.log(s[0]) - s[3] / s[0])) < 1e-12
    assert s[4] == np.max(np.abs(f.astype(np.complex128)) ** 2)
    # ties go to the lowest index
    g = np.zeros(50, np.complex64)
    g[[7, 31]] = [3 + 4j, -5.0]
    g[40] = 4 - 3j
    t = OM.stats(g)
    assert t[5] == 7 and t[4] == 25.0 and np.isnan(t[7]) and t[1] == 0.0
    e = OM.stats(np.zeros(0, np.complex64))
    assert e[5] == -1 and e[0] == 0.0 and e[6] == 0.0


def test_box_peaks_against_masked_argmax():
    rng = np.random.default_rng(3)
    d = (9, 7, 11)
    f = _rand(rng, d)
    f[2, 3, 4] = f[2, 3, 9] = 10.0          # a tie inside one box
    boxes = np.array([[0, 8, 0, 6, 0, 10],   # whole grid
                      [2, 2, 3, 3, 0, 10],   # the tie
                      [-5, 1, -1, 2, 8, 30],  # clipped
                      [20, 30, 0, 1, 0, 1],  # outside
                      [4, 3, 0, 6, 0, 10]])  # empty (lo > hi)
    got = OM.box_peaks(f, boxes)
    a = np.abs(f.astype(np.complex128)) ** 2
    ix, iy, iz = np.meshgrid(*[np.arange(n) for n in d], indexing="ij")
    for b, g in zip(boxes, got):
        m = ((ix >= b[0]) & (ix <= b[1]) & (iy >= b[2]) & (iy <= b[3]) & (iz >= b[4]) & (iz <= b[5]))
        if not m.any():
            assert g == -1
            continue
        assert g == int(np.argmax(np.where(m, a, -1.0).ravel()))
    assert got[1] == (2 * 7 + 3) * 11 + 4


def test_psf_metrics_of_a_sinc():
    """|sinc(x / rho)| sampled at rho / 100 over +-20 rho: -3 dB width 0.8859 rho,
    PSLR -13.26 dB, ISLR from the sine integral (scipy), for sidelobes out to
    20 rho: 10 log10((S(20) - S(1)) / S(1)), S(a) = (2/pi) Si(2 pi a)."""
    from scipy.special import sici
    rho = 9.7e-3
    x = np.arange(-2000, 2001) * rho / 100
    f = np.sinc(x / rho) * np.exp(0.3j)
    w, pslr, islr = OM.psf_metrics(x, f)
    S = lambda a: (2 / np.pi) * sici(2 * np.pi * a)[0]
    assert abs(w / rho - 0.88589) < 2e-4
    assert abs(pslr - 20 * np.log10(0.217234)) < 0.01
    assert abs(islr - 10 * np.log10((S(20) - S(1)) / S(1))) < 0.01
    # shifted and scaled copies measure the same
    w2, p2, i2 = OM.psf_metrics(x + 0.03, 5.0 * f)
    assert abs(w2 - w) < 1e-12 and abs(p2 - pslr) < 1e-9 and abs(i2 - islr) < 1e-9
