"""Pins of the oracle's spectrum-compression geometry (Sec. III), CPU only.

The analytic maps are checked against what the paper states about them: the
gradient of Phi is the spectrum centre k_c, the Jacobian of (u, v, n) is the LLT
matrix T_s up to the orientation of u and v, k7 equals k6 on boresight with a
curl-free k7, the transformed local spectrum fits the unit box, and |det T_s|
on boresight equals the paper's closed form for the sample count.
"""
import math

import numpy as np
import pytest

from oracle import geometry as G

C0 = 299792458.0
K = 2 * math.pi * np.linspace(24e9, 40e9, 64) / C0
KMIN, KMAX = float(K.min()), float(K.max())
RECTS = [(-0.0375, 0.0, 0.0, 0.0375), (-0.15, -0.1125, -0.15, -0.1125), (-0.075, 0.075, -0.075, 0.075)]


def _points(rng, n=40):
    return rng.uniform([-0.1, -0.1, 0.25], [0.1, 0.1, 0.35], (n, 3))


def _fd_grad(fun, p, h=1e-7):
    g = np.zeros_like(p)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        g[:, a] = (fun(p + e) - fun(p - e)) / (2 * h)
    return g


@pytest.mark.parametrize("rect", RECTS)
def test_grad_phi_is_spectrum_centre(rect):
    """grad Phi = k_c = (k5 + k7) / 2 (eq. dp_kc with eq. sdc_phi)."""
    p = _points(np.random.default_rng(0))
    g = _fd_grad(lambda q: G.phi(q, rect, KMIN, KMAX), p)
    kc = G.kc(p, rect, KMIN, KMAX)
    assert np.max(np.abs(g - kc) / np.linalg.norm(kc, axis=1, keepdims=True)) < 1e-7


@pytest.mark.parametrize("rect", RECTS)
def test_jacobian_is_llt_matrix(rect):
    """d(u, v, n)/d(x, y, z) equals T_s = [v1; v2; v3] / 2pi (eq. lltmatrix) with
    u and v oriented opposite to v1, v2 (eq. uvw_xyz as printed)."""
    p = _points(np.random.default_rng(1))
    Jfd = np.stack([_fd_grad(lambda q, a=a: G.uvn(q, rect, KMIN, KMAX)[:, a], p) for a in range(3)], 1)
    Ja = G.jacobian(p, rect, KMIN, KMAX)
    Ts = G.llt_matrix(p, rect, KMIN, KMAX)
    scale = np.abs(Ts).max()
    assert np.max(np.abs(Jfd - Ja)) < 1e-6 * scale
    assert np.max(np.abs(Ja[:, 0] + Ts[:, 0])) < 1e-9 * scale
    assert np.max(np.abs(Ja[:, 1] + Ts[:, 1])) < 1e-9 * scale
    assert np.max(np.abs(Ja[:, 2] - Ts[:, 2])) < 1e-9 * scale


@pytest.mark.parametrize("rect", RECTS)
def test_k7_equals_k6_on_boresight_and_is_curl_free(rect):
    x0, x1, y0, y1 = rect
    zs = np.linspace(0.2, 0.5, 7)
    p = np.column_stack([np.full(7, 0.5 * (x0 + x1)), np.full(7, 0.5 * (y0 + y1)), zs])
    kp = G.key_points(p, rect, KMIN, KMAX)
    assert np.max(np.abs(kp["k7"] - kp["k6"])) < 1e-9 * 2 * KMAX
    # sqrt(r^2 - D^2) = 4 z on boresight (the condition beta is solved from)
    r = G.r_sum(p, rect)
    assert np.max(np.abs(np.sqrt(r * r - G.dsq(rect)) - 4 * zs)) < 1e-12
    # curl k7 = 0 everywhere (eq. k7_curlfree)
    q = _points(np.random.default_rng(2), 10)
    h = 1e-6

    def k7(pts):
        return G.key_points(pts, rect, KMIN, KMAX)["k7"]

    d = np.zeros((q.shape[0], 3, 3))  # d[:, i, j] = d k7_i / d x_j
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        d[:, :, j] = (k7(q + e) - k7(q - e)) / (2 * h)
    curl = np.stack([d[:, 2, 1] - d[:, 1, 2], d[:, 0, 2] - d[:, 2, 0], d[:, 1, 0] - d[:, 0, 1]], 1)
    grad_scale = np.abs(d).max()
    assert np.max(np.abs(curl)) < 1e-6 * grad_scale


def test_local_spectrum_fits_unit_box():
    """After SDC and LLT the local spectrum lies in [-pi, pi]^3 up to a few per
    cent (Fig. locspcm): components of J^-T (k0(p', p, k) - k_c)."""
    rng = np.random.default_rng(3)
    worst = 0.0
    for rect in RECTS:
        p = _points(rng, 60)
        J = G.jacobian(p, rect, KMIN, KMAX)
        kc = G.kc(p, rect, KMIN, KMAX)
        x0, x1, y0, y1 = rect
        for _ in range(40):
            pp = np.array([rng.uniform(x0, x1), rng.uniform(y0, y1), 0.0])
            k = rng.uniform(KMIN, KMAX)
            k0 = G.k0(pp[None, :], p, k)
            w = np.linalg.solve(np.transpose(J, (0, 2, 1)), (k0 - kc)[:, :, None])[:, :, 0]
            worst = max(worst, np.abs(w).max() / math.pi)
    assert worst < 1.15
    assert worst > 0.8  # the box is nearly filled: unity sampling is almost tight


@pytest.mark.parametrize("m,M", [(1, 4), (2, 4), (3, 4)])
def test_det_ts_on_boresight_matches_paper_closed_form(m, M):
    """|det T_s0| at the subarray centre axis equals the closed form of
    eq. 4_subimgsmppresimp (without V(D)) for a square subarray of side
    L 2^((m-M)/2), L the full aperture."""
    L, z = 0.45, 0.4
    s = L * 2 ** ((m - M) / 2)
    rect = (-s / 2, s / 2, -s / 2, s / 2)
    p = np.array([[0.0, 0.0, z]])
    det_ts = abs(np.linalg.det(G.llt_matrix(p, rect, KMIN, KMAX)[0]))
    det_j = abs(np.linalg.det(G.jacobian(p, rect, KMIN, KMAX)[0]))
    closed = (L ** 2 * KMAX ** 2 * (KMAX - 2 * KMIN * z / math.sqrt(2 ** (m - M + 1) * L ** 2 + 4 * z ** 2))
              / (2 ** (M - m - 2) * math.pi ** 3 * (2 ** (m - M) * L ** 2 + 4 * z ** 2)))
    assert abs(det_ts - closed) <= 1e-10 * closed
    assert abs(det_j - closed) <= 1e-10 * closed


def test_sample_ratio_between_levels_tends_to_two():
    """eq. 4_smpratiopresimp -> 2 when the subarray is much smaller than z (eq. smpratiosim2)."""
    L, z, M = 0.45, 0.4, 12

    def det_at(m):
        s = L * 2 ** ((m - M) / 2)
        rect = (-s / 2, s / 2, -s / 2, s / 2)
        return abs(np.linalg.det(G.llt_matrix(np.array([[0.0, 0.0, z]]), rect, KMIN, KMAX)[0]))

    # a level-(m+1) subarray covers twice the area: twice the samples of the union
    assert abs(det_at(2) / det_at(1) - 2.0) < 1e-3
