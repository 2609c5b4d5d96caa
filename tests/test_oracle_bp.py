"""Pins of the oracle's eq. (4) sums (CPU only).

Each test ties the oracle to something other than itself: pure-Python loops,
the matched-filter closed form of a point target, linearity, the adjoint
identity and finite differences.
"""
import math

import numpy as np
import pytest

from oracle import brute, native
from workloads import C0, synth_echoes, voxel_centres

pytestmark = pytest.mark.filterwarnings("ignore")


def _tiny(seed=1, n_pos=5, n_f=4, n_pts=6):
    rng = np.random.default_rng(seed)
    pos = np.column_stack([rng.uniform(-0.02, 0.02, (n_pos, 2)), rng.normal(0, 1e-3, n_pos)])
    fr = np.sort(rng.uniform(20e9, 30e9, n_f))
    s = rng.standard_normal((n_pos, n_f)) + 1j * rng.standard_normal((n_pos, n_f))
    pts = rng.uniform([-0.03, -0.03, 0.2], [0.03, 0.03, 0.3], (n_pts, 3))
    return pos, fr, s, pts


def test_eq4_matches_pure_python_loops():
    pos, fr, s, pts = _tiny()
    k = 2 * math.pi * fr / C0
    got = native.bp_eq4(pos, k, s, pts)
    ref = np.array(brute.bp_eq4(pos.tolist(), fr.tolist(), s.tolist(), pts.tolist()))
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_echo_synthesis_matches_pure_python_loops():
    pos, fr, _, pts = _tiny(seed=2)
    amp = np.array([1.0, 0.5j, -0.3, 2.0, 1 - 1j, 0.1])
    got = synth_echoes(pos, fr, pts, amp)
    ref = np.array(brute.echoes_eq1(pos.tolist(), fr.tolist(), pts.tolist(), amp.tolist()))
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_point_target_closed_form():
    """One unit scatterer on a voxel centre, no noise: the matched-filter sum is
    exactly N_pos * N_f with zero phase there (eq. 1 into eq. 4), and by the
    Cauchy-Schwarz bound every other voxel is strictly smaller."""
    rng = np.random.default_rng(3)
    n_pos, n_f = 64, 16
    pos = np.column_stack([rng.uniform(-0.04, 0.04, (n_pos, 2)), rng.normal(0, 1e-3, n_pos)])
    fr = np.linspace(26e9, 40e9, n_f)
    origin, pitch, dims = np.array([-0.006, -0.006, 0.244]), np.full(3, 2e-3), (7, 7, 7)
    vox = voxel_centres(origin, pitch, dims)
    t = vox[3 * 49 + 3 * 7 + 3][None, :]  # voxel (3, 3, 3)
    s = synth_echoes(pos, fr, t, np.ones(1))
    f = native.bp_eq4(pos, 2 * math.pi * fr / C0, s, vox)
    peak = np.argmax(np.abs(f))
    assert peak == 3 * 49 + 3 * 7 + 3
    assert abs(f[peak] - n_pos * n_f) <= 1e-9 * n_pos * n_f
    others = np.delete(np.abs(f), peak)
    assert others.max() < n_pos * n_f * (1 - 1e-6)


def test_linearity_superposition_and_global_phase():
    pos, fr, s1, pts = _tiny(seed=4)
    _, _, s2, _ = _tiny(seed=5)
    k = 2 * math.pi * fr / C0
    a, b = 0.7 - 0.2j, -1.3 + 0.5j
    f1, f2 = native.bp_eq4(pos, k, s1, pts), native.bp_eq4(pos, k, s2, pts)
    f12 = native.bp_eq4(pos, k, a * s1 + b * s2, pts)
    assert np.max(np.abs(f12 - (a * f1 + b * f2))) <= 1e-12 * np.max(np.abs(f12))
    th = 0.9
    fr_ = native.bp_eq4(pos, k, s1 * np.exp(1j * th), pts)
    assert np.max(np.abs(fr_ - f1 * np.exp(1j * th))) <= 1e-12 * np.max(np.abs(f1))


def test_multi_target_image_is_sum_of_single_target_images():
    pos, fr, _, pts = _tiny(seed=6, n_pts=3)
    k = 2 * math.pi * fr / C0
    grid = _tiny(seed=7, n_pts=20)[3]
    amps = np.array([1.0, -0.5j, 0.25])
    f_all = native.bp_eq4(pos, k, synth_echoes(pos, fr, pts, amps), grid)
    f_sum = sum(native.bp_eq4(pos, k, synth_echoes(pos, fr, pts[i:i + 1], amps[i:i + 1]), grid)
                for i in range(3))
    assert np.max(np.abs(f_all - f_sum)) <= 1e-11 * np.max(np.abs(f_all))


def test_adjoint_dot_identity():
    """<A s, g> = <s, A^H g> with A the eq. (4) operator."""
    pos, fr, s, pts = _tiny(seed=8, n_pts=9)
    k = 2 * math.pi * fr / C0
    rng = np.random.default_rng(9)
    g = rng.standard_normal(pts.shape[0]) + 1j * rng.standard_normal(pts.shape[0])
    lhs = np.vdot(g, native.bp_eq4(pos, k, s, pts))
    rhs = np.vdot(native.bp_eq4_adjoint(pos, k, pts, g), s)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_position_gradient_against_central_differences():
    pos, fr, s, pts = _tiny(seed=10, n_pts=7)
    k = 2 * math.pi * fr / C0
    rng = np.random.default_rng(11)
    w = rng.standard_normal(pts.shape[0]) + 1j * rng.standard_normal(pts.shape[0])

    def loss(p):
        return float(np.real(np.vdot(w, native.bp_eq4(p, k, s, pts))))

    g = native.bp_eq4_dpos(pos, k, s, pts, w)
    h = 1e-7
    for i in range(pos.shape[0]):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, a] += h
            pm[i, a] -= h
            fd = (loss(pp) - loss(pm)) / (2 * h)
            assert abs(fd - g[i, a]) <= 1e-6 * max(1.0, np.max(np.abs(g)))


def _rc_case():
    from workloads import make_config
    w = make_config(0)
    vox = voxel_centres(w.grid_origin, w.grid_pitch, w.grid_dims)[::37]
    k = 2 * math.pi * w.freqs_hz / C0
    return w, vox, k


def test_rc_linear_converges_to_eq4_at_second_order():
    """Range compression with linear interpolation approaches eq. (4) as the
    range oversampling U grows, with error ~ dR^2 (an index or sign slip would
    leave an O(1) or O(dR) error), and the kernel pre-correction removes most
    of it (a missing or wrong correction keeps the mean attenuation)."""
    from oracle import hhffbp as OH
    w, vox, k = _rc_case()
    ref = native.bp_eq4(w.positions, k, w.echoes, vox)
    e, e_raw = [], []
    for U in (4, 8, 16, 32):
        dR = math.pi / (U * (k.max() - k.min()))
        e.append(OH.nrmse(native.bp_rc_linear(w.positions, k, w.echoes, vox, dR), ref))
        e_raw.append(OH.nrmse(native.bp_rc_linear(w.positions, k, w.echoes, vox, dR,
                                                  precorrect=False), ref))
    for a, b in zip(e, e[1:]):
        assert 3.3 < a / b < 4.7
    for a, b in zip(e, e_raw):
        assert a < b / 5
    assert e[1] < 1e-3          # U = 8: below -60 dB
    # the driver function is the same sum
    assert np.array_equal(OH.direct_bp_linear(w.positions, w.freqs_hz, w.echoes, vox, 8),
                          native.bp_rc_linear(w.positions, k, w.echoes, vox,
                                              OH.range_step(k.min(), k.max(), 8)))


def test_rc_linear_linearity_and_global_phase():
    w, vox, k = _rc_case()
    dR = math.pi / (8 * (k.max() - k.min()))
    rng = np.random.default_rng(5)
    s2 = rng.standard_normal(w.echoes.shape) + 1j * rng.standard_normal(w.echoes.shape)
    f1 = native.bp_rc_linear(w.positions, k, w.echoes, vox, dR)
    f2 = native.bp_rc_linear(w.positions, k, s2, vox, dR)
    a, b = 0.7 - 0.2j, -1.3 + 0.5j
    f12 = native.bp_rc_linear(w.positions, k, a * w.echoes + b * s2, vox, dR)
    assert np.linalg.norm(f12 - (a * f1 + b * f2)) <= 1e-12 * np.linalg.norm(f12)
    th = np.exp(0.9j)
    fp = native.bp_rc_linear(w.positions, k, th * w.echoes, vox, dR)
    assert np.linalg.norm(fp - th * f1) <= 1e-12 * np.linalg.norm(f1)
