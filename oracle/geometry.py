"""Analytic spectrum-compression geometry of one subarray (Sec. III), float64.

Test infrastructure (oracle).  A subarray SA is described by its rectangle
``rect = (x0, x1, y0, y1)`` in the aperture plane z' = 0 (the key points are
defined with z' = 0, Sec. III), and by the band limits ``kmin, kmax``.
Points ``p`` are (N, 3) arrays in metres.

Functions follow the paper's notation:

* ``k0``          local spectrum key map  k0(p', p, k) = 2k grad|p - p'|   (eq. kfun_posp)
* ``clamp_xy``    x'_0, y'_0: nearest aperture coordinate inside SA       (Sec. III)
* ``key_points``  k1 .. k7                                                (Sec. III, eq. spv_scl)
* ``r_sum``       r, sum of distances to the four SA vertices             (eq. 4r_sum)
* ``beta``        beta(r) keeping k7 = k6 on boresight                    (Sec. III)
* ``phi``         SDC phase Phi, grad Phi = k_c                           (eq. sdc_phi)
* ``uvn``         LLT coordinates (u, v, n)                               (eq. uvw_xyz)
* ``jacobian``    rows grad u, grad v, grad n of ``uvn``
* ``llt_matrix``  T_s = [v1; v2; v3] / 2pi                                (eq. lltmatrix)

Reading of the paper: the extents inside beta, Phi and n are the subarray's own
(x'_max,SA - x'_min,SA etc.); only then is sqrt(r^2 - D^2) = 4z on boresight,
which is the condition beta is solved from.
"""
import numpy as np

PI = np.pi


def _split(rect):
    x0, x1, y0, y1 = (float(v) for v in rect)
    return x0, x1, y0, y1


def dsq(rect):
    """D^2 = 4 (x'_max - x'_min)^2 + 4 (y'_max - y'_min)^2 for the subarray."""
    x0, x1, y0, y1 = _split(rect)
    return 4.0 * (x1 - x0) ** 2 + 4.0 * (y1 - y0) ** 2


def corners(rect):
    x0, x1, y0, y1 = _split(rect)
    return [(x0, y0), (x0, y1), (x1, y0), (x1, y1)]


def dist_plane(p, ax, ay):
    """|p - (ax, ay, 0)| for points p (N, 3); ax, ay scalars or (N,) arrays."""
    return np.sqrt((p[:, 0] - ax) ** 2 + (p[:, 1] - ay) ** 2 + p[:, 2] ** 2)


def k0(pprime, p, k):
    """k0(p', p, k) = 2k (p - p') / |p - p'|  (eq. kxyz_posp / kfun_posp)."""
    d = p - pprime
    return 2.0 * k * d / np.linalg.norm(d, axis=-1, keepdims=True)


def clamp_xy(p, rect):
    """x'_0 = clip(x, x'_min, x'_max), y'_0 = clip(y, y'_min, y'_max)."""
    x0, x1, y0, y1 = _split(rect)
    return np.clip(p[:, 0], x0, x1), np.clip(p[:, 1], y0, y1)


def r_sum(p, rect):
    """r = sum over the four subarray vertices of |p - vertex| (eq. 4r_sum)."""
    return sum(dist_plane(p, cx, cy) for cx, cy in corners(rect))


def beta(r, rect, kmin, kmax):
    """beta(r) = kmax r / (kmin sqrt(r^2 - D^2))."""
    return kmax * r / (kmin * np.sqrt(r * r - dsq(rect)))


def key_points(p, rect, kmin, kmax):
    """k1..k7 at points p; returns a dict of (N, 3) arrays."""
    x0, x1, y0, y1 = _split(rect)
    xp0, yp0 = clamp_xy(p, rect)
    z = np.zeros(p.shape[0])

    def P(ax, ay):
        return np.stack([np.broadcast_to(ax, z.shape), np.broadcast_to(ay, z.shape), z], 1)

    k1 = k0(P(x0, yp0), p, kmax)
    k2 = k0(P(x1, yp0), p, kmax)
    k3 = k0(P(xp0, y0), p, kmax)
    k4 = k0(P(xp0, y1), p, kmax)
    k5 = sum(k0(P(cx, cy), p, kmin) for cx, cy in corners(rect)) / 4.0
    k6 = 2.0 * kmax * k5 / np.linalg.norm(k5, axis=1, keepdims=True)
    r = r_sum(p, rect)
    k7 = beta(r, rect, kmin, kmax)[:, None] * k5
    return dict(k1=k1, k2=k2, k3=k3, k4=k4, k5=k5, k6=k6, k7=k7)


def kc(p, rect, kmin, kmax):
    """Centre of the local spectrum k_c = (k5 + k7) / 2 (Sec. III)."""
    kp = key_points(p, rect, kmin, kmax)
    return 0.5 * (kp["k5"] + kp["k7"])


def phi(p, rect, kmin, kmax):
    """SDC phase Phi = (kmax/4) sqrt(r^2 - D^2) + (kmin/4) r (eq. sdc_phi)."""
    r = r_sum(p, rect)
    return 0.25 * kmax * np.sqrt(r * r - dsq(rect)) + 0.25 * kmin * r


def uvn(p, rect, kmin, kmax):
    """(u, v, n)(x, y, z) of eq. uvw_xyz, as an (N, 3) array."""
    x0, x1, y0, y1 = _split(rect)
    xp0, yp0 = clamp_xy(p, rect)
    u = (kmax / PI) * (dist_plane(p, x0, yp0) - dist_plane(p, x1, yp0))
    v = (kmax / PI) * (dist_plane(p, xp0, y0) - dist_plane(p, xp0, y1))
    r = r_sum(p, rect)
    n = (kmax / (4 * PI)) * np.sqrt(r * r - dsq(rect)) - (kmin / (4 * PI)) * r
    return np.stack([u, v, n], axis=1)


def _unit_from(p, ax, ay):
    d = np.stack([p[:, 0] - ax, p[:, 1] - ay, p[:, 2]], axis=1)
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def jacobian(p, rect, kmin, kmax):
    """(N, 3, 3) Jacobian d(u, v, n)/d(x, y, z) of ``uvn``.

    The clamped coordinates x'_0, y'_0 contribute nothing: where they follow x
    or y the corresponding component of p - p'_0 is zero.
    """
    x0, x1, y0, y1 = _split(rect)
    xp0, yp0 = clamp_xy(p, rect)
    gu = (kmax / PI) * (_unit_from(p, x0, yp0) - _unit_from(p, x1, yp0))
    gv = (kmax / PI) * (_unit_from(p, xp0, y0) - _unit_from(p, xp0, y1))
    r = r_sum(p, rect)
    gr = sum(_unit_from(p, cx, cy) for cx, cy in corners(rect))
    S = np.sqrt(r * r - dsq(rect))
    gS = (r / S)[:, None] * gr
    gn = (kmax / (4 * PI)) * gS - (kmin / (4 * PI)) * gr
    return np.stack([gu, gv, gn], axis=1)


def grad_phi(p, rect, kmin, kmax):
    """Analytic grad Phi (for tests against k_c)."""
    r = r_sum(p, rect)
    gr = sum(_unit_from(p, cx, cy) for cx, cy in corners(rect))
    S = np.sqrt(r * r - dsq(rect))
    return (0.25 * kmax * (r / S))[:, None] * gr + 0.25 * kmin * gr


def llt_matrix(p, rect, kmin, kmax):
    """T_s = [v1^T; v2^T; v3^T] / 2pi with v1 = k2-k1, v2 = k4-k3, v3 = k7-k5."""
    kp = key_points(p, rect, kmin, kmax)
    v1 = kp["k2"] - kp["k1"]
    v2 = kp["k4"] - kp["k3"]
    v3 = kp["k7"] - kp["k5"]
    return np.stack([v1, v2, v3], axis=1) / (2 * PI)
