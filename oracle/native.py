"""ctypes access to the oracle's C sums (eq. (4), its adjoint, its position derivative).

Test infrastructure only.  Builds the library on first use if it is missing.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _nthreads():
    """ORACLE_THREADS if set, else the usable cores capped by OMP_NUM_THREADS."""
    n = os.environ.get("ORACLE_THREADS")
    if n:
        return int(n)
    try:
        c = max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        c = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit() and int(omp) > 0:
        c = min(c, int(omp))
    return c


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIBRARY")  # another build (tests/sanitized_suite.py)
        if not path:
            if not os.path.exists(_build.LIB) or (
                    os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
                _build.build()
            path = _build.LIB
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lng = ctypes.c_long
        L.or_bp_eq4.argtypes = [lng, dp, lng, dp, dp, lng, dp, dp, ctypes.c_int]
        L.or_bp_eq4_adjoint.argtypes = [lng, dp, lng, dp, lng, dp, dp, dp, ctypes.c_int]
        L.or_bp_eq4_dpos.argtypes = [lng, dp, lng, dp, dp, lng, dp, dp, dp, ctypes.c_int]
        L.or_bp_rclin.argtypes = [lng, dp, lng, dp, dp, ctypes.c_double, ctypes.c_double, dp,
                                  lng, dp, dp, ctypes.c_int]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c128(a):
    return np.ascontiguousarray(a, np.complex128)


def _f64(a):
    return np.ascontiguousarray(a, np.float64)


def bp_eq4(positions, k, echoes, points, nthreads=None):
    """f(q) = sum_i sum_f s_if exp(+j 2 k_f |q - p'_i|), eq. (4), float64."""
    pos, kk, s, pts = _f64(positions), _f64(k), _c128(echoes), _f64(points)
    assert s.shape == (pos.shape[0], kk.shape[0])
    out = np.zeros(pts.shape[0], np.complex128)
    if pts.shape[0] and pos.shape[0]:
        lib().or_bp_eq4(pos.shape[0], _d(pos), kk.shape[0], _d(kk), _d(s.view(np.float64)),
                        pts.shape[0], _d(pts), _d(out.view(np.float64)),
                        nthreads or _nthreads())
    return out


def bp_eq4_adjoint(positions, k, points, w, nthreads=None):
    """g_if = sum_q w(q) exp(-j 2 k_f |q - p'_i|): the transpose of ``bp_eq4``."""
    pos, kk, pts, ww = _f64(positions), _f64(k), _f64(points), _c128(w)
    g = np.zeros((pos.shape[0], kk.shape[0]), np.complex128)
    if pts.shape[0] and pos.shape[0]:
        lib().or_bp_eq4_adjoint(pos.shape[0], _d(pos), kk.shape[0], _d(kk), pts.shape[0],
                                _d(pts), _d(ww.view(np.float64)), _d(g.view(np.float64)),
                                nthreads or _nthreads())
    return g


def bp_eq4_dpos(positions, k, echoes, points, w, nthreads=None):
    """Gradient of L = sum_q Re{conj(w_q) f(q)} with respect to the positions."""
    pos, kk, s, pts, ww = _f64(positions), _f64(k), _c128(echoes), _f64(points), _c128(w)
    g = np.zeros_like(pos)
    if pts.shape[0] and pos.shape[0]:
        lib().or_bp_eq4_dpos(pos.shape[0], _d(pos), kk.shape[0], _d(kk), _d(s.view(np.float64)),
                             pts.shape[0], _d(pts), _d(ww.view(np.float64)), _d(g),
                             nthreads or _nthreads())
    return g


def linear_precorrection(theta):
    """1 / Lambda(theta), Lambda(theta) = (sin(theta/2) / (theta/2))^2: the Fourier
    transform of the unit triangle (linear interpolation) kernel at theta rad per
    sample.  Dividing the range samples by it removes the interpolation's mean
    attenuation of each frequency (the reading of eq. (2) used here)."""
    h = 0.5 * np.asarray(theta, float)
    out = np.ones_like(h)
    nz = np.abs(h) > 1e-12
    out[nz] = (h[nz] / np.sin(h[nz])) ** 2
    return out


def bp_rc_linear(positions, k, echoes, points, dR, precorrect=True, nthreads=None):
    """Eq. (4) through a range profile sampled every dR (grid R_b = b dR, band
    demodulated to k_c = (k_min + k_max) / 2) and linearly interpolated."""
    pos, kk, s, pts = _f64(positions), _f64(k), _c128(echoes), _f64(points)
    assert s.shape == (pos.shape[0], kk.shape[0])
    kc = 0.5 * (kk.min() + kk.max())
    w = _f64(2.0 * (kk - kc))
    c = _f64(linear_precorrection(w * dR) if precorrect else np.ones_like(w))
    out = np.zeros(pts.shape[0], np.complex128)
    if pts.shape[0] and pos.shape[0]:
        lib().or_bp_rclin(pos.shape[0], _d(pos), kk.shape[0], _d(w), _d(c), float(kc), float(dR),
                          _d(s.view(np.float64)), pts.shape[0], _d(pts),
                          _d(out.view(np.float64)), nthreads or _nthreads())
    return out
