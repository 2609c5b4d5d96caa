"""Point-response metrics of image slices (host, numpy), the quantities of the
paper's Table II: mainlobe width, peak sidelobe ratio (PSLR) and integral
sidelobe ratio (ISLR) of a 1-D cut through a point target, and PSNR of an
image against a reference.

The paper reports them without formulas; the definitions used here:
  mainlobe width  -3 dB (half-power) width of |f|^2 around the peak, linearly
                  interpolated on the monotone flanks
  mainlobe        the samples between the first local minima on either side
  PSLR            10 log10(largest sidelobe |f|^2 / peak |f|^2)
  ISLR            10 log10(sidelobe energy / mainlobe energy)
  PSNR            20 log10(max |f_ref| / RMS(f - f_ref))
"""
import numpy as np


def _flank(p, k, step):
    """Index of the first local minimum walking from the peak k by step (+-1)."""
    q = p[k::step] if step > 0 else p[k::-1]
    falling = np.diff(q) < 0
    n = falling.size if falling.all() else int(np.argmin(falling))
    return k + step * n


def psf_metrics(x, f):
    """(width, pslr_db, islr_db) of the slice f (complex) sampled at x (metres)."""
    x = np.asarray(x, float)
    p = np.abs(np.asarray(f)) ** 2
    k = int(np.argmax(p))
    a, b = _flank(p, k, -1), _flank(p, k, +1)
    h = 0.5 * p[k]
    xl = np.interp(h, p[a:k + 1], x[a:k + 1])
    xr = np.interp(h, p[k:b + 1][::-1], x[k:b + 1][::-1])
    inside = np.zeros(p.size, bool)
    inside[a:b + 1] = True
    side = p[~inside]
    if side.size == 0:
        return float(xr - xl), float("-inf"), float("-inf")
    return (float(xr - xl), float(10 * np.log10(side.max() / p[k])),
            float(10 * np.log10(side.sum() / p[inside].sum())))


def psnr_db(f, ref):
    f = np.asarray(f).ravel()
    ref = np.asarray(ref).ravel()
    err = np.sqrt(np.mean(np.abs(f - ref) ** 2))
    return float(20 * np.log10(np.abs(ref).max() / err))
