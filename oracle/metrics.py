"""Image reductions in float64 (test infrastructure; only tests/ and bench.py use it).

Definitions (readings of quantities the paper reports without a formula):
  NRMSE   ||f - r||_2 / ||r||_2 over all voxels, complex
  PSNR    20 log10(max |r| / RMS(f - r)), on complex images (Sec. V reports
          PSNR of images against a reference without defining it)
  entropy H = -sum_v q_v ln q_v, q_v = |f_v|^2 / sum_u |f_u|^2, terms with q_v = 0
          counted as 0 (autofocus quality measure, Sec. I)
  stats   the eight reductions of one image pass, in the order the library
          reports them: sum |f|^2, sum |r|^2, sum |f - r|^2, sum |f|^2 ln |f|^2,
          max |f|^2, its lowest linear index, H, NRMSE
  peaks   per voxel box, the lowest linear index of the largest |f|^2

|f|^2 of a complex64 value is formed as re^2 + im^2 in float64 (both squares
exact), so argmax decisions are reproducible bit for bit.
"""
import numpy as np


def _abs2(f):
    f = np.asarray(f)
    if f.dtype == np.complex64:
        re = f.real.astype(np.float64)
        im = f.imag.astype(np.float64)
        return re * re + im * im
    f = np.asarray(f, np.complex128)
    return f.real * f.real + f.imag * f.imag


def nrmse(f, r):
    f = np.asarray(f, np.complex128).ravel()
    r = np.asarray(r, np.complex128).ravel()
    return float(np.linalg.norm(f - r) / np.linalg.norm(r))


def psnr_db(f, r):
    f = np.asarray(f, np.complex128).ravel()
    r = np.asarray(r, np.complex128).ravel()
    rms = np.sqrt(np.mean(np.abs(f - r) ** 2))
    return float(20.0 * np.log10(np.max(np.abs(r)) / rms))


def entropy(f):
    a = _abs2(f).ravel()
    S = a.sum()
    if S == 0.0:
        return 0.0
    q = a[a > 0] / S
    return float(-np.sum(q * np.log(q)))


def stats(f, r=None):
    a = _abs2(f).ravel()
    S = float(a.sum())
    nz = a > 0
    alna = float(np.sum(a[nz] * np.log(a[nz])))
    if a.size:
        i = int(np.argmax(a))  # first occurrence = lowest index
        amax = float(a[i])
    else:
        i, amax = -1, 0.0
    H = entropy(f)
    if r is None:
        r2, d2, e = 0.0, 0.0, float("nan")
    else:
        fr = np.asarray(f, np.complex128).ravel()
        rr = np.asarray(r, np.complex128).ravel()
        r2 = float(np.sum(np.abs(rr) ** 2))
        d2 = float(np.sum(np.abs(fr - rr) ** 2))
        e = float(np.sqrt(d2 / r2)) if r2 > 0 else float("nan")
    return np.array([S, r2, d2, alna, amax, float(i), H, e])


def box_peaks(f, boxes):
    """f: [d0, d1, d2]; boxes [n, 6] inclusive (x_lo, x_hi, y_lo, y_hi, z_lo, z_hi),
    clipped to the grid; -1 for a box with no voxel inside."""
    a = _abs2(f)
    d = a.shape
    out = []
    for b in np.asarray(boxes).reshape(-1, 6):
        lo = [max(int(b[2 * k]), 0) for k in range(3)]
        hi = [min(int(b[2 * k + 1]), d[k] - 1) for k in range(3)]
        if any(h < l for l, h in zip(lo, hi)):
            out.append(-1)
            continue
        best, bi = -1.0, -1
        for ix in range(lo[0], hi[0] + 1):
            for iy in range(lo[1], hi[1] + 1):
                row = a[ix, iy, lo[2]:hi[2] + 1]
                k = int(np.argmax(row))
                if row[k] > best:
                    best, bi = row[k], (ix * d[1] + iy) * d[2] + lo[2] + k
        out.append(bi)
    return np.array(out, np.int64)


def psf_metrics(x, f):
    """Point-response metrics of a 1-D complex slice f sampled at positions x
    (the paper's Table II reports them without definitions; readings):
      mainlobe width  the -3 dB width of |f|^2 around its peak, linear
                      interpolation of |f|^2 between samples
      PSLR            10 log10(max sidelobe |f|^2 / peak |f|^2), sidelobes being
                      the samples beyond the first local minimum on each side
      ISLR            10 log10(sum of sidelobe |f|^2 / sum of mainlobe |f|^2)
    Returns (width, pslr_db, islr_db)."""
    x = np.asarray(x, float)
    p = np.abs(np.asarray(f, np.complex128)) ** 2
    k = int(np.argmax(p))
    half = 0.5 * p[k]
    # half-power crossings
    i = k
    while i > 0 and p[i - 1] > half:
        i -= 1
    xl = x[i] if i == 0 else x[i - 1] + (half - p[i - 1]) / (p[i] - p[i - 1]) * (x[i] - x[i - 1])
    j = k
    while j < p.size - 1 and p[j + 1] > half:
        j += 1
    xr = x[j] if j == p.size - 1 else x[j] + (p[j] - half) / (p[j] - p[j + 1]) * (x[j + 1] - x[j])
    # first minima
    a = k
    while a > 0 and p[a - 1] < p[a]:
        a -= 1
    b = k
    while b < p.size - 1 and p[b + 1] < p[b]:
        b += 1
    main = p[a:b + 1].sum()
    side = np.concatenate([p[:a], p[b + 1:]])
    pslr = 10 * np.log10(side.max() / p[k]) if side.size else -np.inf
    islr = 10 * np.log10(side.sum() / main) if side.size else -np.inf
    return float(xr - xl), float(pslr), float(islr)
