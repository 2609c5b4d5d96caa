"""Peak-voxel comparison of isolated point targets (the point-target analysis of
Sec. V-A, Table II, applied voxel by voxel).

A point target takes part when
* it is isolated: no other scatterer of the scene lies within 3 resolution cells
  of it along every axis at once (|dx| < 3 rho_x and |dy| < 3 rho_y and
  |dz| < 3 rho_z), with the cells of a matched filter over the aperture and
  the band:
      rho_z = c / (2 (f_max - f_min))                      (range)
      rho_a = lambda_c / (4 sin(atan(L_a / (2 R))))        (a = x, y)
  L_a the aperture's extent along a, R the target's depth in front of the
  mean antenna plane and lambda_c the wavelength at the band's centre;
* its nearest voxel lies at least 2 voxels inside the grid, so that the
  5 x 5 x 5 box around it is whole.

The peak of a box is its largest |f|, ties to the lowest linear index.  The
float64 reference's peak is compared only where its top-two gap,
(|f|_1 - |f|_2) / |f|_1, exceeds 1e-3; otherwise the target is "ambiguous".
"""
import numpy as np

C0 = 299792458.0
ISOLATION_CELLS = 3.0
MARGIN = 2
MIN_GAP = 1e-3


def resolution_cells(w, p):
    """(rho_x, rho_y, rho_z) in metres for a target at p."""
    f = np.asarray(w.freqs_hz, float)
    rho_z = C0 / (2.0 * (f.max() - f.min()))
    lam = C0 / (0.5 * (f.max() + f.min()))
    ext = w.positions[:, :2].max(0) - w.positions[:, :2].min(0)
    depth = p[2] - w.positions[:, 2].mean()
    theta = np.arctan(0.5 * ext / depth)
    rho = lam / (4.0 * np.sin(theta))
    return np.array([rho[0], rho[1], rho_z])


def isolated_targets(w, n_points):
    """Indices (among the first ``n_points`` scene entries, the point targets) of
    the isolated targets, and their nearest voxels (k, 3)."""
    dims = np.asarray(w.grid_dims)
    idx, centres = [], []
    for i in range(n_points):
        p = w.target_pos[i]
        c = np.rint((p - w.grid_origin) / w.grid_pitch).astype(np.int64)
        if np.any(c < MARGIN) or np.any(c >= dims - MARGIN):
            continue
        d = np.abs(w.target_pos - p) / resolution_cells(w, p)
        d[i] = np.inf
        if np.any(np.all(d < ISOLATION_CELLS, axis=1)):
            continue
        idx.append(i)
        centres.append(c)
    return np.array(idx, np.int64), np.array(centres, np.int64).reshape(-1, 3)


def box_linear(dims, c):
    """Linear indices (z fastest) of the 5 x 5 x 5 box around voxel c, in
    (dx, dy, dz) lexicographic order."""
    r = np.arange(-MARGIN, MARGIN + 1)
    dx, dy, dz = np.meshgrid(r, r, r, indexing="ij")
    return (((c[0] + dx) * dims[1] + c[1] + dy) * dims[2] + c[2] + dz).ravel()


def peak_gap(vals):
    """(position of the largest |v| (lowest on ties), relative top-two gap)."""
    a = np.abs(np.asarray(vals))
    k = int(np.argmax(a))
    s = np.sort(a)
    return k, float((s[-1] - s[-2]) / s[-1])


def compare(dims, centres, ref_boxes, img_flat):
    """Peak comparison over the boxes.  ``ref_boxes`` (k, 125) float64 reference
    values in box order, ``img_flat`` the image under test (any indexable of
    linear voxel index).  Returns a dict: compared / matched / ambiguous counts,
    the same at a 1e-2 gap, and per-mismatch (target row, gap, box error
    max|f - f_ref| / max|f_ref|)."""
    out = {"compared": 0, "matched": 0, "ambiguous": 0, "compared_1pct": 0,
           "matched_1pct": 0, "mismatches": []}
    for k, c in enumerate(centres):
        lin = box_linear(dims, c)
        ref = ref_boxes[k]
        got = np.asarray(img_flat[lin])
        pr, gap = peak_gap(ref)
        pg = int(np.argmax(np.abs(got)))
        if gap <= MIN_GAP:
            out["ambiguous"] += 1
            continue
        out["compared"] += 1
        same = pg == pr
        out["matched"] += int(same)
        if gap > 1e-2:
            out["compared_1pct"] += 1
            out["matched_1pct"] += int(same)
        if not same:
            err = float(np.abs(got - ref).max() / np.abs(ref).max())
            out["mismatches"].append((k, round(gap, 5), round(err, 5)))
    return out
