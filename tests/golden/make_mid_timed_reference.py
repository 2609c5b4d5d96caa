"""Write tests/golden/mid_bandlimited_oracle.npz: the float64 oracle HHFFBPA of
the 16384-position, 64-frequency, 128x128x64-voxel handheld workload with
band-limited plan choices (S = 3, Q = 4, band-limited weights, T = 4,
gamma = (2.2, 2.2, 2.6)); with ``--gamma-leaf 1.8,1.8,2.2``
tests/golden/mid_bandlimited_leaf_oracle.npz, the benchmarked choices (the leaf
grids at that oversampling).  Two forms of the level-1 sum:

* "linear": range profiles at U = 4 read by linear interpolation (the timed form);
* "eq4":    eq. (4) itself (what the ES parity mode approximates to ~1e-6).

Stored per form: the image at 16384 seeded voxels plus the 5x5x5 boxes of the
50 point targets, and 4096 seeded grid points of every depth (node, point,
compressed value).  Calls only oracle/ and workloads/; run from the repository
root (a few minutes per form on 8 cores):

    python tests/golden/make_mid_timed_reference.py
    python tests/golden/make_mid_timed_reference.py --gamma-leaf 1.8,1.8,2.2
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import hhffbp as OH  # noqa: E402
from oracle import plan as OP  # noqa: E402
from workloads import make_config  # noqa: E402

GAMMA = (2.2, 2.2, 2.6)
TAPS = 4
STAGES = 3
RANGE_U = 4


def sample_voxels(w, rng):
    dims = w.grid_dims
    idx = set(rng.choice(w.n_vox, 16384, replace=False).tolist())
    for p in w.target_pos[:50]:
        c = np.rint((p - w.grid_origin) / w.grid_pitch).astype(int)
        for dx in range(-2, 3):
            for dy in range(-2, 3):
                for dz in range(-2, 3):
                    q = c + (dx, dy, dz)
                    if np.all(q >= 0) and np.all(q < dims):
                        idx.add(int((q[0] * dims[1] + q[1]) * dims[2] + q[2]))
    return np.array(sorted(idx), np.int64)


def sample_stages(vals, plan, rng, per_depth=4096):
    out = {}
    for d in range(1, STAGES + 1):
        keys = [k for k in vals if k[0] == d]
        sizes = np.array([vals[k].size for k in keys])
        pick = np.sort(rng.choice(int(sizes.sum()), min(per_depth, int(sizes.sum())),
                                  replace=False))
        starts = np.concatenate([[0], np.cumsum(sizes)])
        node = np.searchsorted(starts, pick, side="right") - 1
        point = pick - starts[node]
        out[d] = (np.array([keys[n][1] for n in node], np.int64), point.astype(np.int64),
                  np.array([vals[keys[n]][p] for n, p in zip(node, point)]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gamma-leaf", default=None, help="leaf grids' oversampling, u,v,n")
    args = ap.parse_args()
    gleaf = None if args.gamma_leaf is None else tuple(float(x) for x in args.gamma_leaf.split(","))
    t0 = time.time()
    w = make_config(1)
    pl = OP.build_plan(w.positions, w.freqs_hz, w.grid_origin, w.grid_pitch, w.grid_dims,
                       STAGES, 4, GAMMA, TAPS, kernel="bandlimited", gamma_leaf=gleaf)
    print(f"plan {time.time() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(29)
    index = sample_voxels(w, rng)
    store = dict(index=index, gamma=np.array(GAMMA), taps=TAPS, stages=STAGES, range_u=RANGE_U)
    if gleaf is not None:
        store["gamma_leaf"] = np.array(gleaf)
    for form, ru in (("linear", RANGE_U), ("eq4", None)):
        img, vals = OH.image(pl, w.echoes, w.positions, keep=True, range_u=ru)
        print(f"{form} image {time.time() - t0:.0f} s", flush=True)
        store[f"{form}_image"] = img.ravel()[index]
        for d, (node, point, v) in sample_stages(vals, pl, np.random.default_rng(31)).items():
            store[f"{form}_d{d}_node"] = node
            store[f"{form}_d{d}_point"] = point
            store[f"{form}_d{d}_value"] = v
    name = "mid_bandlimited_leaf_oracle.npz" if gleaf else "mid_bandlimited_oracle.npz"
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), name)
    np.savez_compressed(out, **store)
    print(f"wrote {out}: {index.size} voxels", flush=True)


if __name__ == "__main__":
    main()
