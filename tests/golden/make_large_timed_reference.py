"""Write the float64 oracle HHFFBPA of the 65536-position, 128-frequency,
256x256x128-voxel handheld workload with band-limited weights (T = 4, gamma =
(2.2, 2.2, 2.6), Q = 4) on 16 voxel bricks of 4 x 4 x 4 (8 around point
targets, 8 seeded):

* tests/golden/large_bandlimited_oracle.npz: S = 3 onto the voxel grid (default);
* tests/golden/large_s4_root_oracle.npz: S = 4 with a compressed root grid
  (``--stages 4 --root-grid``);
* tests/golden/large_s4_root_leaf_oracle.npz: the same with the leaf grids at
  gamma = (1.8, 1.8, 2.2), the benchmarked form
  (``--stages 4 --root-grid --gamma-leaf 1.8,1.8,2.2``);

each in two forms of the level-1 sum:

* "linear": range profiles at U = 4 read by linear interpolation (the timed form);
* "eq4":    eq. (4) itself (what the ES parity mode approximates to ~1e-6).

The oracle evaluates only the bricks' cones (oracle.hhffbp.image_at): the grid
points their stencils reach, depth by depth.  Stored per form: the bricks'
voxels and up to 4096 seeded points of every depth of the cones (node, point,
compressed value); with a root grid depth 0 is the root's lattice.  Calls only
oracle/ and workloads/; run from the repository root (CPU echo synthesis takes
~20 minutes on 8 cores):

    python tests/golden/make_large_timed_reference.py
    python tests/golden/make_large_timed_reference.py --stages 4 --root-grid
    python tests/golden/make_large_timed_reference.py --stages 4 --root-grid --gamma-leaf 1.8,1.8,2.2
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
RANGE_U = 4


def bricks(w, rng):
    dims = np.asarray(w.grid_dims)
    corners = []
    for p in w.target_pos[:200]:
        c = np.rint((p - w.grid_origin) / w.grid_pitch).astype(int) - 2
        if np.all(c >= 0) and np.all(c + 4 <= dims):
            corners.append(c)
        if len(corners) == 8:
            break
    for _ in range(8):
        corners.append(rng.integers(0, dims - 4))
    idx = set()
    r = np.arange(4)
    for c in corners:
        for dx in r:
            for dy in r:
                for dz in r:
                    q = c + (dx, dy, dz)
                    idx.add(int((q[0] * dims[1] + q[1]) * dims[2] + q[2]))
    return np.array(sorted(idx), np.int64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stages", type=int, default=3)
    ap.add_argument("--root-grid", action="store_true")
    ap.add_argument("--gamma-leaf", default=None, help="leaf grids' oversampling, u,v,n")
    args = ap.parse_args()
    stages, root = args.stages, args.root_grid
    gleaf = None if args.gamma_leaf is None else tuple(float(x) for x in args.gamma_leaf.split(","))
    name = "large_bandlimited_oracle.npz" if (stages, root, gleaf) == (3, False, None) else \
        f"large_s{stages}{'_root' if root else ''}{'_leaf' if gleaf else ''}_oracle.npz"
    t0 = time.time()
    w = make_config(2)
    print(f"echoes {time.time() - t0:.0f} s", flush=True)
    pl = OP.build_plan(w.positions, w.freqs_hz, w.grid_origin, w.grid_pitch, w.grid_dims,
                       stages, 4, GAMMA, TAPS, kernel="bandlimited", root_grid=root,
                       gamma_leaf=gleaf)
    print(f"plan {time.time() - t0:.0f} s", flush=True)
    index = bricks(w, np.random.default_rng(37))
    store = dict(index=index, gamma=np.array(GAMMA), taps=TAPS, stages=stages, range_u=RANGE_U,
                 root_grid=root)
    if gleaf is not None:
        store["gamma_leaf"] = np.array(gleaf)
    top = 0 if root else 1
    for form, ru in (("linear", RANGE_U), ("eq4", None)):
        img, kept = OH.image_at(pl, w.echoes, w.positions, index, range_u=ru, keep=True)
        print(f"{form} cone {time.time() - t0:.0f} s: "
              + ", ".join(f"depth {d} {sum(v[0].size for k, v in kept.items() if k[0] == d)}"
                          for d in range(top, stages + 1)), flush=True)
        store[f"{form}_image"] = img
        rng = np.random.default_rng(41)
        for d in range(top, stages + 1):
            keys = sorted(k for k in kept if k[0] == d)
            node = np.concatenate([np.full(kept[k][0].size, k[1], np.int64) for k in keys])
            point = np.concatenate([kept[k][0] for k in keys]).astype(np.int64)
            val = np.concatenate([kept[k][1] for k in keys])
            pick = np.sort(rng.choice(node.size, min(4096, node.size), replace=False))
            store[f"{form}_d{d}_node"] = node[pick]
            store[f"{form}_d{d}_point"] = point[pick]
            store[f"{form}_d{d}_value"] = val[pick]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), name)
    np.savez_compressed(out, **store)
    print(f"wrote {out}: {index.size} voxels", flush=True)


if __name__ == "__main__":
    main()
