"""Write tests/golden/large_oracle.npz for the 65536-position, 128-frequency,
256x256x128-voxel handheld workload (44 strokes + 20 dense walks; 200 points
and a 5000-scatterer slab): float64 eq. (4) at a stratified voxel sample (the
5x5x5 neighbourhoods of the isolated point targets plus 4096 seeded voxels),
and the oracle's compressed level-1 subimages (S = 3, Q = 4) at 4096 seeded
leaf grid points.  Calls only oracle/ and workloads/; run from the repository
root (about 15 minutes on 8 cores, most of it echo synthesis):

    python tests/golden/make_large_reference.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import hhffbp as OH  # noqa: E402
from oracle import plan as OP  # noqa: E402
from workloads import make_config, voxel_centres  # noqa: E402

GAMMA = (3.0, 3.0, 3.5)
TAPS = 4
STAGES = 3


def isolated_points(w, min_sep=0.01, margin=2):
    """Point targets (the first 200) with no other scatterer within min_sep and
    at least ``margin`` voxels inside the grid; their nearest voxels."""
    dims = np.asarray(w.grid_dims)
    out = []
    for i, p in enumerate(w.target_pos[:200]):
        d = np.linalg.norm(w.target_pos - p, axis=1)
        d[i] = np.inf
        c = np.rint((p - w.grid_origin) / w.grid_pitch).astype(int)
        if d.min() >= min_sep and np.all(c >= margin) and np.all(c < dims - margin):
            out.append(c)
    return np.array(out, np.int64).reshape(-1, 3)


def main():
    t0 = time.time()
    w = make_config(2)
    print(f"echoes {time.time() - t0:.0f} s", flush=True)
    dims = w.grid_dims
    rng = np.random.default_rng(17)
    uniform = rng.choice(w.n_vox, 4096, replace=False)
    idx = set(uniform.tolist())
    centres = isolated_points(w)
    for c in centres:
        for dx in range(-2, 3):
            for dy in range(-2, 3):
                for dz in range(-2, 3):
                    q = c + (dx, dy, dz)
                    idx.add(int((q[0] * dims[1] + q[1]) * dims[2] + q[2]))
    index = np.array(sorted(idx), np.int64)
    vox = voxel_centres(w.grid_origin, w.grid_pitch, dims)[index]
    bp = OH.direct_bp(w.positions, w.freqs_hz, w.echoes, vox)
    print(f"eq.4 on {index.size} voxels {time.time() - t0:.0f} s", flush=True)
    pl = OP.build_plan(w.positions, w.freqs_hz, w.grid_origin, w.grid_pitch, dims, STAGES, 4,
                       GAMMA, TAPS)
    print(f"plan {time.time() - t0:.0f} s", flush=True)
    leaves = [(i, n) for i, n in enumerate(pl.levels[STAGES]) if not n.empty]
    sizes = np.array([n.lattice.size for _, n in leaves])
    pick = rng.choice(int(sizes.sum()), 4096, replace=False)
    starts = np.concatenate([[0], np.cumsum(sizes)])
    leaf_idx, pt_idx, vals = [], [], []
    for k, (i, n) in enumerate(leaves):
        sel = np.sort(pick[(pick >= starts[k]) & (pick < starts[k + 1])] - starts[k])
        if sel.size == 0:
            continue
        vals.append(OH.leaf_bp_at(pl, n, w.echoes, w.positions, sel))
        leaf_idx.append(np.full(sel.size, i, np.int64))
        pt_idx.append(sel)
    print(f"leaf points {time.time() - t0:.0f} s", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "large_oracle.npz")
    np.savez_compressed(out, index=index, bp=bp, uniform=np.isin(index, uniform), centres=centres, leaf=np.concatenate(leaf_idx),
                        point=np.concatenate(pt_idx), leaf_val=np.concatenate(vals),
                        gamma=np.array(GAMMA), taps=TAPS, stages=STAGES)
    print(f"wrote {out}: {index.size} voxels, {sum(v.size for v in vals)} leaf points", flush=True)


if __name__ == "__main__":
    main()
