"""Write tests/golden/mid_oracle_hhffbp.npz: the float64 oracle HHFFBPA on the
128x128x64-voxel, 16384-position, 64-frequency handheld workload (S = 3, Q = 4)
at 4096 seeded voxels plus the 5x5x5 neighbourhoods of its isolated point
targets.  Calls only oracle/ and workloads/; run from the repository root:

    python tests/golden/make_mid_reference.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import hhffbp as OH  # noqa: E402
from oracle import plan as OP  # noqa: E402
from workloads import make_config  # noqa: E402

GAMMA = (3.0, 3.0, 3.5)
TAPS = 4


def main():
    t0 = time.time()
    w = make_config(1)
    dims = w.grid_dims
    pl = OP.build_plan(w.positions, w.freqs_hz, w.grid_origin, w.grid_pitch, dims, 3, 4,
                       GAMMA, TAPS)
    print(f"plan {time.time() - t0:.0f} s", flush=True)
    img = OH.image(pl, w.echoes, w.positions).ravel()
    print(f"image {time.time() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(11)
    idx = set(rng.choice(img.size, 4096, replace=False).tolist())
    for p in w.target_pos[:50]:
        c = np.rint((p - w.grid_origin) / w.grid_pitch).astype(int)
        for dx in range(-2, 3):
            for dy in range(-2, 3):
                for dz in range(-2, 3):
                    q = c + (dx, dy, dz)
                    if np.all(q >= 0) and np.all(q < dims):
                        idx.add(int((q[0] * dims[1] + q[1]) * dims[2] + q[2]))
    index = np.array(sorted(idx), np.int64)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mid_oracle_hhffbp.npz")
    np.savez_compressed(out, index=index, hhffbp=img[index], gamma=np.array(GAMMA), taps=TAPS)
    print(f"wrote {out}: {index.size} voxels", flush=True)


if __name__ == "__main__":
    main()
