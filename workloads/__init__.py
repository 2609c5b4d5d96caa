"""Seeded synthetic handheld-scan inputs (trajectories, frequencies, scenes, echoes).

This module is shared by the oracle and by the GPU library's tests and benchmark.
It holds no part of the imaging method: no backprojection, no subarray geometry,
no interpolation.  It only draws inputs and synthesises echoes with the monostatic
Born signal model (Sec. II-A, eq. 1), propagation loss neglected.
"""
from .configs import (  # noqa: F401
    C0, Workload, make_config, synth_echoes, voxel_centres, grid_box,
    trajectory_error, CONFIG_NAMES,
)
