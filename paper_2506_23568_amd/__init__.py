"""MI355X (gfx950) HHFFBPA: handheld fast factorised backprojection.

Thin Python binding of ``libhhffbp.so`` (C ABI in ``include/hhffbp.h``).  This
module only marshals arguments: every step of the imaging path runs in the HIP
kernels of the library.  PyTorch supplies device memory and streams.  If the
library has not been built the import still succeeds, but every call raises.
"""
from .binding import (  # noqa: F401
    Plan, HHFFBPError, lib, library_path, STATUS, MODES, RANGE_KERNELS, STORAGE,
    STATS_FIELDS, NOALLOC_WORKSPACE_BYTES, image_stats, stats_dict, loss_grad, box_peaks,
)

__all__ = ["Plan", "HHFFBPError", "lib", "library_path", "hhffbp_image", "image_stats",
           "stats_dict", "loss_grad", "box_peaks"]


def hhffbp_image(echoes, positions, plan):
    """Differentiable HHFFBPA image (see autograd.HHFFBPFunction)."""
    from .autograd import hhffbp_image as _f
    return _f(echoes, positions, plan)
