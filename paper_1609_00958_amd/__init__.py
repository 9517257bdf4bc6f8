"""MI355X (gfx950) generalized Joseph projector (arXiv 1609.00958).

Forward X-ray projection of a voxel grid with driving-axis aligned sampling
and four-neighbour interpolation (Sec. III, Algorithm 1), its exact adjoint,
BF16/FP16 volume storage and a batched persistent launch, all in hand-written
HIP kernels behind the C ABI declared in include/gjp.h.
"""
from ._lib import (BF16, CONE, F16, F32, PARALLEL, W_LINEAR, W_SPLINE, GJPError,  # noqa: F401
                   lib)
from .projector import (Geometry, autotune, back, forward, forward_batched, forward_naive,  # noqa: F401,E501
                        forward_noalloc,
                        get_forward_tile, project, reset_forward_tile, set_forward_tile, timing_enable, timing_read, timing_reset,
                        views_circular_cone,
                        views_parallel)
from .sart import SART, sart  # noqa: F401

lib()  # load the HIP library now: there is no fallback path

__all__ = [
    "Geometry", "forward", "forward_noalloc", "forward_naive", "back", "forward_batched", "project", "autotune",
    "views_circular_cone", "views_parallel", "set_forward_tile", "get_forward_tile",
    "reset_forward_tile", "timing_enable", "timing_read",
    "timing_reset", "SART", "sart",
    "GJPError",
]
