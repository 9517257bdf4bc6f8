"""ctypes loader for libgjp.so (argument marshalling only).

The library is built in-tree by ``paper_1609_00958_amd/build.py`` (or
``__graft_entry__.build()``). There is no fallback: if the shared library is
missing or fails to load, importing the projector raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgjp.so")

GJP_OK, GJP_EINVAL, GJP_ENOMEM, GJP_EHIP, GJP_EUNSUPPORTED = 0, -1, -2, -3, -4
F32, BF16, F16 = 0, 1, 2
CONE, PARALLEL = 0, 1
W_LINEAR, W_SPLINE = 0, 1
CLIP_CYLINDER = 1  # gjp_geometry_desc.flags

# Every symbol include/gjp.h declares.
EXPORTS = (
    "gjp_create_geometry", "gjp_destroy_geometry", "gjp_forward_project",
    "gjp_forward_project_noalloc", "gjp_forward_project_naive", "gjp_back_project",
    "gjp_forward_project_batched", "gjp_views_circular_cone", "gjp_views_parallel",
    "gjp_count_samples", "gjp_autotune_forward", "gjp_set_forward_tile", "gjp_get_forward_tile",
    "gjp_timing_enable",
    "gjp_timing_reset",
    "gjp_timing_read", "gjp_last_error", "gjp_sart_residual", "gjp_sart_update",
)


class GeometryDesc(ctypes.Structure):
    _fields_ = [
        ("vol_shape", ctypes.c_int32 * 3),
        ("voxel_size", ctypes.c_double * 3),
        ("vol_center", ctypes.c_double * 3),
        ("n_views", ctypes.c_int32),
        ("n_u", ctypes.c_int32),
        ("n_v", ctypes.c_int32),
        ("beam", ctypes.c_int32),
        ("views", ctypes.POINTER(ctypes.c_double)),
        ("weight", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]


class GJPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gjp status {status}: {msg}")
        self.status = status


_LIB = None


def lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1609_00958_amd/build.py")
    # torch supplies device memory and streams; load its HIP runtime first so
    # that libgjp binds to that same runtime (one HIP/HSA runtime per process).
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                              ctypes.c_double)
    f64p = ctypes.POINTER(ctypes.c_double)
    L.gjp_create_geometry.argtypes = [ctypes.POINTER(GeometryDesc), ctypes.POINTER(vp)]
    L.gjp_destroy_geometry.argtypes = [vp]
    L.gjp_forward_project.argtypes = [vp, vp, i32, vp, vp]
    L.gjp_forward_project_noalloc.argtypes = [vp, vp, i32, vp, vp]
    L.gjp_forward_project_naive.argtypes = [vp, vp, i32, vp, vp]
    L.gjp_back_project.argtypes = [vp, vp, vp, vp]
    L.gjp_forward_project_batched.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                              ctypes.POINTER(i32), ctypes.POINTER(vp), vp]
    L.gjp_views_circular_cone.argtypes = [i32, f64, f64, f64, f64, i32, i32, f64p]
    L.gjp_views_parallel.argtypes = [i32, f64, f64, i32, i32, f64p]
    L.gjp_count_samples.argtypes = [vp, ctypes.POINTER(u64)]
    L.gjp_autotune_forward.argtypes = [vp, vp, i32, vp, vp, ctypes.POINTER(i32)]
    L.gjp_set_forward_tile.argtypes = [vp, i32, i32, i32, i32]
    L.gjp_get_forward_tile.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                       ctypes.POINTER(i32)]
    L.gjp_timing_enable.argtypes = [i32]
    L.gjp_timing_reset.argtypes = []
    L.gjp_timing_read.argtypes = [ctypes.c_char_p, f64p, ctypes.POINTER(i64)]
    L.gjp_sart_residual.argtypes = [i64, vp, vp, vp, vp, vp]
    L.gjp_sart_update.argtypes = [i64, vp, vp, vp, ctypes.c_float, i32, vp]
    L.gjp_last_error.argtypes = []
    L.gjp_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "gjp_last_error":
            getattr(L, name).restype = ctypes.c_int
    _LIB = L
    return L


def check(status: int) -> None:
    if status != GJP_OK:
        msg = lib().gjp_last_error().decode(errors="replace")
        raise GJPError(int(status), msg)
