"""Python binding of libgjp: geometry handles, forward / adjoint / batched
projection on torch device tensors, and the autograd Function.

Only argument marshalling happens here; every step of the projection runs in
the library's HIP kernels. PyTorch provides device memory and the stream.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import BF16, CONE, F16, F32, PARALLEL, W_LINEAR, W_SPLINE, check, lib

_BEAMS = {"cone": CONE, "parallel": PARALLEL, CONE: CONE, PARALLEL: PARALLEL}
_WEIGHTS = {"linear": W_LINEAR, "spline": W_SPLINE, W_LINEAR: W_LINEAR, W_SPLINE: W_SPLINE}


def _f64p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def views_circular_cone(n_views: int, sod: float, sdd: float, pitch_u: float, pitch_v: float,
                        n_u: int, n_v: int) -> np.ndarray:
    """Circular cone-beam trajectory about axis 2 (n_views x 12, world units)."""
    out = np.zeros((int(n_views), 12), dtype=np.float64)
    check(lib().gjp_views_circular_cone(int(n_views), float(sod), float(sdd), float(pitch_u),
                                        float(pitch_v), int(n_u), int(n_v), _f64p(out)))
    return out


def views_parallel(n_views: int, pitch_u: float, pitch_v: float, n_u: int, n_v: int):
    out = np.zeros((int(n_views), 12), dtype=np.float64)
    check(lib().gjp_views_parallel(int(n_views), float(pitch_u), float(pitch_v), int(n_u),
                                   int(n_v), _f64p(out)))
    return out


class Geometry:
    """Immutable projection geometry (volume grid + views + detector)."""

    def __init__(self, shape: Sequence[int], views: np.ndarray, n_u: int, n_v: int,
                 beam="cone", voxel_size=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0),
                 weight="linear", clip_cylinder=False):
        self.shape = tuple(int(s) for s in shape)
        self.views = np.ascontiguousarray(views, dtype=np.float64).reshape(-1, 12)
        self.n_u, self.n_v = int(n_u), int(n_v)
        self.beam = _BEAMS[beam]
        self.weight = _WEIGHTS[weight]
        self.voxel_size = tuple(float(x) for x in voxel_size)
        self.center = tuple(float(x) for x in center)
        self.clip_cylinder = bool(clip_cylinder)
        d = _lib.GeometryDesc()
        for k in range(3):
            d.vol_shape[k] = self.shape[k]
            d.voxel_size[k] = self.voxel_size[k]
            d.vol_center[k] = self.center[k]
        d.n_views = self.views.shape[0]
        d.n_u, d.n_v = self.n_u, self.n_v
        d.beam = self.beam
        d.views = _f64p(self.views)
        d.weight = self.weight
        d.flags = _lib.CLIP_CYLINDER if self.clip_cylinder else 0
        h = ctypes.c_void_p()
        check(lib().gjp_create_geometry(ctypes.byref(d), ctypes.byref(h)))
        self._h = h

    @classmethod
    def circular_cone(cls, shape, n_views, n_u, n_v, sod, sdd, pitch_u=1.0, pitch_v=1.0,
                      weight="linear", clip_cylinder=False):
        v = views_circular_cone(n_views, sod, sdd, pitch_u, pitch_v, n_u, n_v)
        return cls(shape, v, n_u, n_v, beam="cone", weight=weight, clip_cylinder=clip_cylinder)

    @classmethod
    def parallel(cls, shape, n_views, n_u, n_v, pitch_u=1.0, pitch_v=1.0, weight="linear",
                 clip_cylinder=False):
        v = views_parallel(n_views, pitch_u, pitch_v, n_u, n_v)
        return cls(shape, v, n_u, n_v, beam="parallel", weight=weight,
                   clip_cylinder=clip_cylinder)

    @classmethod
    def from_config(cls, cfg, weight="linear"):
        clip = bool(getattr(cfg, "clip_cylinder", False))
        if cfg.beam == "cone":
            return cls.circular_cone(cfg.shape, cfg.n_views, cfg.n_u, cfg.n_v, cfg.sod, cfg.sdd,
                                     cfg.pitch_u, cfg.pitch_v, weight=weight, clip_cylinder=clip)
        return cls.parallel(cfg.shape, cfg.n_views, cfg.n_u, cfg.n_v, cfg.pitch_u, cfg.pitch_v,
                            weight=weight, clip_cylinder=clip)

    @property
    def n_views(self) -> int:
        return int(self.views.shape[0])

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("geometry destroyed")
        return self._h

    @property
    def sino_shape(self):
        return (self.n_views, self.n_u, self.n_v)

    def count_samples(self) -> int:
        n = ctypes.c_uint64()
        check(lib().gjp_count_samples(self.handle, ctypes.byref(n)))
        return int(n.value)

    def destroy(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().gjp_destroy_geometry(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16
    if t.dtype == torch.float16:
        return F16
    raise TypeError(f"unsupported volume dtype {t.dtype}")


def _stream(device) -> int:
    torch = _torch()
    return int(torch.cuda.current_stream(device).cuda_stream)


def _check_tensor(t, shape, what):
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


def forward(vol, geom: Geometry, out=None):
    """Sinogram A vol, float32 (n_views, n_u, n_v), on vol's device."""
    torch = _torch()
    _check_tensor(vol, geom.shape, "volume")
    if out is None:
        out = torch.empty(geom.sino_shape, dtype=torch.float32, device=vol.device)
    _check_tensor(out, geom.sino_shape, "sinogram")
    if out.dtype != torch.float32:
        raise TypeError("sinogram must be float32")
    if out.device != vol.device:
        raise ValueError("sinogram and volume must be on the same device")
    with torch.cuda.device(vol.device):
        check(lib().gjp_forward_project(geom.handle, vol.data_ptr(), _dtype_code(vol),
                                        out.data_ptr(), _stream(vol.device)))
    return out


def forward_noalloc(vol, geom: Geometry, out):
    """Sinogram A vol into the caller's float32 `out`, with the padded copies
    in the library's fixed device scratch (no allocation; calls on one device
    must not overlap)."""
    torch = _torch()
    _check_tensor(vol, geom.shape, "volume")
    _check_tensor(out, geom.sino_shape, "sinogram")
    if out.dtype != torch.float32:
        raise TypeError("sinogram must be float32")
    if out.device != vol.device:
        raise ValueError("sinogram and volume must be on the same device")
    with torch.cuda.device(vol.device):
        check(lib().gjp_forward_project_noalloc(geom.handle, vol.data_ptr(), _dtype_code(vol),
                                                out.data_ptr(), _stream(vol.device)))
    return out


def forward_naive(vol, geom: Geometry, out=None):
    """Sinogram A vol from the plain one-lane-per-ray kernel (for comparison)."""
    torch = _torch()
    _check_tensor(vol, geom.shape, "volume")
    if out is None:
        out = torch.empty(geom.sino_shape, dtype=torch.float32, device=vol.device)
    _check_tensor(out, geom.sino_shape, "sinogram")
    if out.dtype != torch.float32:
        raise TypeError("sinogram must be float32")
    if out.device != vol.device:
        raise ValueError("sinogram and volume must be on the same device")
    with torch.cuda.device(vol.device):
        check(lib().gjp_forward_project_naive(geom.handle, vol.data_ptr(), _dtype_code(vol),
                                              out.data_ptr(), _stream(vol.device)))
    return out


def back(sino, geom: Geometry, out=None):
    """Adjoint A^T sino, float32 (n0, n1, n2), on sino's device."""
    torch = _torch()
    _check_tensor(sino, geom.sino_shape, "sinogram")
    if sino.dtype != torch.float32:
        raise TypeError("sinogram must be float32")
    if out is None:
        out = torch.empty(geom.shape, dtype=torch.float32, device=sino.device)
    _check_tensor(out, geom.shape, "volume")
    if out.dtype != torch.float32:
        raise TypeError("adjoint output must be float32")
    if out.device != sino.device:
        raise ValueError("volume and sinogram must be on the same device")
    with torch.cuda.device(sino.device):
        check(lib().gjp_back_project(geom.handle, sino.data_ptr(), out.data_ptr(),
                                     _stream(sino.device)))
    return out


def forward_batched(vols: Sequence, geoms: Sequence[Geometry], outs: Optional[Sequence] = None):
    """Batched forward of independent instances in one persistent launch."""
    torch = _torch()
    n = len(vols)
    if n != len(geoms) or n == 0:
        raise ValueError("vols and geoms must be non-empty and of equal length")
    if outs is None:
        outs = [torch.empty(g.sino_shape, dtype=torch.float32, device=v.device)
                for v, g in zip(vols, geoms)]
    dev = vols[0].device
    for v, g, o in zip(vols, geoms, outs):
        # the batched kernel writes float32 sinograms
        if o.dtype != torch.float32:
            raise TypeError("sinogram must be float32")
        _dtype_code(v)
        _check_tensor(v, g.shape, "volume")
        _check_tensor(o, g.sino_shape, "sinogram")
        if v.device != dev or o.device != dev:
            raise ValueError("all tensors of a batch must be on one device")
    VP = ctypes.c_void_p * n
    hs = VP(*[g.handle.value for g in geoms])
    vp = VP(*[v.data_ptr() for v in vols])
    sp = VP(*[o.data_ptr() for o in outs])
    dt = (ctypes.c_int32 * n)(*[_dtype_code(v) for v in vols])
    with torch.cuda.device(dev):
        check(lib().gjp_forward_project_batched(n, hs, vp, dt, sp, _stream(dev)))
    return list(outs)


def autotune(vol, geom: Geometry, out=None) -> int:
    """Time the forward tile candidates for this geometry and dtype; returns tile_v."""
    torch = _torch()
    if out is not None and out.dtype != torch.float32:
        raise TypeError("sinogram must be float32")
    _dtype_code(vol)
    _check_tensor(vol, geom.shape, "volume")
    if out is None:
        out = torch.empty(geom.sino_shape, dtype=torch.float32, device=vol.device)
    _check_tensor(out, geom.sino_shape, "sinogram")
    if out.device != vol.device:
        raise ValueError("volume and sinogram must be on one device")
    tv = ctypes.c_int32()
    with torch.cuda.device(vol.device):
        check(lib().gjp_autotune_forward(geom.handle, vol.data_ptr(), _dtype_code(vol),
                                         out.data_ptr(), _stream(vol.device), ctypes.byref(tv)))
    return int(tv.value)


def set_forward_tile(geom: Geometry, dtype, tile_v: int, view_group: int = 8,
                     load_group: int = 4) -> None:
    """Fix the forward launch configuration for this geometry's shape signature
    and a torch dtype: tile_v = 192 (three pixels per lane sharing their
    loads), 64, 32 or 16 detector pixels along v per wavefront row (for 16-bit
    storage also 128: two pixels per lane), view_group views per tile turn
    (1..64), load_group planes whose loads a lane issues together (2 or 4);
    tile_v = 0 forgets this process's choice."""
    torch = _torch()
    code = {torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16}[dtype]
    check(lib().gjp_set_forward_tile(geom.handle, code, int(tile_v), int(view_group),
                                     int(load_group)))


def reset_forward_tile(geom: Geometry, dtype) -> None:
    """Forget this process's launch configuration for the geometry's shape
    signature and dtype (the on-disk cache or the default applies again)."""
    torch = _torch()
    code = {torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16}[dtype]
    check(lib().gjp_set_forward_tile(geom.handle, code, 0, 0, 0))


def get_forward_tile(geom: Geometry, dtype):
    """(tile_v, view_group, load_group) that forward calls use now for this
    geometry's shape signature and dtype."""
    torch = _torch()
    code = {torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16}[dtype]
    tv, vg, lg = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(lib().gjp_get_forward_tile(geom.handle, code, ctypes.byref(tv), ctypes.byref(vg),
                                     ctypes.byref(lg)))
    return int(tv.value), int(vg.value), int(lg.value)


def timing_enable(on: bool = True) -> None:
    check(lib().gjp_timing_enable(1 if on else 0))


def timing_reset() -> None:
    check(lib().gjp_timing_reset())


def timing_read(kernel: str):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    check(lib().gjp_timing_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


def _autograd_function():
    torch = _torch()

    class Project(torch.autograd.Function):
        """y = A x with the hand-written adjoint as backward (dL/dx = A^T dL/dy)."""

        @staticmethod
        def forward(ctx, vol, geom):
            ctx.geom = geom
            ctx.vol_dtype = vol.dtype
            return forward(vol.contiguous(), geom)

        @staticmethod
        def backward(ctx, grad_out):
            g = back(grad_out.contiguous().to(torch.float32), ctx.geom)
            if ctx.vol_dtype != torch.float32:
                g = g.to(ctx.vol_dtype)
            return g, None

    return Project


_PROJECT = None


def project(vol, geom: Geometry):
    """Differentiable forward projection (autograd)."""
    global _PROJECT
    if _PROJECT is None:
        _PROJECT = _autograd_function()
    return _PROJECT.apply(vol, geom)


def __getattr__(name):
    if name == "Project":
        global _PROJECT
        if _PROJECT is None:
            _PROJECT = _autograd_function()
        return _PROJECT
    raise AttributeError(name)
