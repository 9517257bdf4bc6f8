"""FP64 CPU oracle of the branchless generalized Joseph projector.

TEST INFRASTRUCTURE ONLY. The test suite, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package; the GPU library and
its Python binding never do. The oracle shares no code with the GPU path: the
projector itself is plain C in double precision (``gjp_oracle.c``, built by
``oracle/build.py`` with gcc), written from Sec. III of the paper (Eqs. 1-14,
Algorithm 1); ``oracle.phantom`` holds the analytic ellipsoid line integrals
(Sec. IV-A) used as closed-form references.

Every function here is pinned by a test in ``tests/test_oracle_*.py`` against
something other than itself (closed forms, invariants, library routines,
brute force); see the pin list in each test module.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np

from . import build as _build

_LIB = None

CONE, PARALLEL = 0, 1
W_LINEAR, W_SPLINE = 0, 1
CLIP_CYLINDER = 1

_i32p = ctypes.POINTER(ctypes.c_int)
_f64p = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_longlong)


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        geo = [_i32p, _f64p, _f64p, ctypes.c_int, ctypes.c_int, _f64p, ctypes.c_int, ctypes.c_int,
               ctypes.c_int]
        L.gjo_views_circular_cone.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                              ctypes.c_int, _f64p]
        L.gjo_views_parallel.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int, _f64p]
        L.gjo_forward.argtypes = geo + [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, _f64p]
        L.gjo_forward_rays.argtypes = geo + [ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                             ctypes.c_longlong, _i32p, _f64p, _i64p]
        L.gjo_adjoint.argtypes = geo + [ctypes.c_int, _f64p, _f64p]
        L.gjo_count_samples.argtypes = geo
        L.gjo_count_samples.restype = ctypes.c_longlong
        L.gjo_ray_info.argtypes = geo + [ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p, _f64p,
                                         _f64p]
        L.gjo_num_threads.restype = ctypes.c_int
        L.gjo_set_num_threads.argtypes = [ctypes.c_int]
        _LIB = L
    return _LIB


def _p(a, t):
    return a.ctypes.data_as(t)


def num_threads() -> int:
    return int(lib().gjo_num_threads())


def set_num_threads(n: int) -> None:
    lib().gjo_set_num_threads(int(n))


def views_circular_cone(n_views, sod, sdd, pitch_u, pitch_v, n_u, n_v) -> np.ndarray:
    out = np.zeros((n_views, 12), dtype=np.float64)
    rc = lib().gjo_views_circular_cone(int(n_views), float(sod), float(sdd), float(pitch_u),
                                       float(pitch_v), int(n_u), int(n_v), _p(out, _f64p))
    if rc != 0:
        raise ValueError("invalid circular cone parameters")
    return out


def views_parallel(n_views, pitch_u, pitch_v, n_u, n_v) -> np.ndarray:
    out = np.zeros((n_views, 12), dtype=np.float64)
    rc = lib().gjo_views_parallel(int(n_views), float(pitch_u), float(pitch_v), int(n_u),
                                  int(n_v), _p(out, _f64p))
    if rc != 0:
        raise ValueError("invalid parallel parameters")
    return out


@dataclasses.dataclass
class Geometry:
    shape: tuple
    views: np.ndarray            # (n_views, 12) world units
    n_u: int
    n_v: int
    beam: int = CONE
    voxel_size: tuple = (1.0, 1.0, 1.0)
    center: tuple = (0.0, 0.0, 0.0)
    weight: int = W_LINEAR
    clip_cylinder: bool = False  # Sec. IV-C sample range clipping

    def __post_init__(self):
        self.views = np.ascontiguousarray(self.views, dtype=np.float64).reshape(-1, 12)
        self._shape = np.asarray(self.shape, dtype=np.int32)
        self._vs = np.asarray(self.voxel_size, dtype=np.float64)
        self._ctr = np.asarray(self.center, dtype=np.float64)

    @property
    def n_views(self) -> int:
        return int(self.views.shape[0])

    def _args(self):
        return (_p(self._shape, _i32p), _p(self._vs, _f64p), _p(self._ctr, _f64p),
                int(self.beam), self.n_views, _p(self.views, _f64p), int(self.n_u),
                int(self.n_v), CLIP_CYLINDER if self.clip_cylinder else 0)


def _vol_arg(vol):
    if vol.dtype == np.float64:
        return np.ascontiguousarray(vol), 0
    if vol.dtype == np.float32:
        return np.ascontiguousarray(vol), 1
    return np.ascontiguousarray(vol, dtype=np.float64), 0


def forward(g: Geometry, vol: np.ndarray) -> np.ndarray:
    """A x over the whole sinogram, (n_views, n_u, n_v) float64."""
    v, dt = _vol_arg(vol)
    assert v.shape == tuple(g.shape)
    out = np.zeros((g.n_views, g.n_u, g.n_v), dtype=np.float64)
    rc = lib().gjo_forward(*g._args(), int(g.weight), v.ctypes.data_as(ctypes.c_void_p), dt,
                           _p(out, _f64p))
    if rc != 0:
        raise ValueError("oracle forward: invalid arguments")
    return out


def forward_rays(g: Geometry, vol: np.ndarray, rays: np.ndarray, with_counts: bool = False):
    """A x at a list of rays (n, 3) = (view, iu, iv)."""
    v, dt = _vol_arg(vol)
    assert v.shape == tuple(g.shape)
    rays = np.ascontiguousarray(rays, dtype=np.int32).reshape(-1, 3)
    out = np.zeros(rays.shape[0], dtype=np.float64)
    cnt = np.zeros(rays.shape[0], dtype=np.int64)
    rc = lib().gjo_forward_rays(*g._args(), int(g.weight), v.ctypes.data_as(ctypes.c_void_p),
                                dt, int(rays.shape[0]), _p(rays, _i32p), _p(out, _f64p),
                                _p(cnt, _i64p))
    if rc != 0:
        raise ValueError("oracle forward_rays: invalid arguments")
    return (out, cnt) if with_counts else out


def adjoint(g: Geometry, sino: np.ndarray) -> np.ndarray:
    """A^T y, (n0, n1, n2) float64."""
    s = np.ascontiguousarray(sino, dtype=np.float64)
    assert s.shape == (g.n_views, g.n_u, g.n_v)
    out = np.zeros(tuple(g.shape), dtype=np.float64)
    rc = lib().gjo_adjoint(*g._args(), int(g.weight), _p(s, _f64p), _p(out, _f64p))
    if rc != 0:
        raise ValueError("oracle adjoint: invalid arguments or out of memory")
    return out


def count_samples(g: Geometry) -> int:
    n = int(lib().gjo_count_samples(*g._args()))
    if n < 0:
        raise ValueError("oracle count: invalid arguments")
    return n


def ray_info(g: Geometry, view: int, iu: int, iv: int):
    """(driving axis m or -1, step length, r~) for one ray."""
    m = np.zeros(1, dtype=np.int32)
    ln = np.zeros(1, dtype=np.float64)
    rt = np.zeros(3, dtype=np.float64)
    lib().gjo_ray_info(*g._args(), int(view), int(iu), int(iv), _p(m, _i32p), _p(ln, _f64p),
                       _p(rt, _f64p))
    return int(m[0]), float(ln[0]), rt


def geometry_for(cfg, weight: int = W_LINEAR) -> Geometry:
    """Oracle geometry for a workload configuration (circular trajectory;
    cylinder clipping when the configuration asks for it)."""
    if cfg.beam == "cone":
        views = views_circular_cone(cfg.n_views, cfg.sod, cfg.sdd, cfg.pitch_u, cfg.pitch_v,
                                    cfg.n_u, cfg.n_v)
        beam = CONE
    else:
        views = views_parallel(cfg.n_views, cfg.pitch_u, cfg.pitch_v, cfg.n_u, cfg.n_v)
        beam = PARALLEL
    return Geometry(tuple(cfg.shape), views, cfg.n_u, cfg.n_v, beam=beam, weight=weight,
                    clip_cylinder=bool(getattr(cfg, "clip_cylinder", False)))
