"""Seeded random scan geometries and ray subsets.

Views are 12 doubles in world units: cone = (src, det00, du, dv), parallel =
(dir, det00, du, dv), with pixel (iu, iv) centred at det00 + iu du + iv dv.
These generators place sources and detectors at random orientations
(including ones where the third axis is the dominant ray direction) so that
tests exercise every driving axis; they do not compute anything about rays.
"""
from __future__ import annotations

import numpy as np


def _random_frame(rng):
    """Random unit vector w and an orthonormal pair (e1, e2) perpendicular to it."""
    w = rng.normal(size=3)
    w /= np.linalg.norm(w)
    t = rng.normal(size=3)
    e1 = t - w * float(t @ w)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(w, e1)
    return w, e1, e2


def random_cone_views(seed: int, n_views: int, shape, n_u: int, n_v: int,
                      voxel_size=(1.0, 1.0, 1.0), dist_range=(1.2, 3.0), mag_range=(1.1, 2.5),
                      tilt: float = 0.3) -> np.ndarray:
    """Cone-beam views with random source directions around the volume centre.
    The source sits at a random distance (in units of the grid diagonal) and the
    detector, slightly tilted, behind the volume, large enough to cover it."""
    rng = np.random.default_rng(seed)
    ext = np.array([shape[k] * voxel_size[k] for k in range(3)], dtype=np.float64)
    diag = float(np.linalg.norm(ext))
    out = np.zeros((n_views, 12), dtype=np.float64)
    for k in range(n_views):
        w, e1, e2 = _random_frame(rng)
        sod = rng.uniform(*dist_range) * diag
        sdd = sod * rng.uniform(*mag_range)
        src = sod * w
        # tilt the detector axes a little so that pixels are not axis aligned
        t1 = rng.uniform(-tilt, tilt)
        t2 = rng.uniform(-tilt, tilt)
        du = e1 + t1 * w
        dv = e2 + t2 * w
        size = 1.3 * diag * sdd / sod
        du *= size / n_u / np.linalg.norm(du)
        dv *= size / n_v / np.linalg.norm(dv)
        center = src - sdd * w
        det00 = center - 0.5 * (n_u - 1) * du - 0.5 * (n_v - 1) * dv
        out[k] = np.concatenate([src, det00, du, dv])
    return out


def random_parallel_views(seed: int, n_views: int, shape, n_u: int, n_v: int,
                          voxel_size=(1.0, 1.0, 1.0), tilt: float = 0.3) -> np.ndarray:
    """Parallel-beam views with random directions; the detector plane passes
    near the volume centre and covers the grid."""
    rng = np.random.default_rng(seed)
    ext = np.array([shape[k] * voxel_size[k] for k in range(3)], dtype=np.float64)
    diag = float(np.linalg.norm(ext))
    out = np.zeros((n_views, 12), dtype=np.float64)
    for k in range(n_views):
        w, e1, e2 = _random_frame(rng)
        t1 = rng.uniform(-tilt, tilt)
        t2 = rng.uniform(-tilt, tilt)
        du = e1 + t1 * w
        dv = e2 + t2 * w
        size = 1.2 * diag
        du *= size / n_u / np.linalg.norm(du)
        dv *= size / n_v / np.linalg.norm(dv)
        offset = rng.uniform(-0.05, 0.05, size=3) * ext
        det00 = offset - 0.5 * (n_u - 1) * du - 0.5 * (n_v - 1) * dv
        out[k] = np.concatenate([-w, det00, du, dv])
    return out


def sample_rays(seed: int, n_rays: int, n_views: int, n_u: int, n_v: int) -> np.ndarray:
    """n_rays distinct (view, iu, iv) triples drawn uniformly, as int32 (n_rays, 3)."""
    rng = np.random.default_rng(seed)
    total = n_views * n_u * n_v
    n = min(n_rays, total)
    flat = rng.choice(total, size=n, replace=False)
    flat.sort()
    view = flat // (n_u * n_v)
    rem = flat % (n_u * n_v)
    return np.stack([view, rem // n_v, rem % n_v], axis=1).astype(np.int32)
