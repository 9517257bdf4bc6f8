"""Ellipsoid phantoms: parameter sets and point-sampled rasterisation.

An ellipsoid is (centre c, semi-axes a, rotation R, density rho) in world
units; a world point x is inside when || diag(1/a) R^T (x - c) ||^2 <= 1.
Densities of overlapping ellipsoids add. Rasterisation samples each voxel
at its centre; voxel (i0, i1, i2) of an N0 x N1 x N2 grid with voxel size
h and centre c_vol sits at world position (i_k - (N_k - 1)/2) h_k + c_vol_k.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np


@dataclasses.dataclass(frozen=True)
class Ellipsoid:
    center: tuple      # world units
    semi_axes: tuple   # world units
    rotation: tuple    # 3x3 row-major; columns are the ellipsoid's axes in world coords
    density: float

    def rot(self) -> np.ndarray:
        return np.asarray(self.rotation, dtype=np.float64).reshape(3, 3)


def _rot_z(deg: float) -> tuple:
    t = math.radians(deg)
    c, s = math.cos(t), math.sin(t)
    return (c, -s, 0.0, s, c, 0.0, 0.0, 0.0, 1.0)


# Nested head-like stand-in, in units of the half edge of the grid
# (centre x, y, z, semi-axes x, y, z, rotation about axis 2 in degrees, density).
_SL_STAND_IN = [
    (0.00, 0.00, 0.00, 0.72, 0.92, 0.88, 0.0, 1.00),
    (0.00, -0.015, 0.00, 0.67, 0.87, 0.83, 0.0, -0.78),
    (0.20, 0.05, 0.00, 0.10, 0.30, 0.22, 15.0, -0.18),
    (-0.24, 0.02, 0.05, 0.14, 0.38, 0.26, -20.0, -0.16),
    (0.00, 0.33, 0.10, 0.20, 0.24, 0.20, 0.0, 0.09),
    (0.00, 0.08, -0.05, 0.05, 0.05, 0.05, 0.0, 0.12),
    (0.00, -0.12, 0.03, 0.045, 0.045, 0.06, 0.0, 0.11),
    (-0.07, -0.58, -0.12, 0.045, 0.025, 0.05, 30.0, 0.08),
    (0.05, -0.60, -0.10, 0.025, 0.03, 0.03, 0.0, 0.07),
    (0.05, 0.62, 0.35, 0.06, 0.04, 0.08, 40.0, 0.13),
]


def sl_stand_in(shape: Sequence[int], voxel_size=(1.0, 1.0, 1.0)) -> List[Ellipsoid]:
    """The 10-ellipsoid nested stand-in phantom scaled to a grid of `shape`."""
    half = [0.5 * shape[k] * voxel_size[k] for k in range(3)]
    out = []
    for cx, cy, cz, ax, ay, az, deg, rho in _SL_STAND_IN:
        out.append(Ellipsoid(
            center=(cx * half[0], cy * half[1], cz * half[2]),
            semi_axes=(ax * half[0], ay * half[1], az * half[2]),
            rotation=_rot_z(deg),
            density=rho,
        ))
    return out


def random_ellipsoids(seed: int, shape: Sequence[int], n: int = 12,
                      voxel_size=(1.0, 1.0, 1.0)) -> List[Ellipsoid]:
    """Seeded random ellipsoids: centres uniform in the inner 80% of each edge,
    semi-axes uniform in [5%, 40%] of the smallest edge, rotations uniform on
    SO(3) (normalised Gaussian quaternion), densities uniform in [-0.5, 1.0]."""
    rng = np.random.default_rng(seed)
    edges = np.array([shape[k] * voxel_size[k] for k in range(3)], dtype=np.float64)
    small = float(edges.min())
    out = []
    for _ in range(n):
        c = rng.uniform(-0.4, 0.4, size=3) * edges
        a = rng.uniform(0.05, 0.40, size=3) * small
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        w, x, y, z = q
        R = np.array([
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
        ])
        rho = float(rng.uniform(-0.5, 1.0))
        out.append(Ellipsoid(tuple(c.tolist()), tuple(a.tolist()),
                             tuple(R.reshape(-1).tolist()), rho))
    return out


def _axis_coords(shape, voxel_size, center):
    return [((np.arange(shape[k], dtype=np.float64) - 0.5 * (shape[k] - 1)) * voxel_size[k]
             + center[k]) for k in range(3)]


def rasterize(ellipsoids: Sequence[Ellipsoid], shape: Sequence[int],
              voxel_size=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0),
              dtype=np.float32, supersample: int = 1) -> np.ndarray:
    """Point-sample the phantom at voxel centres (FP64 inside test), C order.
    With supersample = k each voxel is the mean over k^3 regularly spaced
    points at offsets ((j + 0.5) / k - 0.5) voxel per axis (Sec. IV-A uses
    k = 5)."""
    shape = tuple(int(s) for s in shape)
    k = int(supersample)
    offs = [((j + 0.5) / k - 0.5) for j in range(k)]
    vol = np.zeros(shape, dtype=np.float64)
    for o0 in offs:
        for o1 in offs:
            for o2 in offs:
                xs, ys, zs = _axis_coords(shape, voxel_size, center)
                xs = xs + o0 * voxel_size[0]
                ys = ys + o1 * voxel_size[1]
                zs = zs + o2 * voxel_size[2]
                Y, Z = np.meshgrid(ys, zs, indexing="ij")
                for e in ellipsoids:
                    R = e.rot()
                    inv_a = 1.0 / np.asarray(e.semi_axes, dtype=np.float64)
                    cx, cy, cz = e.center
                    for i0, x in enumerate(xs):
                        dx, dy, dz = x - cx, Y - cy, Z - cz
                        q = np.zeros_like(Y)
                        for j in range(3):
                            loc = R[0, j] * dx + R[1, j] * dy + R[2, j] * dz
                            q += (loc * inv_a[j]) ** 2
                        vol[i0] += np.where(q <= 1.0, e.density, 0.0)
    return (vol / float(k ** 3)).astype(dtype)


def rasterize_torch(ellipsoids: Sequence[Ellipsoid], shape: Sequence[int], device,
                    voxel_size=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0), dtype=None,
                    supersample: int = 1):
    """Same point sampling as `rasterize` (including `supersample`), evaluated
    with torch in FP64 one x-slab at a time (for grids too large for numpy on
    the host)."""
    import torch
    dtype = dtype or torch.float32
    shape = tuple(int(s) for s in shape)
    k = int(supersample)
    offs = torch.tensor([((j + 0.5) / k - 0.5) for j in range(k)], dtype=torch.float64,
                        device=device)
    base = [torch.as_tensor(a, dtype=torch.float64, device=device)
            for a in _axis_coords(shape, voxel_size, center)]
    # sub-sample coordinates of one slab: (k, n1, 1) along y and (k, 1, n2) along z,
    # combined by broadcasting into (k, k, n1, n2)
    ys = (base[1][None, :] + offs[:, None] * voxel_size[1])[:, None, :, None]
    zs = (base[2][None, :] + offs[:, None] * voxel_size[2])[None, :, None, :]
    vol = torch.empty(shape, dtype=dtype, device=device)
    ells = [(torch.as_tensor(e.rot(), dtype=torch.float64, device=device),
             [1.0 / a for a in e.semi_axes], e.center, e.density) for e in ellipsoids]
    for i0 in range(shape[0]):
        acc = torch.zeros((shape[1], shape[2]), dtype=torch.float64, device=device)
        for o0 in range(k):
            x = base[0][i0] + offs[o0] * voxel_size[0]
            for R, inv_a, (cx, cy, cz), rho in ells:
                dx, dy, dz = x - cx, ys - cy, zs - cz
                q = None
                for j in range(3):
                    loc = R[0, j] * dx + R[1, j] * dy + R[2, j] * dz
                    t = (loc * inv_a[j]) ** 2
                    q = t if q is None else q + t
                acc += torch.where(q <= 1.0, rho, 0.0).sum(dim=(0, 1))
        vol[i0] = (acc / float(k ** 3)).to(dtype)
    return vol
