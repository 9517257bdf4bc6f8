"""Analytic line integrals through uniform ellipsoids (test infrastructure).

The paper's ground truth for projection quality (Sec. IV-A) is the exact
line integral of the ellipsoid phantom. For one ray x(t) = a + t u and an
ellipsoid (centre c, semi-axes s, rotation R, density rho), the local point
A + t B with A = diag(1/s) R^T (a - c), B = diag(1/s) R^T u is inside the unit
sphere for t between the roots of |B|^2 t^2 + 2 (A.B) t + |A|^2 - 1 = 0, so the
integral is rho |u| (t2 - t1). With ``clip`` the chord is additionally
restricted to the grid box [-0.5, N-0.5]^3 (grid coordinates), i.e. the part
of space the rasterised volume represents.
"""
from __future__ import annotations

import numpy as np


def ray_lines(g, rays: np.ndarray, offsets=(0.0, 0.0)):
    """World-space (point, direction) of each ray (view, iu, iv); `offsets`
    shifts the detector point by a fraction of a pixel along u and v."""
    rays = np.asarray(rays, dtype=np.int64).reshape(-1, 3)
    V = g.views[rays[:, 0]]
    iu = rays[:, 1:2].astype(np.float64) + offsets[0]
    iv = rays[:, 2:3].astype(np.float64) + offsets[1]
    d = V[:, 3:6] + iu * V[:, 6:9] + iv * V[:, 9:12]
    if g.beam == 0:
        a = V[:, 0:3]
        u = d - a
    else:
        a = d
        u = V[:, 0:3].copy()
    return a, u


def box_interval(g, a: np.ndarray, u: np.ndarray):
    """Parameter interval [t0, t1] of x = a + t u inside the grid box."""
    shape = np.asarray(g.shape, dtype=np.float64)
    vs = np.asarray(g.voxel_size, dtype=np.float64)
    ctr = np.asarray(g.center, dtype=np.float64)
    lo = ctr - 0.5 * shape * vs
    hi = ctr + 0.5 * shape * vs
    t0 = np.full(a.shape[0], -np.inf)
    t1 = np.full(a.shape[0], np.inf)
    for k in range(3):
        uk = u[:, k]
        nz = uk != 0.0
        ta = np.where(nz, (lo[k] - a[:, k]) / np.where(nz, uk, 1.0), -np.inf)
        tb = np.where(nz, (hi[k] - a[:, k]) / np.where(nz, uk, 1.0), np.inf)
        lo_t = np.minimum(ta, tb)
        hi_t = np.maximum(ta, tb)
        inside = (a[:, k] >= lo[k]) & (a[:, k] <= hi[k])
        lo_t = np.where(nz, lo_t, np.where(inside, -np.inf, np.inf))
        hi_t = np.where(nz, hi_t, np.where(inside, np.inf, -np.inf))
        t0 = np.maximum(t0, lo_t)
        t1 = np.minimum(t1, hi_t)
    return t0, t1


def line_integrals(ellipsoids, g, rays: np.ndarray, clip: bool = True,
                   offsets=(0.0, 0.0)) -> np.ndarray:
    a, u = ray_lines(g, rays, offsets)
    ulen = np.linalg.norm(u, axis=1)
    if clip:
        tb0, tb1 = box_interval(g, a, u)
    out = np.zeros(a.shape[0], dtype=np.float64)
    for e in ellipsoids:
        R = e.rot()
        inv_s = 1.0 / np.asarray(e.semi_axes, dtype=np.float64)
        A = ((a - np.asarray(e.center)) @ R) * inv_s
        B = (u @ R) * inv_s
        qa = np.einsum("ij,ij->i", B, B)
        qb = np.einsum("ij,ij->i", A, B)
        qc = np.einsum("ij,ij->i", A, A) - 1.0
        disc = qb * qb - qa * qc
        hit = disc > 0.0
        sq = np.sqrt(np.where(hit, disc, 0.0))
        t1 = (-qb - sq) / qa
        t2 = (-qb + sq) / qa
        if clip:
            t1 = np.maximum(t1, tb0)
            t2 = np.minimum(t2, tb1)
        seg = np.where(hit, np.maximum(t2 - t1, 0.0), 0.0)
        out += e.density * seg * ulen
    return out


def pixel_integrals(ellipsoids, g, rays: np.ndarray, n_sub: int = 8, clip: bool = True):
    """Mean of the line integrals over n_sub x n_sub regularly spaced points of
    each detector pixel (Sec. IV-A averages 8 x 8 rays per pixel)."""
    offs = [((j + 0.5) / n_sub - 0.5) for j in range(n_sub)]
    acc = np.zeros(np.asarray(rays).reshape(-1, 3).shape[0])
    for ou in offs:
        for ov in offs:
            acc += line_integrals(ellipsoids, g, rays, clip=clip, offsets=(ou, ov))
    return acc / float(n_sub * n_sub)
