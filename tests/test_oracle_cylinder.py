"""Pins of the oracle's cylinder clipping of the sample range (Sec. IV-C: the
first sample and the number of samples follow the ray-cylinder intersection).

The reading: a sample also needs its axis-0/axis-1 position strictly inside
the circle of radius min(N0, N1)/2 about ((N0-1)/2, (N1-1)/2), the cylinder
inscribed in the grid box with its axis along the rotation axis (axis 2).

Pins:
* axis-aligned parallel rays through integer grid points: the sample count is
  the number of lattice points strictly inside the chord, computed here with
  exact integer arithmetic (including points exactly on the circle, which are
  excluded), and the projection of a volume of ones equals that count;
* a volume supported well inside the cylinder projects and back-projects
  identically with and without clipping (bitwise);
* clipping only removes samples, and the counts of a square grid are the same
  for views 90 degrees apart.
"""
import numpy as np
import pytest

import oracle


def _axis_views(n_views, n_u, n_v):
    return oracle.views_parallel(n_views, 1.0, 1.0, n_u, n_v)


def _lattice_count(n0, n1, iu):
    # #{i in [0, n0): (i - (n0-1)/2)^2 + (iu - (n1-1)/2)^2 < (min(n0, n1)/2)^2}, times 4
    m = min(n0, n1)
    b = 2 * iu - (n1 - 1)
    return sum(1 for i in range(n0) if (2 * i - (n0 - 1)) ** 2 + b * b < m * m)


@pytest.mark.parametrize("shape", [(6, 5, 3), (9, 9, 2), (12, 7, 4), (5, 8, 3)])
def test_axis_aligned_chord_counts(shape):
    n0, n1, n2 = shape
    # view 0 of a parallel trajectory: rays along -x through (y, z) = (iu, iv)
    views = _axis_views(4, n1, n2)[:1]
    g = oracle.Geometry(shape, views, n1, n2, beam=oracle.PARALLEL, clip_cylinder=True)
    rays = np.array([(0, iu, iv) for iu in range(n1) for iv in range(n2)], dtype=np.int32)
    ones = np.ones(shape)
    val, cnt = oracle.forward_rays(g, ones, rays, with_counts=True)
    want = np.array([_lattice_count(n0, n1, iu) for iu in range(n1) for iv in range(n2)])
    np.testing.assert_array_equal(cnt, want)
    np.testing.assert_array_equal(val, want.astype(np.float64))
    # the (6, 5) grid has lattice points exactly on the circle; they are excluded
    if shape[:2] == (6, 5):
        assert _lattice_count(6, 5, 0) == 2  # i = 2, 3 only (i = 1, 4 lie on the circle)


def _circular_cone(shape, n_views, n_u, n_v, seed):
    rng = np.random.default_rng(seed)
    sod = 3.0 * max(shape)
    views = oracle.views_circular_cone(n_views, sod, 1.7 * sod, 1.3, 1.1, n_u, n_v)
    # a small random tilt keeps every driving axis and ray orientation generic
    return views + rng.normal(scale=1e-3, size=views.shape)


@pytest.mark.parametrize("beam", ["cone", "parallel"])
def test_support_inside_cylinder_is_unchanged(beam):
    shape = (14, 12, 9)
    n0, n1, n2 = shape
    rng = np.random.default_rng(7)
    vol = rng.uniform(-1.0, 1.0, size=shape)
    x = np.arange(n0)[:, None] - 0.5 * (n0 - 1)
    y = np.arange(n1)[None, :] - 0.5 * (n1 - 1)
    rad = 0.5 * min(n0, n1)
    vol[(x * x + y * y) >= (rad - 1.5) ** 2] = 0.0  # support within r - 1.5
    if beam == "cone":
        views, b = _circular_cone(shape, 7, 18, 13, 3), oracle.CONE
    else:
        views, b = oracle.views_parallel(7, 1.0, 1.0, 18, 13), oracle.PARALLEL
    g0 = oracle.Geometry(shape, views, 18, 13, beam=b)
    g1 = oracle.Geometry(shape, views, 18, 13, beam=b, clip_cylinder=True)
    y0, y1 = oracle.forward(g0, vol), oracle.forward(g1, vol)
    np.testing.assert_array_equal(y0, y1)
    assert oracle.count_samples(g1) < oracle.count_samples(g0)
    # back-projection agrees on the support (every sample that reaches it is kept)
    s = rng.uniform(-1.0, 1.0, size=y0.shape)
    a0, a1 = oracle.adjoint(g0, s), oracle.adjoint(g1, s)
    inside = np.broadcast_to(((x * x + y * y) < (rad - 1.5) ** 2)[:, :, None], shape)
    np.testing.assert_array_equal(a0[inside], a1[inside])


def test_clipping_removes_samples_and_respects_symmetry():
    shape = (16, 16, 6)
    views = oracle.views_parallel(4, 1.0, 1.0, 16, 6)  # 0, 90, 180, 270 degrees
    g0 = oracle.Geometry(shape, views, 16, 6, beam=oracle.PARALLEL)
    g1 = oracle.Geometry(shape, views, 16, 6, beam=oracle.PARALLEL, clip_cylinder=True)
    rays = np.array([(v, iu, iv) for v in range(4) for iu in range(16) for iv in range(6)],
                    dtype=np.int32)
    ones = np.ones(shape)
    _, c0 = oracle.forward_rays(g0, ones, rays, with_counts=True)
    _, c1 = oracle.forward_rays(g1, ones, rays, with_counts=True)
    assert np.all(c1 <= c0) and c1.sum() < c0.sum()
    per_view = c1.reshape(4, -1).sum(axis=1)
    assert np.all(per_view == per_view[0])
    # a ray through the axis keeps the full diameter: 16 samples
    assert c1.reshape(4, 16, 6)[0, 8, 0] == 16
