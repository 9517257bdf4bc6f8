"""Pins of the analytic ellipsoid line integrals and the point-sampled rasteriser."""
import math

import numpy as np
import pytest

import workloads
from workloads.phantoms import Ellipsoid

from conftest import parallel_rays_views

IDENT = (1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0)


def _geom(oracle_mod, shape, point_grid, direction):
    views = parallel_rays_views(shape, direction, point_grid, (0, 1.0, 0), (0, 0, 1.0))
    return oracle_mod.Geometry(shape, views, 1, 1, beam=oracle_mod.PARALLEL)


def test_sphere_chords(oracle_mod):
    from oracle import phantom
    shape = (64, 64, 64)
    R = 10.0
    e = [Ellipsoid((0.0, 0.0, 0.0), (R, R, R), IDENT, 2.0)]
    c = 31.5
    for b in (0.0, 3.0, 7.5, 9.99):
        g = _geom(oracle_mod, shape, (0.0, c + b, c), (1.0, 0.0, 0.0))
        val = phantom.line_integrals(e, g, np.array([[0, 0, 0]]))[0]
        assert val == pytest.approx(2.0 * 2 * math.sqrt(R * R - b * b), rel=1e-12)
    g = _geom(oracle_mod, shape, (0.0, c + 11.0, c), (1.0, 0.0, 0.0))
    assert phantom.line_integrals(e, g, np.array([[0, 0, 0]]))[0] == 0.0


def test_rotated_ellipsoid_chord(oracle_mod):
    from oracle import phantom
    shape = (64, 64, 64)
    t = math.radians(30.0)
    R = (math.cos(t), -math.sin(t), 0.0, math.sin(t), math.cos(t), 0.0, 0.0, 0.0, 1.0)
    e = [Ellipsoid((1.0, -2.0, 3.0), (12.0, 4.0, 6.0), R, 1.0)]
    # a ray through the centre along the ellipsoid's first axis has chord 2*12
    d = np.array([math.cos(t), math.sin(t), 0.0])
    p = np.array([1.0, -2.0, 3.0]) + 31.5 - 20.0 * d
    g = _geom(oracle_mod, shape, p, d)
    val = phantom.line_integrals(e, g, np.array([[0, 0, 0]]))[0]
    assert val == pytest.approx(24.0, rel=1e-12)


def test_box_clipping(oracle_mod):
    from oracle import phantom
    shape = (20, 30, 40)
    big = [Ellipsoid((0.0, 0.0, 0.0), (100.0, 100.0, 100.0), IDENT, 1.0)]
    g = _geom(oracle_mod, shape, (0.0, 14.5, 19.5), (1.0, 0.0, 0.0))
    assert phantom.line_integrals(big, g, np.array([[0, 0, 0]]), clip=True)[0] == \
        pytest.approx(20.0, rel=1e-13)
    assert phantom.line_integrals(big, g, np.array([[0, 0, 0]]), clip=False)[0] == \
        pytest.approx(200.0, rel=1e-13)
    d = np.array([1.0, 0.5, 0.25])
    g = _geom(oracle_mod, shape, (9.5, 14.5, 19.5), d)
    # through the centre: the x-faces at -0.5 and 19.5 bound the chord
    assert phantom.line_integrals(big, g, np.array([[0, 0, 0]]), clip=True)[0] == \
        pytest.approx(20.0 * np.linalg.norm(d), rel=1e-13)


def test_rasterise_sphere_volume_and_overlap():
    shape = (48, 48, 48)
    R = 15.0
    e = [Ellipsoid((0.0, 0.0, 0.0), (R, R, R), IDENT, 1.0),
         Ellipsoid((0.0, 0.0, 0.0), (5.0, 5.0, 5.0), IDENT, 0.5)]
    vol = workloads.rasterize(e, shape)
    assert vol.dtype == np.float32
    # point sampling at voxel centres: the inside count is the number of
    # half-integer lattice points in the ball (brute force), close to its volume
    c = np.arange(48) - 23.5
    brute = sum(1 for x in c for y in c for z in c if x * x + y * y + z * z <= R * R)
    assert (vol > 0).sum() == brute
    assert brute == pytest.approx(4.0 / 3.0 * math.pi * R ** 3, rel=0.03)
    # densities add where ellipsoids overlap
    assert vol.max() == pytest.approx(1.5)
    # grid centre (23.5) is between voxels 23 and 24: both central voxels inside
    assert vol[23, 23, 23] == vol[24, 24, 24] == pytest.approx(1.5)
    assert vol[0, 0, 0] == 0.0


def test_random_ellipsoid_recipe():
    shape = (100, 120, 80)
    e = workloads.random_ellipsoids(2, shape, n=12)
    assert len(e) == 12
    for x in e:
        R = x.rot()
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-12)
        assert np.linalg.det(R) == pytest.approx(1.0)
        for k in range(3):
            assert abs(x.center[k]) <= 0.4 * shape[k]
            assert 0.05 * 80 <= x.semi_axes[k] <= 0.40 * 80
        assert -0.5 <= x.density <= 1.0
    # seeded: same seed, same draw
    assert workloads.random_ellipsoids(2, shape) == e
