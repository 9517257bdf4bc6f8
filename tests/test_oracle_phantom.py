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


# ---------------------------------------------------------------------------
# Sub-pixel rays (Sec. IV-A averages the analytic line integrals over 8 x 8
# rays per detector pixel): `offsets` are fractions of a pixel along u and v,
# and pixel_integrals takes the mean over n_sub x n_sub points centred in
# equal sub-squares of the pixel.
# ---------------------------------------------------------------------------
def _parallel_pixel_geom(oracle_mod, shape, y0, z0, pu, pv):
    """One parallel-beam pixel (n_u = n_v = 1) with rays along +x through the
    world point (0, y0, z0); pixel pitch pu along y and pv along z (world)."""
    views = np.zeros((1, 12))
    views[0, 0:3] = (1.0, 0.0, 0.0)
    views[0, 3:6] = (0.0, y0, z0)
    views[0, 6:9] = (0.0, pu, 0.0)
    views[0, 9:12] = (0.0, 0.0, pv)
    return oracle_mod.Geometry(shape, views, 1, 1, beam=oracle_mod.PARALLEL)


def _sphere_chord(R, rho, b2):
    return 2.0 * rho * math.sqrt(R * R - b2) if b2 < R * R else 0.0


def test_line_integral_offsets_are_pixel_fractions(oracle_mod):
    """Parallel beam through a sphere: the offset ray's impact parameter moves
    by offset x pitch (world units), checked against the chord by hand."""
    from oracle import phantom
    R, rho = 10.0, 1.5
    e = [Ellipsoid((0.0, 0.0, 0.0), (R, R, R), IDENT, rho)]
    g = _parallel_pixel_geom(oracle_mod, (64, 64, 64), 1.0, -2.0, 2.0, 1.5)
    for ou, ov in ((0.0, 0.0), (0.25, 0.0), (0.0, -0.375), (-0.4375, 0.3125)):
        y, z = 1.0 + 2.0 * ou, -2.0 + 1.5 * ov
        want = _sphere_chord(R, rho, y * y + z * z)
        got = phantom.line_integrals(e, g, np.array([[0, 0, 0]]), offsets=(ou, ov))[0]
        assert got == pytest.approx(want, rel=1e-12)


def test_line_integral_offsets_cone_equal_shifted_detector(oracle_mod):
    """Cone beam: an offset ray equals the centre ray of a detector whose first
    pixel is moved by the same fraction of du and dv (the source stays)."""
    from oracle import phantom
    shape = (40, 40, 40)
    e = workloads.random_ellipsoids(7, shape, n=6)
    views = oracle_mod.views_circular_cone(5, 160.0, 240.0, 1.7, 1.3, 30, 26)
    g = oracle_mod.Geometry(shape, views, 30, 26, beam=oracle_mod.CONE)
    rays = workloads.sample_rays(8, 60, 5, 30, 26)
    ou, ov = 0.3125, -0.1875
    shifted = views.copy()
    shifted[:, 3:6] += ou * views[:, 6:9] + ov * views[:, 9:12]
    gs = oracle_mod.Geometry(shape, shifted, 30, 26, beam=oracle_mod.CONE)
    got = phantom.line_integrals(e, g, rays, offsets=(ou, ov))
    want = phantom.line_integrals(e, gs, rays)
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-10)
    assert np.abs(got - phantom.line_integrals(e, g, rays)).max() > 1e-3


def test_pixel_integrals_one_subray_is_centre_ray(oracle_mod):
    from oracle import phantom
    shape = (32, 36, 28)
    e = workloads.random_ellipsoids(9, shape, n=5)
    views = oracle_mod.views_circular_cone(4, 120.0, 200.0, 1.5, 1.5, 20, 18)
    g = oracle_mod.Geometry(shape, views, 20, 18, beam=oracle_mod.CONE)
    rays = workloads.sample_rays(10, 50, 4, 20, 18)
    np.testing.assert_array_equal(phantom.pixel_integrals(e, g, rays, n_sub=1),
                                  phantom.line_integrals(e, g, rays))


def test_pixel_integrals_uniform_slab(oracle_mod):
    """A constant region covering the grid box and rays normal to its x faces:
    every sub-ray's clipped chord is the box length, so the mean is too."""
    from oracle import phantom
    shape = (20, 30, 40)
    big = [Ellipsoid((0.0, 0.0, 0.0), (500.0, 500.0, 500.0), IDENT, 0.75)]
    g = _parallel_pixel_geom(oracle_mod, shape, 3.0, -4.0, 2.0, 2.0)
    val = phantom.pixel_integrals(big, g, np.array([[0, 0, 0]]), n_sub=8)[0]
    assert val == pytest.approx(0.75 * 20.0, rel=1e-13)


def test_pixel_integrals_sphere_footprint(oracle_mod):
    """Sphere, parallel rays along x, pixel of pitch 2 x 1.5 centred at
    (y0, z0): the 8 x 8 mean equals the mean of the chords at the 64 sub-square
    centres worked out by hand, and with more sub-rays the mean converges
    (second order) to the chord averaged over the pixel's area."""
    from scipy import integrate
    from oracle import phantom
    R, rho = 10.0, 1.0
    y0, z0, pu, pv = 4.0, 3.0, 2.0, 1.5
    e = [Ellipsoid((0.0, 0.0, 0.0), (R, R, R), IDENT, rho)]
    g = _parallel_pixel_geom(oracle_mod, (64, 64, 64), y0, z0, pu, pv)
    ray = np.array([[0, 0, 0]])
    n = 8
    want = 0.0
    for j in range(n):
        for k in range(n):
            y = y0 + pu * ((j + 0.5) / n - 0.5)
            z = z0 + pv * ((k + 0.5) / n - 0.5)
            want += _sphere_chord(R, rho, y * y + z * z)
    want /= n * n
    assert phantom.pixel_integrals(e, g, ray, n_sub=n)[0] == pytest.approx(want, rel=1e-12)
    area, _ = integrate.dblquad(lambda z, y: _sphere_chord(R, rho, y * y + z * z),
                                y0 - 0.5 * pu, y0 + 0.5 * pu, z0 - 0.5 * pv, z0 + 0.5 * pv,
                                epsabs=1e-12, epsrel=1e-12)
    area /= pu * pv
    errs = [abs(phantom.pixel_integrals(e, g, ray, n_sub=m)[0] - area) for m in (2, 4, 8, 16)]
    for a, b in zip(errs, errs[1:]):
        assert b < 0.3 * a
    assert errs[2] < 1e-3 * area
