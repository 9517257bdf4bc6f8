"""Pins of the oracle's circular scan trajectories (the per-view geometry step).

The trajectory is fixed by its parameters: the source circles the rotation
axis (third grid axis) at distance sod, the flat detector is perpendicular to
the central ray at distance sdd from the source, du is tangential with length
pitch_u, dv is parallel to the rotation axis with length pitch_v, and the
pixel grid is centred on the central ray. These are checked as geometric
invariants and through projections of known points.
"""
import math

import numpy as np
import pytest


def _centre(v, n_u, n_v):
    return v[3:6] + 0.5 * (n_u - 1) * v[6:9] + 0.5 * (n_v - 1) * v[9:12]


@pytest.mark.parametrize("n_views,n_u,n_v", [(64, 64, 64), (7, 33, 18), (360, 5, 4)])
def test_circular_cone_invariants(oracle_mod, n_views, n_u, n_v):
    sod, sdd, pu, pv = 256.0, 512.0, 2.0, 1.5
    V = oracle_mod.views_circular_cone(n_views, sod, sdd, pu, pv, n_u, n_v)
    assert V.shape == (n_views, 12)
    prev = None
    for k in range(n_views):
        v = V[k]
        src, du, dv = v[0:3], v[6:9], v[9:12]
        c = _centre(v, n_u, n_v)
        assert np.linalg.norm(src) == pytest.approx(sod, rel=1e-14)
        assert src[2] == 0.0
        assert np.linalg.norm(c - src) == pytest.approx(sdd, rel=1e-14)
        # the central ray passes through the rotation axis (origin)
        assert np.linalg.norm(np.cross(c - src, -src)) <= 1e-9 * sod * sdd
        assert np.linalg.norm(du) == pytest.approx(pu, rel=1e-14)
        assert abs(du @ (c - src)) <= 1e-12 * sdd
        assert np.allclose(dv, [0.0, 0.0, pv], rtol=0, atol=0)
        # counter-clockwise steps of 2 pi / n_views about +axis 2
        ang = math.atan2(src[1], src[0]) % (2 * math.pi)
        assert ang == pytest.approx((2 * math.pi * k / n_views) % (2 * math.pi), abs=1e-12)
        if prev is not None:
            assert np.cross(prev, src)[2] > 0
        prev = src


def _project_cone(v, x, n_u, n_v):
    """Continuous pixel coordinates (u, v) where the ray from the source through
    world point x meets the detector plane."""
    src, det00, du, dv = v[0:3], v[3:6], v[6:9], v[9:12]
    M = np.stack([du, dv, -(x - src)], axis=1)
    u, w, t = np.linalg.solve(M, src - det00)
    return u, w


def test_circular_cone_projects_known_points(oracle_mod):
    sod, sdd, n_u, n_v = 1024.0, 1536.0, 384, 384
    V = oracle_mod.views_circular_cone(12, sod, sdd, 1.0, 1.0, n_u, n_v)
    for v in V:
        # the isocentre lands on the detector centre
        u, w = _project_cone(v, np.zeros(3), n_u, n_v)
        assert u == pytest.approx(0.5 * (n_u - 1), abs=1e-9)
        assert w == pytest.approx(0.5 * (n_v - 1), abs=1e-9)
        # a point on the rotation axis is magnified by sdd / sod
        u, w = _project_cone(v, np.array([0.0, 0.0, 40.0]), n_u, n_v)
        assert w == pytest.approx(0.5 * (n_v - 1) + 40.0 * sdd / sod, abs=1e-9)
        assert u == pytest.approx(0.5 * (n_u - 1), abs=1e-9)


def test_first_view_orientation(oracle_mod):
    # view 0: source on +axis 0, detector on the opposite side, du along +axis 1
    V = oracle_mod.views_circular_cone(4, 100.0, 300.0, 1.0, 1.0, 3, 3)
    assert np.allclose(V[0, 0:3], [100.0, 0.0, 0.0])
    assert np.allclose(_centre(V[0], 3, 3), [-200.0, 0.0, 0.0])
    assert np.allclose(V[0, 6:9], [0.0, 1.0, 0.0])
    # view 1 (90 degrees): source on +axis 1
    assert np.allclose(V[1, 0:3], [0.0, 100.0, 0.0], atol=1e-12)


@pytest.mark.parametrize("n_views,n_u,n_v", [(180, 64, 32), (5, 7, 9)])
def test_parallel_invariants(oracle_mod, n_views, n_u, n_v):
    V = oracle_mod.views_parallel(n_views, 1.25, 0.75, n_u, n_v)
    for k in range(n_views):
        v = V[k]
        d, du, dv = v[0:3], v[6:9], v[9:12]
        assert np.linalg.norm(d) == pytest.approx(1.0, rel=1e-14)
        assert d[2] == 0.0
        assert np.allclose(_centre(v, n_u, n_v), 0.0, atol=1e-12)
        assert abs(d @ du) <= 1e-14
        assert np.linalg.norm(du) == pytest.approx(1.25, rel=1e-14)
        assert np.allclose(dv, [0.0, 0.0, 0.75])
        th = 2 * math.pi * k / n_views
        assert np.allclose(d, [-math.cos(th), -math.sin(th), 0.0], atol=1e-15)


def test_invalid_trajectory_parameters(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.views_circular_cone(0, 1.0, 2.0, 1.0, 1.0, 4, 4)
    with pytest.raises(ValueError):
        oracle_mod.views_parallel(3, 1.0, 1.0, 0, 4)
