"""Projection quality against analytic line integrals (Sec. IV-A, Fig. 2).

The paper compares projectors by the normalised l1 residual between the
projection of a 5^3-supersampled raster of a Shepp-Logan phantom and the
analytic projections averaged over 8 x 8 rays per detector pixel, with a 10
degree cone and about (pi/2) N views. Here: the Shepp-Logan-type stand-in
phantom (the published table is not reconstructed), the same raster and
detector averaging, residuals accumulated over a seeded sample of rays from all
views (the analytic reference of every ray of every view would dominate the
run time). The figure's values are not printed in the paper, so nothing
numeric is matched: the tests check that the residuals shrink at least at
first order when the voxel size halves, bound them near the measured values,
and at the paper's scale check its qualitative finding (linear below spline). At 48^3 the
order is reversed on this phantom: the finding is a property of fine grids.
"""
import numpy as np
import pytest

import workloads
from gpu_helpers import cuda, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gjp():
    import paper_1609_00958_amd as m
    return m


def _quality(gjp, oracle_mod, n, n_views, n_rays):
    import torch
    from oracle import phantom
    dev = cuda()
    sod = 0.5 * n / np.tan(np.radians(5.0))  # detector half-width subtends 5 degrees
    cfg = workloads.WorkloadConfig("q", (n, n, n), n_views, n, n, beam="cone", sod=sod,
                                   sdd=2.0 * sod, pitch_u=2.0, pitch_v=2.0, phantom="sl")
    ells = cfg.phantom_ellipsoids()
    note(f"quality {n}^3: rasterise (5^3 supersampling)")
    vol = workloads.rasterize_torch(ells, cfg.shape, dev, supersample=5)
    rays = workloads.sample_rays(99, n_rays, n_views, n, n)
    idx = torch.from_numpy(rays.astype(np.int64))
    og = oracle_mod.geometry_for(cfg)
    note(f"quality {n}^3: analytic reference, 8 x 8 rays per pixel")
    ref = phantom.pixel_integrals(ells, og, rays, n_sub=8)
    out = {}
    for w in ("linear", "spline"):
        G = gjp.Geometry.from_config(cfg, weight=w)
        y = gjp.forward(vol, G)
        got = y[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
        out[w] = float(np.abs(got - ref).sum() / np.abs(ref).sum())
    note(f"quality {n}^3, {n_views} views: normalised l1 linear {out['linear']:.5f}, "
         f"spline {out['spline']:.5f}")
    return out


def test_quality_128(gjp, oracle_mod):
    r = _quality(gjp, oracle_mod, 128, 201, 6000)
    # regression bounds about 40% above the measured 0.0073 (linear) and
    # 0.0089 (spline)
    assert 0.0 < r["linear"] < 0.010 and 0.0 < r["spline"] < 0.0125


def test_quality_converges(gjp, oracle_mod):
    """Halving the voxel size (64^3 -> 128^3, the same scaled geometry, about
    (pi/2) N views) shrinks the residual against the analytic projections at
    least as fast as first order (ratio <= 0.7, 0.5 expected): a wrong grid
    or detector convention, a half-voxel shift or a scaling error would leave
    a residual that does not shrink with the voxel size."""
    r64 = _quality(gjp, oracle_mod, 64, 101, 6000)
    r128 = _quality(gjp, oracle_mod, 128, 201, 6000)
    for w in ("linear", "spline"):
        ratio = r128[w] / r64[w]
        note(f"quality convergence {w}: {r64[w]:.5f} -> {r128[w]:.5f} (ratio {ratio:.3f})")
        assert ratio <= 0.7, (w, r64[w], r128[w])


@pytest.mark.slow
def test_quality_paper_scale(gjp, oracle_mod):
    """512^3, 512^2 detector, 803 views (the paper's configuration)."""
    r = _quality(gjp, oracle_mod, 512, 803, 6000)
    # regression bounds about 40% above the measured 0.00141 / 0.00202
    assert 0.0 < r["linear"] < 0.002 and 0.0 < r["spline"] < 0.0028
    # the paper's finding at this scale: linear weights fit the analytic
    # projections better than the spline weights (measured: 0.0014 vs 0.0020)
    assert r["linear"] < r["spline"]
