"""GPU: the forward that allocates nothing (fixed device scratch) against the
ordinary forward and the FP64 oracle, through the C ABI.

Two calls in a row share the scratch, the second with a smaller input, so a
stale value left by the first call would show up in the second. The sums are
the ordinary forward's bit for bit (same kernels, launch configuration and
rounding order) and within 1e-5 relative L2 of the oracle.
"""
import numpy as np
import pytest

import workloads
from gpu_helpers import assert_parity, cuda, note

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


@pytest.fixture(scope="module")
def gjp():
    import paper_1609_00958_amd as m
    return m


def _to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _random_case(gjp, seed, shape, n_views, n_u, n_v):
    views = workloads.random_cone_views(seed, n_views, shape, n_u, n_v)
    G = gjp.Geometry(shape, views, n_u, n_v, beam="cone")
    vol = workloads.rasterize(workloads.random_ellipsoids(seed + 1, shape), shape)
    vol += np.random.default_rng(seed + 2).uniform(0, 0.05, size=shape).astype(np.float32)
    return G, vol


def _oracle_geom(oracle_mod, G):
    beam = oracle_mod.CONE if G.beam == 0 else oracle_mod.PARALLEL
    return oracle_mod.Geometry(G.shape, G.views, G.n_u, G.n_v, beam=beam,
                               voxel_size=G.voxel_size, center=G.center, weight=G.weight,
                               clip_cylinder=G.clip_cylinder)


def test_noalloc_two_calls_shrinking(gjp, oracle_mod):
    import torch
    dev = cuda()
    cfg = workloads.config("c1")
    vol1 = workloads.rasterize(cfg.phantom_ellipsoids(), cfg.shape)
    G1 = gjp.Geometry.from_config(cfg)
    G2, vol2 = _random_case(gjp, 91, (37, 29, 46), 7, 45, 67)
    x1, x2 = _to_dev(vol1, dev), _to_dev(vol2, dev)
    # the ordinary forward first: it also makes the geometries' device copies
    note("noalloc: ordinary forwards (c1, random 37x29x46)")
    ref1 = gjp.forward(x1, G1).cpu().numpy()
    ref2 = gjp.forward(x2, G2).cpu().numpy()
    y1 = torch.full(G1.sino_shape, float("nan"), device=dev)
    y2 = torch.full(G2.sino_shape, float("nan"), device=dev)
    note("noalloc: call 1 (c1 64^3)")
    gjp.forward_noalloc(x1, G1, y1)
    torch.cuda.synchronize()
    note("noalloc: call 2 (37x29x46, smaller)")
    gjp.forward_noalloc(x2, G2, y2)
    torch.cuda.synchronize()
    got1, got2 = y1.cpu().numpy(), y2.cpu().numpy()
    assert np.array_equal(got1, ref1)
    assert np.array_equal(got2, ref2)
    assert_parity(got1, oracle_mod.forward(oracle_mod.geometry_for(cfg), vol1), TOL32)
    assert_parity(got2, oracle_mod.forward(_oracle_geom(oracle_mod, G2), vol2), TOL32)


def test_noalloc_16bit_and_repeat(gjp, oracle_mod):
    """BF16 storage, then the FP32 call again: the scratch holds the other
    element size's copies in between."""
    import torch
    dev = cuda()
    G, vol = _random_case(gjp, 93, (41, 52, 33), 5, 60, 48)
    x = _to_dev(vol, dev)
    xb = x.to(torch.bfloat16)
    ref = gjp.forward(x, G).cpu().numpy()
    refb = gjp.forward(xb, G).cpu().numpy()
    yb = torch.empty(G.sino_shape, device=dev)
    y = torch.empty(G.sino_shape, device=dev)
    note("noalloc: bf16 41x52x33 then fp32")
    gjp.forward_noalloc(xb, G, yb)
    gjp.forward_noalloc(x, G, y)
    torch.cuda.synchronize()
    assert np.array_equal(yb.cpu().numpy(), refb)
    assert np.array_equal(y.cpu().numpy(), ref)
    og = _oracle_geom(oracle_mod, G)
    assert_parity(yb.cpu().numpy(), oracle_mod.forward(og, xb.float().cpu().numpy()), TOL32)


def test_noalloc_rejects_oversize_and_unuploaded(gjp):
    import torch
    dev = cuda()
    # 160^3 FP32: the two padded copies need more than the 64 MiB scratch
    shape = (160, 160, 160)
    views = workloads.random_cone_views(95, 2, shape, 8, 8)
    G = gjp.Geometry(shape, views, 8, 8, beam="cone")
    x = torch.zeros(shape, device=dev)
    y = torch.empty(G.sino_shape, device=dev)
    note("noalloc: oversize (host check only)")
    with pytest.raises(gjp.GJPError, match="scratch"):
        gjp.forward_noalloc(x, G, y)
    # a geometry never used on this device has no device copy yet
    G2, vol2 = _random_case(gjp, 96, (16, 16, 16), 2, 8, 8)
    y2 = torch.empty(G2.sino_shape, device=dev)
    with pytest.raises(gjp.GJPError, match="no copy on this device"):
        gjp.forward_noalloc(_to_dev(vol2, dev), G2, y2)
    # after an ordinary call it works
    gjp.forward(_to_dev(vol2, dev), G2)
    gjp.forward_noalloc(_to_dev(vol2, dev), G2, y2)
    torch.cuda.synchronize()
    assert np.array_equal(y2.cpu().numpy(), gjp.forward(_to_dev(vol2, dev), G2).cpu().numpy())
