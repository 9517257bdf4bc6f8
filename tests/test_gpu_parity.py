"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: relative L2 <= 1e-5 for FP32 volumes, <= 5e-3 for 16-bit storage
against the unrounded volume, and <= 1e-5 against the 16-bit-rounded volume
(the kernel's own error). Integer outcomes (sample counts) are exact.
"""
import numpy as np
import pytest

import workloads
from gpu_helpers import assert_parity, cuda, note, rel_l2

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL16 = 5e-3


@pytest.fixture(scope="module")
def gjp():
    import paper_1609_00958_amd as m
    return m


def _oracle_geom(oracle_mod, G):
    beam = oracle_mod.CONE if G.beam == 0 else oracle_mod.PARALLEL
    return oracle_mod.Geometry(G.shape, G.views, G.n_u, G.n_v, beam=beam,
                               voxel_size=G.voxel_size, center=G.center, weight=G.weight,
                               clip_cylinder=G.clip_cylinder)


def _to_dev(a, dev, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return t if dtype is None else t.to(dtype)


# ---------------------------------------------------------------------------
# forward, small configurations: full sinograms against the oracle
# ---------------------------------------------------------------------------
def test_forward_c1_fp32(gjp, oracle_mod):
    dev = cuda()
    cfg = workloads.config("c1")
    vol = workloads.rasterize(cfg.phantom_ellipsoids(), cfg.shape)
    G = gjp.Geometry.from_config(cfg)
    note("forward c1 fp32")
    y = gjp.forward(_to_dev(vol, dev), G).cpu().numpy()
    want = oracle_mod.forward(oracle_mod.geometry_for(cfg), vol)
    assert_parity(y, want, TOL32)


@pytest.mark.parametrize("beam", ["cone", "parallel"])
@pytest.mark.parametrize("weight", ["linear", "spline"])
def test_forward_random_geometry(gjp, oracle_mod, beam, weight):
    """Random orientations (every driving axis), ragged detector and grid sizes
    that span several tiles, anisotropic voxels and an offset grid centre."""
    dev = cuda()
    shape = (37, 29, 70)
    vs = (1.0, 1.25, 0.8)
    ctr = (3.0, -1.5, 2.0)
    n_views, n_u, n_v = 11, 45, 131
    gen = workloads.random_cone_views if beam == "cone" else workloads.random_parallel_views
    views = gen(71, n_views, shape, n_u, n_v, voxel_size=vs)
    for k in (0, 3) if beam == "cone" else (3,):
        views[:, k:k + 3] += ctr
    G = gjp.Geometry(shape, views, n_u, n_v, beam=beam, voxel_size=vs, center=ctr, weight=weight)
    og = _oracle_geom(oracle_mod, G)
    vol = workloads.rasterize(workloads.random_ellipsoids(72, shape, voxel_size=vs), shape,
                              voxel_size=vs, center=ctr)
    vol += np.random.default_rng(73).uniform(0, 0.05, size=shape).astype(np.float32)
    note(f"forward random {beam} {weight}")
    y = gjp.forward(_to_dev(vol, dev), G).cpu().numpy()
    want = oracle_mod.forward(og, vol)
    axes = {oracle_mod.ray_info(og, v, n_u // 2, n_v // 2)[0] for v in range(n_views)}
    assert len(axes) >= 2
    assert_parity(y, want, TOL32)


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_forward_16bit_storage(gjp, oracle_mod, dtype):
    import torch
    dev = cuda()
    cfg = workloads.config("c1")
    vol = workloads.rasterize(cfg.phantom_ellipsoids(), cfg.shape)
    vol += np.random.default_rng(74).normal(0, 0.01, size=vol.shape).astype(np.float32)
    tdt = torch.bfloat16 if dtype == "bf16" else torch.float16
    v16 = _to_dev(vol, dev).to(tdt)
    G = gjp.Geometry.from_config(cfg)
    note(f"forward c1 {dtype}")
    y = gjp.forward(v16, G).cpu().numpy()
    og = oracle_mod.geometry_for(cfg)
    rounded = v16.float().cpu().numpy()
    assert_parity(y, oracle_mod.forward(og, rounded), TOL32)   # kernel error
    assert_parity(y, oracle_mod.forward(og, vol), TOL16)       # storage error


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("beam", ["cone", "parallel"])
@pytest.mark.parametrize("weight", ["linear", "spline"])
def test_adjoint_random_geometry(gjp, oracle_mod, beam, weight):
    dev = cuda()
    shape = (23, 31, 66)
    n_views, n_u, n_v = 9, 40, 75
    gen = workloads.random_cone_views if beam == "cone" else workloads.random_parallel_views
    views = gen(81, n_views, shape, n_u, n_v)
    G = gjp.Geometry(shape, views, n_u, n_v, beam=beam, weight=weight)
    og = _oracle_geom(oracle_mod, G)
    y = np.random.default_rng(82).uniform(0, 1, size=G.sino_shape).astype(np.float32)
    note(f"adjoint random {beam} {weight}")
    x = gjp.back(_to_dev(y, dev), G).cpu().numpy()
    want = oracle_mod.adjoint(og, y)
    assert_parity(x, want, TOL32)


def test_adjoint_c1(gjp, oracle_mod):
    dev = cuda()
    cfg = workloads.config("c1")
    G = gjp.Geometry.from_config(cfg)
    y = np.random.default_rng(83).normal(size=G.sino_shape).astype(np.float32)
    note("adjoint c1")
    x = gjp.back(_to_dev(y, dev), G).cpu().numpy()
    want = oracle_mod.adjoint(oracle_mod.geometry_for(cfg), y)
    assert_parity(x, want, TOL32)


@pytest.mark.parametrize("beam", ["cone", "parallel"])
def test_dot_product_gpu(gjp, beam):
    import torch
    dev = cuda()
    shape = (40, 36, 52)
    n_views, n_u, n_v = 13, 57, 61
    gen = workloads.random_cone_views if beam == "cone" else workloads.random_parallel_views
    G = gjp.Geometry(shape, gen(91, n_views, shape, n_u, n_v), n_u, n_v, beam=beam)
    g = torch.Generator(device="cpu").manual_seed(92)
    for signed in (False, True):
        x = torch.rand(shape, generator=g)
        y = torch.randn(G.sino_shape, generator=g) if signed else torch.rand(G.sino_shape,
                                                                              generator=g)
        note(f"dot test {beam} signed={signed}")
        Ax = gjp.forward(x.to(dev), G).double().cpu()
        ATy = gjp.back(y.to(dev), G).double().cpu()
        lhs = float((Ax * y.double()).sum())
        rhs = float((x.double() * ATy).sum())
        assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), abs(rhs))


def test_deterministic(gjp):
    import torch
    dev = cuda()
    cfg = workloads.config("c1")
    G = gjp.Geometry.from_config(cfg)
    x = torch.rand(cfg.shape, generator=torch.Generator().manual_seed(5)).to(dev)
    note("determinism")
    a, b = gjp.forward(x, G), gjp.forward(x, G)
    assert torch.equal(a, b)
    c, d = gjp.back(a, G), gjp.back(a, G)
    assert torch.equal(c, d)
    # random orientations: the tile-splat adjoint
    shape = (30, 34, 40)
    G = gjp.Geometry(shape, workloads.random_cone_views(6, 5, shape, 50, 60), 50, 60)
    y = torch.rand(G.sino_shape, generator=torch.Generator().manual_seed(7)).to(dev)
    c, d = gjp.back(y, G), gjp.back(y, G)
    assert torch.equal(c, d)


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------
def test_edge_cases(gjp, oracle_mod):
    dev = cuda()
    rng = np.random.default_rng(95)
    cases = [
        ((1, 1, 1), 3, 1, 1), ((1, 5, 9), 4, 7, 3), ((9, 1, 4), 5, 2, 65), ((2, 3, 130), 3, 65, 1),
    ]
    for shape, n_views, n_u, n_v in cases:
        for beam in ("cone", "parallel"):
            gen = workloads.random_cone_views if beam == "cone" else workloads.random_parallel_views
            G = gjp.Geometry(shape, gen(96, n_views, shape, n_u, n_v), n_u, n_v, beam=beam)
            og = _oracle_geom(oracle_mod, G)
            vol = rng.uniform(0, 1, size=shape).astype(np.float32)
            note(f"edge {shape} {beam} det {n_u}x{n_v}")
            y = gjp.forward(_to_dev(vol, dev), G).cpu().numpy()
            want = oracle_mod.forward(og, vol)
            assert_parity(y, want, TOL32)
            ys = rng.uniform(0, 1, size=G.sino_shape).astype(np.float32)
            x = gjp.back(_to_dev(ys, dev), G).cpu().numpy()
            assert_parity(x, oracle_mod.adjoint(og, ys), TOL32)
    # rays that miss the grid and a degenerate ray (source on the pixel)
    views = np.zeros((1, 12))
    views[0, 0:3] = [0.25, 0.5, -0.75]
    views[0, 3:6] = [0.25, 0.5, -0.75]
    views[0, 6:9] = [100.0, 0.0, 0.0]
    views[0, 9:12] = [0.0, 100.0, 0.0]
    G = gjp.Geometry((6, 6, 6), views, 3, 2)
    note("edge degenerate")
    y = gjp.forward(_to_dev(np.ones((6, 6, 6), np.float32), dev), G).cpu().numpy()
    og = _oracle_geom(oracle_mod, G)
    np.testing.assert_allclose(y, oracle_mod.forward(og, np.ones((6, 6, 6))), rtol=1e-5,
                               atol=1e-6)
    assert y[0, 0, 0] == 0.0


def test_tile_shapes_bitwise_identical(gjp):
    import torch
    dev = cuda()
    shape = (48, 40, 56)
    n_views, n_u, n_v = 7, 77, 90
    G = gjp.Geometry(shape, workloads.random_cone_views(97, n_views, shape, n_u, n_v), n_u, n_v)
    x = torch.rand(shape, generator=torch.Generator().manual_seed(98)).to(dev)
    note("tile shapes")
    ref = gjp.forward(x, G)
    tv = gjp.autotune(x, G)
    assert tv in (64, 32, 16)
    assert torch.equal(gjp.forward(x, G), ref)


# ---------------------------------------------------------------------------
# 64-bit addressing: a padded plane beyond 24-bit multiplies (or a padded
# volume beyond 4 GiB) selects the 64-bit offset path; small non-cubic grids
# with large planes reach it cheaply.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,shape", [("f32", (5, 1500, 1500)), ("bf16", (4, 2100, 2100))])
def test_forward_64bit_offsets(gjp, oracle_mod, dtype, shape):
    import torch
    dev = cuda()
    # plane stride in bytes of the padded copy exceeds 2^23
    es = 4 if dtype == "f32" else 2
    assert (shape[1] + 2) * (shape[2] + 2) * es >= (1 << 23)
    n_views, n_u, n_v = 6, 40, 90
    for beam in ("cone", "parallel"):
        gen = workloads.random_cone_views if beam == "cone" else workloads.random_parallel_views
        G = gjp.Geometry(shape, gen(101, n_views, shape, n_u, n_v), n_u, n_v, beam=beam)
        og = _oracle_geom(oracle_mod, G)
        vol = np.random.default_rng(102).uniform(0, 1, size=shape).astype(np.float32)
        x = _to_dev(vol, dev)
        if dtype == "bf16":
            x = x.to(torch.bfloat16)
            vol = x.float().cpu().numpy()
        note(f"64-bit offsets {dtype} {shape} {beam}")
        y = gjp.forward(x, G).cpu().numpy()
        rays = workloads.sample_rays(103, 1500, n_views, n_u, n_v)
        got = y[rays[:, 0], rays[:, 1], rays[:, 2]]
        want = oracle_mod.forward_rays(og, vol, rays)
        # Element bound: coordinates here reach ~3000 (ray base plus plane
        # times slope), so each single-precision sample position carries up
        # to delta ~ 2^-24 * 3000 = 1.8e-4 voxel of rounding. On white noise
        # (neighbour differences of sd 0.41) a ray of n samples then errs by
        # about sqrt(n) * 0.41 * delta against a sum of about n / 2, i.e.
        # 0.82 * delta / sqrt(n) = 2e-5 relative at the shortest compared rays
        # (n ~ 50); 1e-4 of the largest value is that at 5 sigma. The relative
        # L2 bound stays the stated 1e-5.
        assert_parity(got, want, TOL32, elem=1e-4)


def test_two_rays_per_lane_64bit_offsets(gjp, oracle_mod):
    """Circular trajectory over planes beyond 24-bit byte strides (the 64-bit
    per-lane fallback is compiled into the two-ray kernel as well)."""
    import torch
    dev = cuda()
    shape = (4, 2050, 2050)
    assert (shape[1] + 2) * (shape[2] + 2) * 2 >= (1 << 23)
    n_views, n_u, n_v = 8, 40, 130
    G = gjp.Geometry.circular_cone(shape, n_views, n_u, n_v, 6000.0, 9000.0, 40.0, 1.2)
    og = _oracle_geom(oracle_mod, G)
    # a smooth phantom: rays here run up to 2050 planes at coordinates in the
    # thousands, where uncorrelated voxel noise would turn single-precision
    # coordinate rounding into more than the tolerance
    vol = workloads.rasterize(workloads.random_ellipsoids(104, shape), shape)
    x = _to_dev(vol, dev).to(torch.bfloat16)
    vol = x.float().cpu().numpy()
    gjp.set_forward_tile(G, torch.bfloat16, 64, 8, 4)
    note("two rays per lane, 64-bit strides: reference tile")
    ref = gjp.forward(x, G)
    gjp.set_forward_tile(G, torch.bfloat16, 128, 8, 2)
    note("two rays per lane, 64-bit strides: 128-wide tile")
    y = gjp.forward(x, G)
    assert torch.equal(y, ref)
    rays = workloads.sample_rays(105, 1500, n_views, n_u, n_v)
    got = y.cpu().numpy()[rays[:, 0], rays[:, 1], rays[:, 2]]
    assert_parity(got, oracle_mod.forward_rays(og, vol, rays), TOL32)


@pytest.mark.parametrize("beam", ["cone", "parallel"])
def test_circular_tiles_bitwise_and_adjoint(gjp, oracle_mod, beam):
    """Circular trajectories: the 64-wide tile takes the row-uniform sampling
    loop, the 32- and 16-wide tiles the per-lane loop; all give identical
    sinograms. The adjoint takes the column-form gather."""
    import torch
    dev = cuda()
    shape = (40, 44, 70)
    n_views, n_u, n_v = 12, 70, 100
    if beam == "cone":
        G = gjp.Geometry.circular_cone(shape, n_views, n_u, n_v, 180.0, 300.0, 1.0, 1.2)
    else:
        G = gjp.Geometry.parallel(shape, n_views, n_u, n_v, 0.9, 0.8)
    og = _oracle_geom(oracle_mod, G)
    vol = workloads.rasterize(workloads.random_ellipsoids(111, shape), shape)
    x = _to_dev(vol, dev)
    outs = []
    configs = [(64, 8, 4), (64, 8, 2), (64, 1, 4), (64, 16, 2), (32, 8, 4), (16, 3, 2)]
    for dt in (torch.float32, torch.bfloat16):
        got = []
        pairs = [(128, 8, 2), (128, 1, 4)] if dt != torch.float32 else []
        for tv, vg, lg in configs + pairs:
            gjp.set_forward_tile(G, dt, tv, vg, lg)
            note(f"circular {beam} tile {tv} views {vg} loads {lg} {dt}")
            got.append(gjp.forward(x.to(dt), G))
        assert all(torch.equal(got[0], o) for o in got[1:])
        outs.append(got[0])
    assert_parity(outs[0].cpu().numpy(), oracle_mod.forward(og, vol), TOL32)
    y = np.random.default_rng(112).uniform(0, 1, size=G.sino_shape).astype(np.float32)
    note(f"circular {beam} adjoint")
    got = gjp.back(_to_dev(y, dev), G).cpu().numpy()
    assert_parity(got, oracle_mod.adjoint(og, y), TOL32)


# ---------------------------------------------------------------------------
# cylinder clipping of the sample range (Sec. IV-C)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("beam", ["cone", "parallel"])
def test_cylinder_clipping_random_geometry(gjp, oracle_mod, beam):
    """Random orientations (general adjoint path), non-square cross-section."""
    dev = cuda()
    shape = (41, 33, 27)
    n_views, n_u, n_v = 9, 47, 39
    gen = workloads.random_cone_views if beam == "cone" else workloads.random_parallel_views
    views = gen(91, n_views, shape, n_u, n_v)
    G = gjp.Geometry(shape, views, n_u, n_v, beam=beam, clip_cylinder=True)
    og = _oracle_geom(oracle_mod, G)
    assert G.count_samples() == oracle_mod.count_samples(og)
    vol = np.random.default_rng(92).uniform(0, 1, size=shape).astype(np.float32)
    note(f"clip forward random {beam}")
    y = gjp.forward(_to_dev(vol, dev), G).cpu().numpy()
    assert_parity(y, oracle_mod.forward(og, vol), TOL32)
    s = np.random.default_rng(93).uniform(0, 1, size=G.sino_shape).astype(np.float32)
    note(f"clip adjoint random {beam}")
    x = gjp.back(_to_dev(s, dev), G).cpu().numpy()
    assert_parity(x, oracle_mod.adjoint(og, s), TOL32)


@pytest.mark.parametrize("beam", ["cone", "parallel"])
def test_cylinder_clipping_circular(gjp, oracle_mod, beam):
    """Circular trajectory (column-form adjoint), grids spanning several tiles
    and a ragged detector."""
    dev = cuda()
    if beam == "cone":
        cfg = workloads.WorkloadConfig("k", (70, 58, 45), 24, 101, 77, beam="cone", sod=240.0,
                                       sdd=480.0, pitch_u=1.6, pitch_v=1.6, clip_cylinder=True)
    else:
        cfg = workloads.WorkloadConfig("q", (66, 66, 40), 20, 90, 41, beam="parallel",
                                       pitch_u=0.8, pitch_v=1.0, clip_cylinder=True)
    G = gjp.Geometry.from_config(cfg)
    og = oracle_mod.geometry_for(cfg)
    vol = workloads.rasterize(workloads.random_ellipsoids(94, cfg.shape), cfg.shape)
    note(f"clip forward circular {beam}")
    y = gjp.forward(_to_dev(vol, dev), G).cpu().numpy()
    assert_parity(y, oracle_mod.forward(og, vol), TOL32)
    s = np.random.default_rng(95).normal(size=G.sino_shape).astype(np.float32)
    note(f"clip adjoint circular {beam}")
    x = gjp.back(_to_dev(s, dev), G).cpu().numpy()
    assert_parity(x, oracle_mod.adjoint(og, s), TOL32)


# ---------------------------------------------------------------------------
# plain one-lane-per-ray forward (comparison kernel)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("beam,weight,clip", [("cone", "linear", False),
                                              ("parallel", "spline", False),
                                              ("cone", "linear", True)])
def test_naive_forward_random_geometry(gjp, oracle_mod, beam, weight, clip):
    """Every driving axis, ragged sizes; against the oracle and the tuned kernel
    (same setup, weights and summation order, so the two agree to rounding)."""
    dev = cuda()
    shape = (33, 27, 52)
    n_views, n_u, n_v = 9, 41, 77
    gen = workloads.random_cone_views if beam == "cone" else workloads.random_parallel_views
    views = gen(76, n_views, shape, n_u, n_v)
    G = gjp.Geometry(shape, views, n_u, n_v, beam=beam, weight=weight, clip_cylinder=clip)
    og = _oracle_geom(oracle_mod, G)
    vol = workloads.rasterize(workloads.random_ellipsoids(77, shape), shape)
    note(f"naive forward {beam} {weight} clip={clip}")
    tv = _to_dev(vol, dev)
    y = gjp.forward_naive(tv, G).cpu().numpy()
    assert_parity(y, oracle_mod.forward(og, vol), TOL32)
    y_tuned = gjp.forward(tv, G).cpu().numpy()
    assert rel_l2(y, y_tuned) <= 1e-6
    note(f"naive vs tuned: {int(np.sum(y != y_tuned))} of {y.size} values differ in rounding")


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_naive_forward_16bit(gjp, oracle_mod, dtype):
    import torch
    dev = cuda()
    cfg = workloads.config("c1")
    vol = workloads.rasterize(cfg.phantom_ellipsoids(), cfg.shape)
    tdt = torch.bfloat16 if dtype == "bf16" else torch.float16
    v16 = _to_dev(vol, dev).to(tdt)
    G = gjp.Geometry.from_config(cfg)
    note(f"naive forward c1 {dtype}")
    y = gjp.forward_naive(v16, G).cpu().numpy()
    og = oracle_mod.geometry_for(cfg)
    assert_parity(y, oracle_mod.forward(og, v16.float().cpu().numpy()), TOL32)
    assert_parity(y, oracle_mod.forward(og, vol), TOL16)


# ---------------------------------------------------------------------------
# two rays per lane (16-bit storage, 128-wide tiles): the shared load applies
# when the two rays' axis-2 coordinates stay within a voxel; otherwise each ray
# runs alone. Either way the sums equal the one-ray tiles' bit for bit.
# ---------------------------------------------------------------------------
def _flip_v(views, n_v):
    out = views.copy()
    out[:, 3:6] = views[:, 3:6] + (n_v - 1) * views[:, 9:12]
    out[:, 9:12] = -views[:, 9:12]
    return out


@pytest.mark.parametrize("case", ["cone", "flipped", "coarse", "parallel", "clipped"])
def test_two_rays_per_lane_bitwise(gjp, oracle_mod, case):
    import torch
    dev = cuda()
    shape = (46, 40, 66)
    n_views, n_u, n_v = 10, 53, 141  # odd n_v: the last lane's second ray is off the detector
    clip = case == "clipped"
    if case == "parallel":
        views = gjp.views_parallel(n_views, 0.9, 0.8, n_u, n_v)
        beam = "parallel"
    else:
        # coarse: v pitch of about 2.4 voxels at the axis, so the rays of a
        # lane drift more than a voxel apart and the path falls back
        pv = 3.6 if case == "coarse" else 1.1
        views = gjp.views_circular_cone(n_views, 160.0, 240.0, 1.2, pv, n_u, n_v)
        beam = "cone"
    if case == "flipped":
        views = _flip_v(views, n_v)
    G = gjp.Geometry(shape, views, n_u, n_v, beam=beam, clip_cylinder=clip)
    vol = workloads.rasterize(workloads.random_ellipsoids(121, shape), shape)
    for dt in (torch.bfloat16, torch.float16):
        x = _to_dev(vol, dev).to(dt)
        gjp.set_forward_tile(G, dt, 64, 8, 4)
        note(f"two rays per lane {case} {dt}: reference tile")
        ref = gjp.forward(x, G)
        for vg, lg in ((8, 2), (1, 4), (16, 2)):
            gjp.set_forward_tile(G, dt, 128, vg, lg)
            note(f"two rays per lane {case} {dt}: views {vg} loads {lg}")
            assert torch.equal(gjp.forward(x, G), ref)
    og = _oracle_geom(oracle_mod, G)
    rounded = _to_dev(vol, dev).to(torch.float16).float().cpu().numpy()
    y = gjp.forward(_to_dev(vol, dev).to(torch.float16), G).cpu().numpy()
    assert_parity(y, oracle_mod.forward(og, rounded), TOL32)


# ---------------------------------------------------------------------------
# three rays per lane (192-wide tiles): one 16-byte load (two for FP32) serves
# three rays whose axis-2 coordinates step by less than a voxel; each element
# is interpolated along the row first, so the sums match the oracle (on the
# 16-bit-rounded volume for 16-bit storage) within the FP32 tolerance rather
# than bit for bit.
# Geometries where the check fails run the one-ray path.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["cone", "flipped", "coarse", "parallel", "clipped", "spline"])
def test_three_rays_per_lane(gjp, oracle_mod, case):
    import torch
    dev = cuda()
    shape = (46, 40, 66)
    n_views, n_u, n_v = 10, 53, 200  # 200 = 192 + 8: a ragged second tile
    clip = case == "clipped"
    weight = "spline" if case == "spline" else "linear"
    if case == "parallel":
        views = gjp.views_parallel(n_views, 0.9, 0.33, n_u, n_v)
        beam = "parallel"
    else:
        # coarse: v pitch of about 1.7 voxels at the axis, so neighbouring
        # rays drift more than a voxel apart and the path falls back
        pv = 2.6 if case == "coarse" else 0.45
        views = gjp.views_circular_cone(n_views, 160.0, 240.0, 1.2, pv, n_u, n_v)
        beam = "cone"
    if case == "flipped":
        views = _flip_v(views, n_v)
    G = gjp.Geometry(shape, views, n_u, n_v, beam=beam, clip_cylinder=clip, weight=weight)
    og = _oracle_geom(oracle_mod, G)
    vol = workloads.rasterize(workloads.random_ellipsoids(141, shape), shape)
    vol += np.random.default_rng(142).uniform(0, 0.05, size=shape).astype(np.float32)
    for dt in (torch.float32, torch.bfloat16, torch.float16):
        x = _to_dev(vol, dev).to(dt)
        rounded = x.float().cpu().numpy()
        want = oracle_mod.forward(og, rounded)
        for vg, lg in ((16, 2), (1, 4)):
            gjp.set_forward_tile(G, dt, 192, vg, lg)
            note(f"three rays per lane {case} {dt}: views {vg} loads {lg}")
            y = gjp.forward(x, G).cpu().numpy()
            assert_parity(y, want, TOL32)
        gjp.reset_forward_tile(G, dt)


@pytest.mark.parametrize("beam", ["cone", "parallel"])
def test_circular_spline_adjoint(gjp, oracle_mod, beam):
    """Spline weights (Eq. 14) on circular trajectories: the column-form gather
    with the forward's floor-and-select weights, against the oracle."""
    dev = cuda()
    shape = (38, 42, 60)
    n_views, n_u, n_v = 11, 64, 90
    if beam == "cone":
        G = gjp.Geometry.circular_cone(shape, n_views, n_u, n_v, 170.0, 290.0, 1.1, 1.1,
                                       weight="spline")
    else:
        G = gjp.Geometry.parallel(shape, n_views, n_u, n_v, 0.9, 0.8, weight="spline")
    og = _oracle_geom(oracle_mod, G)
    vol = workloads.rasterize(workloads.random_ellipsoids(131, shape), shape)
    note(f"circular spline {beam}: forward")
    y = gjp.forward(_to_dev(vol, dev), G).cpu().numpy()
    assert_parity(y, oracle_mod.forward(og, vol), TOL32)
    s = np.random.default_rng(132).uniform(0, 1, size=G.sino_shape).astype(np.float32)
    note(f"circular spline {beam}: adjoint")
    got = gjp.back(_to_dev(s, dev), G).cpu().numpy()
    assert_parity(got, oracle_mod.adjoint(og, s), TOL32)


# ---------------------------------------------------------------------------
# column-form adjoint gather: branches that need special geometries
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("weight", ["linear", "spline"])
def test_gather_fine_detector_pitch(gjp, oracle_mod, weight):
    """A detector pitch of 0.25 voxel along v at magnification 1.5 (six
    detector rows per voxel): a voxel's candidate rays per detector column
    exceed the unrolled lengths, so the gather takes its per-lane loop."""
    dev = cuda()
    shape = (30, 26, 22)
    n_views, n_u, n_v = 8, 60, 140
    G = gjp.Geometry.circular_cone(shape, n_views, n_u, n_v, 120.0, 180.0, 1.0, 0.25,
                                   weight=weight)
    og = _oracle_geom(oracle_mod, G)
    y = np.random.default_rng(141).uniform(0, 1, size=G.sino_shape).astype(np.float32)
    note(f"gather fine v pitch {weight}")
    x = gjp.back(_to_dev(y, dev), G).cpu().numpy()
    assert_parity(x, oracle_mod.adjoint(og, y), TOL32)
    vol = workloads.rasterize(workloads.random_ellipsoids(142, shape), shape)
    note(f"forward fine v pitch {weight}")
    f = gjp.forward(_to_dev(vol, dev), G).cpu().numpy()
    assert_parity(f, oracle_mod.forward(og, vol), TOL32)


@pytest.mark.parametrize("sod", [9.0, 14.0])
def test_gather_source_inside_grid(gjp, oracle_mod, sod):
    """Source closer to the rotation axis than the grid's half extent: every
    ray is a full line through the grid (Algorithm 1 samples every plane the
    line crosses), so voxels on or behind the source plane receive
    contributions; the gather cannot bound their detector windows and reads
    whole columns."""
    dev = cuda()
    shape = (36, 34, 16)
    n_views, n_u, n_v = 10, 70, 20
    G = gjp.Geometry.circular_cone(shape, n_views, n_u, n_v, sod, sod + 30.0, 1.5, 0.9)
    og = _oracle_geom(oracle_mod, G)
    y = np.random.default_rng(143).uniform(0, 1, size=G.sino_shape).astype(np.float32)
    note(f"gather source inside grid sod={sod}")
    x = gjp.back(_to_dev(y, dev), G).cpu().numpy()
    want = oracle_mod.adjoint(og, y)
    assert_parity(x, want, TOL32)
    vol = workloads.rasterize(workloads.random_ellipsoids(144, shape), shape)
    note(f"forward source inside grid sod={sod}")
    f = gjp.forward(_to_dev(vol, dev), G).cpu().numpy()
    assert_parity(f, oracle_mod.forward(og, vol), TOL32)


# ---------------------------------------------------------------------------
# system matrix entry by entry on tiny grids (forward columns from one-hot
# volumes, adjoint columns from one-hot sinograms)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["cone_random", "parallel_random", "circular", "spline"])
def test_system_matrix_entries(gjp, oracle_mod, case):
    import torch
    dev = cuda()
    shape = (5, 4, 6)
    n_views, n_u, n_v = 3, 5, 7
    weight = "spline" if case == "spline" else "linear"
    if case == "cone_random":
        G = gjp.Geometry(shape, workloads.random_cone_views(151, n_views, shape, n_u, n_v),
                         n_u, n_v, beam="cone")
    elif case == "parallel_random":
        G = gjp.Geometry(shape, workloads.random_parallel_views(152, n_views, shape, n_u, n_v),
                         n_u, n_v, beam="parallel")
    else:
        G = gjp.Geometry.circular_cone(shape, n_views, n_u, n_v, 20.0, 32.0, 1.6, 1.6,
                                       weight=weight)
    og = _oracle_geom(oracle_mod, G)
    n_vox = int(np.prod(shape))
    n_rays = n_views * n_u * n_v
    A_gpu = np.zeros((n_rays, n_vox))
    A_ora = np.zeros((n_rays, n_vox))
    note(f"system matrix {case}: forward columns")
    for j in range(n_vox):
        e = np.zeros(n_vox, dtype=np.float32)
        e[j] = 1.0
        e = e.reshape(shape)
        A_gpu[:, j] = gjp.forward(_to_dev(e, dev), G).cpu().numpy().reshape(-1)
        A_ora[:, j] = oracle_mod.forward(og, e).reshape(-1)
    assert np.abs(A_ora).max() > 0.5
    np.testing.assert_allclose(A_gpu, A_ora, rtol=0, atol=1e-6)
    note(f"system matrix {case}: adjoint columns")
    AT_gpu = np.zeros((n_vox, n_rays))
    for r in range(n_rays):
        e = torch.zeros(n_rays)
        e[r] = 1.0
        AT_gpu[:, r] = gjp.back(e.reshape(G.sino_shape).to(dev), G).cpu().numpy().reshape(-1)
    np.testing.assert_allclose(AT_gpu, A_ora.T, rtol=0, atol=1e-6)
