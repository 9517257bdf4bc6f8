"""GPU tests of the batched persistent launch, the autograd wrapper and the
full-size workload configurations (checked on sampled rays)."""
import numpy as np
import pytest

import workloads
from gpu_helpers import assert_parity, cuda, note, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gjp():
    import paper_1609_00958_amd as m
    return m


def _oracle_geom(oracle_mod, G):
    beam = oracle_mod.CONE if G.beam == 0 else oracle_mod.PARALLEL
    return oracle_mod.Geometry(G.shape, G.views, G.n_u, G.n_v, beam=beam,
                               voxel_size=G.voxel_size, center=G.center, weight=G.weight,
                               clip_cylinder=G.clip_cylinder)


# ---------------------------------------------------------------------------
# batched persistent launch
# ---------------------------------------------------------------------------
def _small_instances(gjp, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(7):
        shape = tuple(int(s) for s in rng.integers(9, 60, size=3))
        n_views = int(rng.integers(3, 12))
        n_u, n_v = (int(s) for s in rng.integers(5, 90, size=2))
        beam = "cone" if k % 2 == 0 else "parallel"
        gen = workloads.random_cone_views if beam == "cone" else workloads.random_parallel_views
        G = gjp.Geometry(shape, gen(seed + k, n_views, shape, n_u, n_v), n_u, n_v, beam=beam,
                         weight="spline" if k == 3 else "linear")
        out.append(G)
    return out


def test_batched_equals_single_launches(gjp):
    import torch
    dev = cuda()
    geoms = _small_instances(gjp, 200)
    dtypes = [torch.float32, torch.bfloat16, torch.float32, torch.float16, torch.float32,
              torch.float32, torch.bfloat16]
    for rep in range(3):   # first call captures the graph, later calls replay it
        gen = torch.Generator().manual_seed(300 + rep)
        vols = [torch.rand(G.shape, generator=gen).to(dev).to(dt) for G, dt in zip(geoms, dtypes)]
        note(f"batched rep {rep}")
        outs = gjp.forward_batched(vols, geoms)
        torch.cuda.synchronize()
        for v, G, o in zip(vols, geoms, outs):
            ref = gjp.forward(v, G)
            assert torch.equal(o, ref)


def test_batched_with_cylinder_clipping(gjp, oracle_mod):
    """Clipped and unclipped instances in one batched launch: each equals its
    single-instance forward bitwise and the oracle within the FP32 bound."""
    import torch
    dev = cuda()
    geoms = []
    for k, cfg in enumerate((
            workloads.WorkloadConfig("a", (40, 36, 30), 12, 50, 33, beam="cone", sod=150.0,
                                     sdd=300.0, pitch_u=1.7, pitch_v=1.7, clip_cylinder=True),
            workloads.WorkloadConfig("b", (33, 33, 20), 9, 44, 21, beam="parallel",
                                     clip_cylinder=True),
            workloads.WorkloadConfig("c", (28, 31, 25), 7, 40, 30, beam="cone", sod=120.0,
                                     sdd=240.0, pitch_u=1.6, pitch_v=1.6))):
        geoms.append(gjp.Geometry.from_config(cfg, weight="spline" if k == 1 else "linear"))
    gen = torch.Generator().manual_seed(310)
    vols = [torch.rand(G.shape, generator=gen).to(dev) for G in geoms]
    note("batched clipped")
    outs = gjp.forward_batched(vols, geoms)
    torch.cuda.synchronize()
    for v, G, o in zip(vols, geoms, outs):
        assert torch.equal(o, gjp.forward(v, G))
        want = oracle_mod.forward(_oracle_geom(oracle_mod, G), v.cpu().numpy())
        assert_parity(o.cpu().numpy(), want, 1e-5)


def test_batched_matches_oracle(gjp, oracle_mod):
    import torch
    dev = cuda()
    geoms = _small_instances(gjp, 210)
    gen = torch.Generator().manual_seed(311)
    vols = [torch.rand(G.shape, generator=gen) for G in geoms]
    note("batched vs oracle")
    outs = gjp.forward_batched([v.to(dev) for v in vols], geoms)
    for v, G, o in zip(vols, geoms, outs):
        want = oracle_mod.forward(_oracle_geom(oracle_mod, G), v.numpy())
        assert_parity(o.cpu().numpy(), want, 1e-5)


def test_batched_two_streams_one_plan(gjp):
    """Two streams replay the same plan (same geometry list) with different
    volumes and outputs: each replay waits for the previous one on the device,
    so both results equal the single-instance forwards bit for bit."""
    import torch
    dev = cuda()
    geoms = _small_instances(gjp, 220)
    gen = torch.Generator().manual_seed(320)
    vols_a = [torch.rand(G.shape, generator=gen).to(dev) for G in geoms]
    vols_b = [torch.rand(G.shape, generator=gen).to(dev) for G in geoms]
    note("batched two streams: plan")
    gjp.forward_batched(vols_a, geoms)   # builds and captures the plan
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs_a = [torch.empty(G.sino_shape, device=dev) for G in geoms]
    outs_b = [torch.empty(G.sino_shape, device=dev) for G in geoms]
    note("batched two streams: replays")
    for _ in range(3):
        with torch.cuda.stream(s1):
            gjp.forward_batched(vols_a, geoms, outs_a)
        with torch.cuda.stream(s2):
            gjp.forward_batched(vols_b, geoms, outs_b)
    torch.cuda.synchronize()
    for va, vb, G, oa, ob in zip(vols_a, vols_b, geoms, outs_a, outs_b):
        assert torch.equal(oa, gjp.forward(va, G))
        assert torch.equal(ob, gjp.forward(vb, G))


def test_batched_full_c4_instances(gjp, oracle_mod):
    """The uneven batched workload at its real size (32 instances, edges
    96-320, 90-360 views, detectors 128^2-512^2, cone or parallel): every
    instance's sinogram equals its single-instance forward bit for bit and
    matches the oracle on sampled rays."""
    import torch
    from workloads.configs import batched_instances
    dev = cuda()
    insts = batched_instances()
    note("c4 batched: rasterise 32 instances")
    geoms = [gjp.Geometry.from_config(cfg) for cfg in insts]
    vols = [workloads.rasterize_torch(cfg.phantom_ellipsoids(), cfg.shape, dev) for cfg in insts]
    note("c4 batched: one batched launch")
    outs = gjp.forward_batched(vols, geoms)
    torch.cuda.synchronize()
    for k, (cfg, G, v, o) in enumerate(zip(insts, geoms, vols, outs)):
        note(f"c4 batched: instance {k} {cfg.shape} {cfg.beam} {cfg.n_views} views {cfg.n_u}^2")
        assert torch.equal(o, gjp.forward(v, G)), k
        rays = workloads.sample_rays(400 + k, 150, cfg.n_views, cfg.n_u, cfg.n_v)
        got = o.cpu().numpy()[rays[:, 0], rays[:, 1], rays[:, 2]]
        want = oracle_mod.forward_rays(oracle_mod.geometry_for(cfg), v.cpu().numpy(), rays)
        assert_parity(got, want, 1e-5)


def test_batched_fewer_groups_than_queues(gjp, oracle_mod):
    """Instances of one view and one ray tile each (classes with fewer view
    groups than the per-XCD queues, so most queues start empty and
    workgroups take their items from other XCDs' queues), alone and mixed
    with a larger instance: bitwise equal to the single launches (capture and
    replay) and within the FP32 bound of the oracle."""
    import torch
    dev = cuda()
    geoms = []
    for k, (shape, n_u, n_v, beam) in enumerate((((7, 9, 11), 5, 6, "cone"),
                                                  ((12, 8, 10), 3, 8, "parallel"),
                                                  ((9, 9, 9), 4, 4, "cone"))):
        gen = workloads.random_cone_views if beam == "cone" else workloads.random_parallel_views
        geoms.append(gjp.Geometry(shape, gen(500 + k, 1, shape, n_u, n_v), n_u, n_v, beam=beam))
    big = _small_instances(gjp, 230)[0]
    gen = torch.Generator().manual_seed(330)
    dtypes = [torch.float32, torch.bfloat16, torch.float32]
    vols = [torch.rand(G.shape, generator=gen).to(dev).to(dt) for G, dt in zip(geoms, dtypes)]
    vol_big = torch.rand(big.shape, generator=gen).to(dev)
    for sel in ([0], [0, 1, 2], [0, 1, 2, 3]):
        gs = [geoms[i] if i < 3 else big for i in sel]
        vs = [vols[i] if i < 3 else vol_big for i in sel]
        for rep in range(2):
            note(f"batched tiny instances {sel} rep {rep}")
            outs = gjp.forward_batched(vs, gs)
            torch.cuda.synchronize()
            for v, G, o in zip(vs, gs, outs):
                assert torch.equal(o, gjp.forward(v, G))
    for v, G in zip(vols, geoms):
        want = oracle_mod.forward(_oracle_geom(oracle_mod, G), v.float().cpu().numpy())
        assert_parity(gjp.forward(v, G).cpu().numpy(), want, 1e-5)


def test_batched_tuned_tiles(gjp, oracle_mod):
    """Instances of the uneven workload with set tile shapes (three rays per
    lane, one ray, two rays per lane for 16-bit storage) in one batched
    launch: the three-rays-per-lane instances run in classes of their own;
    every sinogram equals the single-instance forward with the same tile bit
    for bit (capture and replay) and matches the oracle on sampled rays."""
    import torch
    from workloads.configs import batched_instances
    dev = cuda()
    insts = batched_instances()[:6]
    dts = [torch.float32, torch.bfloat16, torch.float16, torch.float32, torch.float16,
           torch.bfloat16]
    tiles = [(192, 8, 4), (64, 8, 4), (128, 16, 4), (192, 16, 2), (192, 1, 4), (64, 16, 2)]
    geoms = [gjp.Geometry.from_config(cfg) for cfg in insts]
    vols = [workloads.rasterize_torch(cfg.phantom_ellipsoids(), cfg.shape, dev).to(dt)
            for cfg, dt in zip(insts, dts)]
    try:
        for G, dt, t in zip(geoms, dts, tiles):
            gjp.set_forward_tile(G, dt, *t)
        for rep in range(2):
            note(f"batched tuned tiles: rep {rep}")
            outs = gjp.forward_batched(vols, geoms)
            torch.cuda.synchronize()
            for k, (cfg, G, v, o) in enumerate(zip(insts, geoms, vols, outs)):
                assert torch.equal(o, gjp.forward(v, G)), (k, tiles[k])
        for k, (cfg, v, o) in enumerate(zip(insts, vols, outs)):
            rays = workloads.sample_rays(700 + k, 150, cfg.n_views, cfg.n_u, cfg.n_v)
            got = o.cpu().numpy()[rays[:, 0], rays[:, 1], rays[:, 2]]
            want = oracle_mod.forward_rays(oracle_mod.geometry_for(cfg),
                                           v.float().cpu().numpy(), rays)
            assert_parity(got, want, 1e-5)
    finally:
        for G, dt in zip(geoms, dts):
            gjp.set_forward_tile(G, dt, 0, 1, 4)


# ---------------------------------------------------------------------------
# autograd wrapper: gradient = adjoint; central differences of the quadratic loss
# ---------------------------------------------------------------------------
def test_autograd_gradient_is_adjoint(gjp):
    import torch
    dev = cuda()
    cfg = workloads.config("c1")
    G = gjp.Geometry.from_config(cfg)
    x = torch.rand(cfg.shape, generator=torch.Generator().manual_seed(7)).to(dev)
    x.requires_grad_(True)
    w = torch.randn(G.sino_shape, generator=torch.Generator().manual_seed(8)).to(dev)
    note("autograd")
    y = gjp.project(x, G)
    (y * w).sum().backward()
    assert torch.equal(x.grad, gjp.back(w, G))
    # bf16 input: gradient comes back in the input's dtype
    xb = x.detach().to(torch.bfloat16).requires_grad_(True)
    (gjp.project(xb, G) * w).sum().backward()
    assert xb.grad.dtype == torch.bfloat16


def test_finite_differences_gpu(gjp):
    """L(x) = 0.5 ||Ax - b||^2 is quadratic, so the central difference equals the
    gradient A^T(Ax - b) up to rounding; losses accumulated in FP64."""
    import torch
    dev = cuda()
    shape = (48, 48, 48)
    G = gjp.Geometry(shape, workloads.random_cone_views(121, 16, shape, 72, 72), 72, 72)
    gen = torch.Generator().manual_seed(122)
    x = torch.rand(shape, generator=gen).to(dev)
    b = (gjp.forward(x, G) + 0.5 * torch.randn(G.sino_shape, generator=gen).to(dev)).detach()
    x0 = torch.rand(shape, generator=gen).to(dev)

    def loss(z):
        r = gjp.forward(z, G).double() - b.double()
        return 0.5 * float((r * r).sum())

    note("finite differences")
    grad = gjp.back(gjp.forward(x0, G) - b, G).double()
    rng = np.random.default_rng(123)
    idx = [tuple(int(t) for t in rng.integers(8, 40, size=3)) for _ in range(64)]
    # the loss is quadratic, so the central difference is exact for any step; a
    # large step keeps the FP32 rounding of the affected rays (~1e-6 relative,
    # divided by 2 eps) well under the tolerance
    eps = float(x0.abs().max())
    for v in idx:
        xp = x0.clone()
        xm = x0.clone()
        xp[v] += eps
        xm[v] -= eps
        fd = (loss(xp) - loss(xm)) / (2 * eps)
        g = float(grad[v])
        assert abs(fd - g) <= 1e-4 * max(abs(g), 1e-3 * float(grad.abs().max())), (v, fd, g)


def test_gradient_descent_monotone(gjp):
    import torch
    dev = cuda()
    shape = (40, 40, 40)
    G = gjp.Geometry(shape, gjp.views_circular_cone(48, 160.0, 240.0, 1.0, 1.0, 60, 60), 60, 60)
    ells = workloads.random_ellipsoids(131, shape)
    truth = torch.from_numpy(workloads.rasterize(ells, shape)).to(dev)
    b = gjp.forward(truth, G)
    # step 1/L with L from power iterations on A^T A
    v = torch.rand(shape, generator=torch.Generator().manual_seed(132)).to(dev)
    for _ in range(10):
        v = gjp.back(gjp.forward(v, G), G)
        lam = float(v.norm())
        v = v / lam
    x = torch.zeros(shape, device=dev, requires_grad=True)
    losses = []
    note("gradient descent")
    for _ in range(8):
        x.grad = None
        loss = 0.5 * ((gjp.project(x, G) - b) ** 2).sum()
        loss.backward()
        losses.append(float(loss))
        with torch.no_grad():
            x -= x.grad / (1.05 * lam)
    assert all(b2 < b1 for b1, b2 in zip(losses, losses[1:]))
    assert losses[-1] < 0.5 * losses[0]


# ---------------------------------------------------------------------------
# full-size configurations in the benchmark's launch setup, on sampled rays
# ---------------------------------------------------------------------------
def _full_config_check(gjp, oracle_mod, name, n_rays, dtypes=("f32",), pairs=False, tiles=()):
    """Sampled rays of the full workload against the oracle; with pairs, every
    16-bit sinogram of the two-rays-per-lane tile is also compared bit for bit
    with the one-ray tile's; tiles: further launch configurations (tile_v,
    view group, load group) checked against the oracle on the same rays."""
    import torch
    dev = cuda()
    cfg = workloads.config(name)
    note(f"{name}: rasterise {cfg.shape}")
    x = workloads.rasterize_torch(cfg.phantom_ellipsoids(), cfg.shape, dev)
    G = gjp.Geometry.from_config(cfg)
    og = oracle_mod.geometry_for(cfg)
    rays = workloads.sample_rays(51, n_rays, cfg.n_views, cfg.n_u, cfg.n_v)
    idx = torch.from_numpy(rays.astype(np.int64))
    for dt in dtypes:
        xd = {"f32": x, "bf16": x.to(torch.bfloat16), "f16": x.to(torch.float16)}[dt]
        note(f"{name}: forward {dt}")
        tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[dt]
        if pairs:
            gjp.set_forward_tile(G, tdt, 64, 8, 4)
        y = gjp.forward(xd, G)
        if pairs and dt != "f32":
            note(f"{name}: forward {dt}, two rays per lane")
            gjp.set_forward_tile(G, tdt, 128, 16, 2)
            y2 = gjp.forward(xd, G)
            gjp.set_forward_tile(G, tdt, 64, 8, 4)
            assert torch.equal(y2, y), (name, dt)
            del y2
        got = y[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
        del y
        host = xd.float().cpu().numpy()
        want = oracle_mod.forward_rays(og, host, rays)
        note(f"{name}: {dt} parity on {len(rays)} sampled rays")
        assert_parity(got, want, 1e-5)
        if pairs:
            # three rays per lane: row-first interpolation, equal up to rounding
            note(f"{name}: forward {dt}, three rays per lane")
            gjp.set_forward_tile(G, tdt, 192, 16, 2)
            y3 = gjp.forward(xd, G)
            gjp.set_forward_tile(G, tdt, 64, 8, 4)
            assert_parity(y3[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy(), want, 1e-5)
            del y3
        for t in tiles:
            note(f"{name}: forward {dt}, launch configuration {t}")
            gjp.set_forward_tile(G, tdt, *t)
            yt = gjp.forward(xd, G)
            gjp.set_forward_tile(G, tdt, 0, 1, 4)
            assert_parity(yt[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy(), want, 1e-5)
            del yt
        if dt != "f32":
            want32 = oracle_mod.forward_rays(og, x.cpu().numpy(), rays)
            assert_parity(got, want32, 5e-3)
        del host, xd
    return cfg, G, og, x


def test_full_c2_forward_and_adjoint(gjp, oracle_mod):
    import torch
    cfg, G, og, x = _full_config_check(gjp, oracle_mod, "c2", 4000,
                                       dtypes=("f32", "bf16", "f16"), pairs=True)
    dev = x.device
    # adjoint: sinogram non-zero on three views only, so the oracle stays cheap
    y = torch.zeros(G.sino_shape)
    gen = torch.Generator().manual_seed(52)
    for v in (0, 45, 181):
        y[v] = torch.rand(G.n_u, G.n_v, generator=gen)
    note("c2: adjoint")
    got = gjp.back(y.to(dev), G).cpu().numpy()
    want = oracle_mod.adjoint(og, y.numpy())
    # Element bound: at these coordinates (source 1024 voxels out, ray bases
    # in the hundreds) single-precision sample positions, and so the weights,
    # err by up to delta ~ 2^-24 * 700 = 4e-5; a voxel sums about 27 terms
    # (three views, about 3 x 3 rays each) of white-noise values y in [0, 1),
    # so at random signs |error| ~ sqrt(27) * 2 * delta * 0.5 = 2e-4, about 3e-5
    # of the largest value (6.6); 1e-4 of it is that at about 3 sigma. The
    # relative L2 bound stays the stated 1e-5.
    assert_parity(got, want, 1e-5, elem=1e-4)


def test_full_c3_forward(gjp, oracle_mod):
    """512^3 / 720 views / 768^2 in FP32, BF16 and FP16; the 16-bit sinograms of
    the two-rays-per-lane tile equal the one-ray tile's bit for bit."""
    _full_config_check(gjp, oracle_mod, "c3", 3000, dtypes=("f32", "bf16", "f16"), pairs=True)


def test_full_t1_forward_clipped(gjp, oracle_mod):
    """The paper's speed geometry (512^3, 512^2 detector, 10 degree cone, 360
    views, sample range clipped to the inscribed cylinder), FP32 and BF16."""
    _full_config_check(gjp, oracle_mod, "t1", 3000, dtypes=("f32", "bf16"))


@pytest.mark.slow
def test_full_c5a_forward_16bit(gjp, oracle_mod):
    _full_config_check(gjp, oracle_mod, "c5a", 2000, dtypes=("bf16", "f16"))


@pytest.mark.slow
def test_full_c5b_forward_2048(gjp, oracle_mod):
    """2048^3 FP32 (34 GB, 64-bit offsets), 64 views, 3072^2 detector, checked on
    sampled rays against the oracle reading the same volume on the host, with
    the default one-ray tile and with three rays per lane (the benchmark's
    configuration)."""
    _full_config_check(gjp, oracle_mod, "c5b", 1500, tiles=[(192, 8, 4)])


def _analytic_sinogram_torch(cfg, G, dev):
    """Exact line integrals of the configuration's ellipsoid phantom through the
    grid box for every ray (chord of each ellipsoid clipped to [-0.5, N-0.5]^3 in
    grid units), in FP64 on the device one group of views at a time. Same
    construction as oracle.phantom.line_integrals, evaluated with torch so the
    full 512^3 / 720-view sinogram stays cheap."""
    import torch
    f64 = torch.float64
    views = torch.from_numpy(G.views).to(dev, f64)
    iu = torch.arange(G.n_u, device=dev, dtype=f64)[:, None, None]
    iv = torch.arange(G.n_v, device=dev, dtype=f64)[None, :, None]
    lo = torch.tensor([-0.5 * s for s in cfg.shape], device=dev, dtype=f64)
    hi = -lo
    out = torch.empty(G.sino_shape, device=dev, dtype=torch.float32)
    ells = [(torch.as_tensor(e.rot(), device=dev, dtype=f64),
             torch.tensor(e.semi_axes, device=dev, dtype=f64),
             torch.tensor(e.center, device=dev, dtype=f64), e.density)
            for e in cfg.phantom_ellipsoids()]
    for v in range(G.n_views):
        V = views[v]
        d = V[3:6] + iu * V[6:9] + iv * V[9:12]          # (n_u, n_v, 3)
        a = V[0:3].expand_as(d)
        u = d - a
        ulen = torch.linalg.vector_norm(u, dim=-1)
        t0 = torch.full(ulen.shape, -torch.inf, device=dev, dtype=f64)
        t1 = torch.full(ulen.shape, torch.inf, device=dev, dtype=f64)
        for k in range(3):
            uk = u[..., k]
            uk = torch.where(uk == 0.0, torch.full_like(uk, 1e-300), uk)  # parallel to a face
            ta = (lo[k] - a[..., k]) / uk
            tb = (hi[k] - a[..., k]) / uk
            t0 = torch.maximum(t0, torch.minimum(ta, tb))
            t1 = torch.minimum(t1, torch.maximum(ta, tb))
        acc = torch.zeros(ulen.shape, device=dev, dtype=f64)
        for R, s, c, rho in ells:
            A = ((a - c) @ R) / s
            B = (u @ R) / s
            qa = (B * B).sum(-1)
            qb = (A * B).sum(-1)
            qc = (A * A).sum(-1) - 1.0
            disc = qb * qb - qa * qc
            sq = torch.sqrt(torch.clamp(disc, min=0.0))
            e1 = torch.maximum((-qb - sq) / qa, t0)
            e2 = torch.minimum((-qb + sq) / qa, t1)
            acc += torch.where(disc > 0, rho * torch.clamp(e2 - e1, min=0.0) * ulen, 0.0)
        out[v] = acc.float()
    return out


def _footprint_rays(og, voxel, margin=2):
    """Every ray (view, iu, iv) that can carry weight on grid voxel `voxel`
    of a cone-beam geometry: a sample weights the voxel only within one voxel
    of it on both transverse axes, so its ray passes through the cube
    [voxel - 1, voxel + 1]^3; the rays through that convex cube hit the
    detector inside the box spanned by its eight corners' projections, taken
    here widened by `margin` pixels."""
    shape = np.asarray(og.shape, dtype=np.float64)
    vs = np.asarray(og.voxel_size, dtype=np.float64)
    ctr = np.asarray(og.center, dtype=np.float64)
    corners = np.array([[voxel[0] + a, voxel[1] + b, voxel[2] + c]
                        for a in (-1, 1) for b in (-1, 1) for c in (-1, 1)], dtype=np.float64)
    world = (corners - 0.5 * (shape - 1.0)) * vs + ctr
    out = []
    for vi, v in enumerate(og.views):
        s, d00, du, dv = v[0:3], v[3:6], v[6:9], v[9:12]
        uv = []
        for p in world:
            # s + t (p - s) = d00 + a du + b dv
            M = np.stack([p - s, -du, -dv], axis=1)
            t, a, b = np.linalg.solve(M, d00 - s)
            uv.append((a, b))
        uv = np.asarray(uv)
        u0 = max(0, int(np.floor(uv[:, 0].min())) - margin)
        u1 = min(og.n_u - 1, int(np.ceil(uv[:, 0].max())) + margin)
        v0 = max(0, int(np.floor(uv[:, 1].min())) - margin)
        v1 = min(og.n_v - 1, int(np.ceil(uv[:, 1].max())) + margin)
        if u0 > u1 or v0 > v1:
            continue
        iu, iv = np.meshgrid(np.arange(u0, u1 + 1), np.arange(v0, v1 + 1), indexing="ij")
        out.append(np.stack([np.full(iu.size, vi), iu.ravel(), iv.ravel()], axis=1))
    return np.concatenate(out).astype(np.int32)


@pytest.mark.slow
@pytest.mark.parametrize("name", ["c3", "t1"])
def test_full_adjoint_sampled_voxels(gjp, oracle_mod, name):
    """Full-size adjoints on 12 sampled voxels against the oracle: c3 (512^3,
    720 views; value table and column gather, as the benchmark runs it) and
    t1 (the paper's speed geometry, clipped to the cylinder; 16-byte ray
    table). (A^T y)[v] = sum over rays of the ray's weight on v times y, the
    weights being the oracle's forward projection of the one-hot volume e_v
    on every ray whose detector footprint can reach v."""
    import torch
    dev = cuda()
    cfg = workloads.config(name)
    G = gjp.Geometry.from_config(cfg)
    og = oracle_mod.geometry_for(cfg)
    gen = torch.Generator(device="cpu").manual_seed(60)
    y = torch.rand(G.sino_shape, generator=gen)
    note(f"{name} adjoint: GPU")
    xb = gjp.back(y.to(dev), G).cpu().numpy()
    y_np = y.numpy()
    rng = np.random.default_rng(61)
    n = cfg.shape
    voxels = [tuple(int(rng.integers(0, n[k])) for k in range(3)) for _ in range(10)]
    voxels += [(0, n[1] // 2, n[2] - 1), (n[0] - 1, 0, 0)]   # grid faces and corners
    onehot = np.zeros(cfg.shape, dtype=np.float32)
    got, want = [], []
    for v in voxels:
        rays = _footprint_rays(og, v)
        onehot[v] = 1.0
        w = oracle_mod.forward_rays(og, onehot, rays)
        onehot[v] = 0.0
        want.append(float(np.dot(w, y_np[rays[:, 0], rays[:, 1], rays[:, 2]].astype(np.float64))))
        got.append(float(xb[v]))
        note(f"{name} adjoint: voxel {v}: {len(rays)} footprint rays, oracle {want[-1]:.6f}, "
             f"GPU {got[-1]:.6f}")
    assert_parity(np.array(got), np.array(want), 1e-5)


@pytest.mark.slow
def test_full_c3_differentiable(gjp, oracle_mod):
    """The differentiable-projector workload at full size: 512^3, 720 views,
    768^2. b = analytic line integrals + Gaussian noise (sigma = 1% of max b);
    loss 0.5 ||Ax - b||^2; the autograd gradient (hand-written A^T) against
    central differences at 64 random voxels; 20 gradient-descent steps with
    alpha = 1/lambda, lambda from 10 power iterations on A^T A; the loss must
    decrease at every step."""
    import time
    import torch
    dev = cuda()
    cfg = workloads.config("c3")
    G = gjp.Geometry.from_config(cfg)
    note("c3 differentiable: analytic sinogram")
    b = _analytic_sinogram_torch(cfg, G, dev)
    # spot-check the device evaluation against the oracle's analytic integrals
    from oracle import phantom
    rays = workloads.sample_rays(53, 400, G.n_views, G.n_u, G.n_v)
    ref = phantom.line_integrals(cfg.phantom_ellipsoids(), oracle_mod.geometry_for(cfg), rays)
    got = b[rays[:, 0], rays[:, 1], rays[:, 2]].double().cpu().numpy()
    assert rel_l2(got, ref) <= 1e-6
    gen = torch.Generator(device="cpu").manual_seed(3)
    b = b + (0.01 * float(b.max())) * torch.randn(G.sino_shape, generator=gen).to(dev)

    def loss_of(z):
        r = gjp.forward(z, G).double() - b.double()
        return 0.5 * float((r * r).sum())

    # gradient at x0 through autograd, against central differences
    x0 = torch.rand(cfg.shape, generator=torch.Generator().manual_seed(30)).to(dev) * 0.1
    x = x0.clone().requires_grad_(True)
    r = gjp.project(x, G) - b
    (0.5 * (r * r).sum()).backward()
    grad = x.grad.double()
    rng = np.random.default_rng(31)
    idx = [tuple(int(t) for t in rng.integers(64, 448, size=3)) for _ in range(64)]
    eps = 1.0
    note("c3 differentiable: finite differences at 64 voxels")
    for v in idx:
        xp = x0.clone()
        xm = x0.clone()
        xp[v] += eps
        xm[v] -= eps
        fd = (loss_of(xp) - loss_of(xm)) / (2 * eps)
        g = float(grad[v])
        # the loss is quadratic: the central difference is exact up to the FP32
        # rounding of the sums (~1e-7 of the loss, over 2 eps)
        assert abs(fd - g) <= 1e-3 * max(abs(g), 1e-2 * float(grad.abs().max())), (v, fd, g)
    # step size from power iterations on A^T A
    note("c3 differentiable: power iterations")
    q = torch.rand(cfg.shape, generator=torch.Generator().manual_seed(32)).to(dev)
    lam = 0.0
    for _ in range(10):
        q = gjp.back(gjp.forward(q, G), G)
        lam = float(torch.linalg.vector_norm(q))
        q = q / lam
    note("c3 differentiable: 20 gradient-descent steps")
    x = torch.zeros(cfg.shape, device=dev, requires_grad=True)
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        x.grad = None
        r = gjp.project(x, G) - b
        L = 0.5 * (r * r).sum()
        L.backward()
        losses.append(float(L))
        with torch.no_grad():
            x -= x.grad / lam
    torch.cuda.synchronize()
    note(f"c3 differentiable: 20 steps in {time.perf_counter() - t0:.2f} s, "
         f"loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert all(l2 < l1 for l1, l2 in zip(losses, losses[1:]))


def test_autotune_cache_on_disk(gjp, tmp_path, monkeypatch):
    """GJP_TUNE_CACHE: the autotuner's choice is written to the file, tagged
    with the device, and read back once this process's own choice is
    forgotten; a shape signature without an entry keeps the default."""
    import torch
    dev = cuda()
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("GJP_TUNE_CACHE", str(path))
    shape = (36, 30, 44)
    G = gjp.Geometry.circular_cone(shape, 9, 50, 70, 150.0, 225.0)
    x = torch.rand(shape, generator=torch.Generator().manual_seed(9)).to(dev)
    note("autotune with on-disk cache")
    tv = gjp.autotune(x, G)
    chosen = gjp.get_forward_tile(G, torch.float32)
    assert chosen[0] == tv
    lines = [l.split() for l in path.read_text().splitlines() if l.strip()]
    assert len(lines) == 1 and lines[0][0].startswith("gfx")
    assert [int(v) for v in lines[0][2:]] == [{64: 6, 32: 5, 16: 4}[tv], chosen[1], chosen[2]]
    gjp.reset_forward_tile(G, torch.float32)
    assert gjp.get_forward_tile(G, torch.float32) == chosen
    # same sizes, another dtype: no entry
    assert gjp.get_forward_tile(G, torch.float16) == (64, 8, 4)
    ref = gjp.forward(x, G)
    gjp.set_forward_tile(G, torch.float32, 64, 8, 4)
    assert torch.equal(gjp.forward(x, G), ref)
