"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names what it pins. Together they are chosen so that a plausible
mistake anywhere in the oracle (a dropped neighbour, a swapped floor/ceil
weight, an off-by-half grid convention, a wrong step length, a wrong sample
range, a wrong boundary reading, a non-transposed adjoint) fails one of them.
"""
import math
import os

import numpy as np
import pytest

from conftest import grid_point, parallel_rays_views

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _one_ray(oracle_mod, shape, s_grid, r, weight=0):
    views = parallel_rays_views(shape, r, s_grid, (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))
    return oracle_mod.Geometry(tuple(shape), views, 1, 1, beam=oracle_mod.PARALLEL,
                               weight=weight)


# ---------------------------------------------------------------------------
# P1: single-voxel responses derived by hand (tests/golden/single_voxel.txt,
# Eqs. 10-14). Pins the neighbour set, the weight formulas and ||r~||.
# ---------------------------------------------------------------------------
def _golden_cases():
    rows = []
    with open(os.path.join(GOLDEN, "single_voxel.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            w = int(tok[0])
            s = [float(x) for x in tok[1:4]]
            r = [float(x) for x in tok[4:7]]
            v = [int(x) for x in tok[7:10]]
            expr = " ".join(tok[10:])
            rows.append((w, s, r, v, expr))
    return rows


@pytest.mark.parametrize("case", _golden_cases())
def test_single_voxel_golden(oracle_mod, case):
    w, s, r, v, expr = case
    shape = (8, 8, 8)
    g = _one_ray(oracle_mod, shape, s, r, weight=w)
    vol = np.zeros(shape)
    vol[tuple(v)] = 1.0
    got = oracle_mod.forward(g, vol)[0, 0, 0]
    want = eval(expr, {"sqrt": math.sqrt})
    assert got == pytest.approx(want, abs=1e-14, rel=1e-14)


# ---------------------------------------------------------------------------
# P2: rays parallel to a grid axis. Through voxel centres the projection is the
# column sum; at a fractional offset it is the bilinear blend of the four
# neighbouring column sums (textbook bilinear interpolation). Every driving
# axis, pins the sample range 0..N_m-1 and the indexing.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("frac", [(0.0, 0.0), (0.3, 0.7), (0.5, 0.25)])
def test_axis_aligned_columns(oracle_mod, axis, frac):
    shape = (7, 9, 11)
    rng = np.random.default_rng(10 + axis)
    vol = rng.uniform(-1, 1, size=shape)
    others = [k for k in range(3) if k != axis]
    a0, b0 = 2, 3
    fa, fb = frac
    s = [0.0, 0.0, 0.0]
    s[axis] = 0.0
    s[others[0]] = a0 + fa
    s[others[1]] = b0 + fb
    r = [0.0, 0.0, 0.0]
    r[axis] = -1.0 if axis == 1 else 1.0
    g = _one_ray(oracle_mod, shape, s, r)
    got = oracle_mod.forward(g, vol)[0, 0, 0]
    col = vol.sum(axis=axis)  # 2-D over the two other axes, in increasing axis order
    want = ((1 - fa) * (1 - fb) * col[a0, b0] + (1 - fa) * fb * col[a0, b0 + 1]
            + fa * (1 - fb) * col[a0 + 1, b0] + fa * fb * col[a0 + 1, b0 + 1])
    assert got == pytest.approx(want, rel=1e-13, abs=1e-13)


# ---------------------------------------------------------------------------
# P3: a box of ones. For rays that enter and leave through the driving-axis
# faces and keep all four neighbours inside the box on every plane it spans,
# the projection equals the exact chord through [lo-0.5, hi+0.5] (the grid
# convention: voxel k is centred at coordinate k). Pins the step length
# ||r~||, the box extent and the sample count.
# ---------------------------------------------------------------------------
def test_constant_box_chord(oracle_mod):
    shape = (24, 24, 24)
    lo, hi = 6, 17
    vol = np.zeros(shape)
    vol[lo:hi + 1, lo:hi + 1, lo:hi + 1] = 1.0
    rng = np.random.default_rng(3)
    n_checked = 0
    for _ in range(60):
        gy, gz = rng.uniform(-0.25, 0.25, size=2)
        y0, z0 = rng.uniform(lo + 3.0, hi - 3.0, size=2)   # position at the box centre plane
        xc = 0.5 * (lo + hi)
        # keep transverse coordinates within [lo, hi] on planes lo..hi
        ys = y0 + (np.array([lo, hi]) - xc) * gy
        zs = z0 + (np.array([lo, hi]) - xc) * gz
        if ys.min() < lo or ys.max() > hi or zs.min() < lo or zs.max() > hi:
            continue
        s = [xc, y0, z0]
        g = _one_ray(oracle_mod, shape, s, [1.0, gy, gz])
        got = oracle_mod.forward(g, vol)[0, 0, 0]
        # exact chord of the line through the extended box (slab method)
        d = np.array([1.0, gy, gz])
        p0 = np.array(s)
        t_lo, t_hi = -np.inf, np.inf
        for k in range(3):
            ta = (lo - 0.5 - p0[k]) / d[k] if d[k] != 0 else -np.inf
            tb = (hi + 0.5 - p0[k]) / d[k] if d[k] != 0 else np.inf
            t_lo = max(t_lo, min(ta, tb))
            t_hi = min(t_hi, max(ta, tb))
        want = (t_hi - t_lo) * np.linalg.norm(d)
        assert got == pytest.approx(want, rel=1e-13)
        n_checked += 1
    assert n_checked > 20


# ---------------------------------------------------------------------------
# P4: an affine field f(x) = alpha + beta . x. Bilinear interpolation of an
# affine field is exact and the unit-step sum over planes 0..N-1 is the
# midpoint rule on [-0.5, N-0.5], exact for affine integrands, so the
# projection is the exact line integral over the chord. An off-by-half in the
# sample positions shows up at first order.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_affine_field_line_integral(oracle_mod, axis):
    shape = (12, 14, 16)
    alpha = 0.7
    beta = np.array([0.11, -0.23, 0.05])
    idx = np.indices(shape).astype(np.float64)
    vol = alpha + beta[0] * idx[0] + beta[1] * idx[1] + beta[2] * idx[2]
    rng = np.random.default_rng(4 + axis)
    N = shape[axis]
    others = [k for k in range(3) if k != axis]
    for _ in range(10):
        g_ = rng.uniform(-0.2, 0.2, size=2)
        d = np.zeros(3)
        d[axis] = 1.0
        d[others[0]], d[others[1]] = g_
        mid = np.zeros(3)
        mid[axis] = 0.5 * (N - 1)
        for j, k in enumerate(others):
            mid[k] = 0.5 * (shape[k] - 1) + rng.uniform(-1.0, 1.0)
        # all samples stay within [0, N_k - 1] on the transverse axes
        for j, k in enumerate(others):
            ends = mid[k] + np.array([-0.5 * (N - 1), 0.5 * (N - 1)]) * d[k]
            assert ends.min() >= 0 and ends.max() <= shape[k] - 1
        g = _one_ray(oracle_mod, shape, mid, d)
        got = oracle_mod.forward(g, vol)[0, 0, 0]
        f_mid = alpha + float(beta @ mid)
        want = np.linalg.norm(d) * N * f_mid   # integral of an affine f over the chord
        assert got == pytest.approx(want, rel=1e-12)


# ---------------------------------------------------------------------------
# P5: lattice mass conservation. Parallel rays whose hit points on every
# sampling plane form a unit lattice covering (-1, N): each voxel's weights
# over the lattice sum to one for any w with w(1-d) = 1 - w(d) (Eq. 9), so
# sum_rays (A x) = ||r~|| sum_v x_v. Pins Eq. 9/11, the zero-padded reading of
# "in volume" and the step length, for both weight functions.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("weight", [0, 1])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_lattice_mass_conservation(oracle_mod, weight, axis):
    shape = (10, 12, 9)
    rng = np.random.default_rng(20 + axis + 3 * weight)
    vol = rng.uniform(0.0, 1.0, size=shape)
    others = [k for k in range(3) if k != axis]
    gsl = rng.uniform(-0.6, 0.6, size=2)
    d = np.zeros(3)
    d[axis] = 1.0
    d[others[0]], d[others[1]] = gsl
    N = shape[axis]
    # lattice offsets: cover (-1, N_k) on every plane; extra rays only sample zeros
    span = [int(math.ceil(abs(gsl[j]) * N)) + 3 for j in range(2)]
    off = rng.uniform(0.0, 1.0, size=2)
    n_a = shape[others[0]] + 2 * span[0]
    n_b = shape[others[1]] + 2 * span[1]
    det00 = np.zeros(3)
    det00[axis] = 0.0
    det00[others[0]] = -span[0] + off[0]
    det00[others[1]] = -span[1] + off[1]
    du = np.zeros(3)
    du[others[0]] = 1.0
    dv = np.zeros(3)
    dv[others[1]] = 1.0
    views = parallel_rays_views(shape, d, det00, du, dv)
    g = oracle_mod.Geometry(shape, views, n_a, n_b, beam=oracle_mod.PARALLEL, weight=weight)
    total = oracle_mod.forward(g, vol).sum()
    want = np.linalg.norm(d) * vol.sum()
    assert total == pytest.approx(want, rel=1e-12)


# ---------------------------------------------------------------------------
# P6: equality with a library trilinear interpolator. On integer planes of the
# driving axis, the four-neighbour weights are the zero-padded trilinear
# interpolant T, so A x = ||r~|| sum_{i=0}^{N_m-1} T(p_i), with T taken from
# scipy's RegularGridInterpolator on a zero-padded copy of the grid.
# ---------------------------------------------------------------------------
def test_matches_scipy_trilinear(oracle_mod):
    from scipy.interpolate import RegularGridInterpolator
    shape = (9, 10, 11)
    rng = np.random.default_rng(5)
    vol = rng.uniform(-1, 1, size=shape)
    pad = np.pad(vol, 1)
    axes = [np.arange(-1, shape[k] + 1, dtype=np.float64) for k in range(3)]
    T = RegularGridInterpolator(axes, pad, method="linear", bounds_error=False, fill_value=0.0)
    n_views, n_u, n_v = 6, 7, 5
    import workloads
    views = workloads.random_cone_views(7, n_views, shape, n_u, n_v)
    g = oracle_mod.Geometry(shape, views, n_u, n_v, beam=oracle_mod.CONE)
    got = oracle_mod.forward(g, vol)
    want = np.zeros_like(got)
    ctr = 0.5 * (np.asarray(shape) - 1.0)
    for v in range(n_views):
        src = views[v, 0:3] + ctr
        for iu in range(n_u):
            for iv in range(n_v):
                d = views[v, 3:6] + ctr + iu * views[v, 6:9] + iv * views[v, 9:12]
                r = d - src
                m = int(np.argmax(np.abs(r)))
                rt = r / r[m]
                i = np.arange(shape[m], dtype=np.float64)
                P = src[None, :] + (i[:, None] - src[m]) * rt[None, :]
                P[:, m] = i
                want[v, iu, iv] = np.linalg.norm(rt) * T(P).sum()
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
    assert np.abs(want).max() > 1.0


# ---------------------------------------------------------------------------
# P7: brute force on tiny grids: build A column by column from one-hot
# volumes and A^T column by column from one-hot sinograms; they must be
# transposes entry by entry. Covers cone and parallel beams, both weights,
# and every driving axis (random orientations).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("beam", [0, 1])
@pytest.mark.parametrize("weight", [0, 1])
def test_brute_force_transpose(oracle_mod, beam, weight):
    import workloads
    shape = (4, 5, 3)
    n_views, n_u, n_v = 3, 4, 3
    if beam == 0:
        views = workloads.random_cone_views(11 + weight, n_views, shape, n_u, n_v)
    else:
        views = workloads.random_parallel_views(11 + weight, n_views, shape, n_u, n_v)
    g = oracle_mod.Geometry(shape, views, n_u, n_v, beam=beam, weight=weight)
    nvox = int(np.prod(shape))
    nray = n_views * n_u * n_v
    A = np.zeros((nray, nvox))
    for j in range(nvox):
        e = np.zeros(nvox)
        e[j] = 1.0
        A[:, j] = oracle_mod.forward(g, e.reshape(shape)).reshape(-1)
    AT = np.zeros((nvox, nray))
    for j in range(nray):
        e = np.zeros(nray)
        e[j] = 1.0
        AT[:, j] = oracle_mod.adjoint(g, e.reshape(n_views, n_u, n_v)).reshape(-1)
    np.testing.assert_allclose(AT, A.T, rtol=0, atol=1e-14)
    assert np.count_nonzero(A) > 20
    # all three driving axes occur across the random views
    axes = {oracle_mod.ray_info(g, v, iu, iv)[0] for v in range(n_views) for iu in range(n_u)
            for iv in range(n_v)}
    assert axes <= {0, 1, 2}


def test_every_driving_axis_occurs(oracle_mod):
    import workloads
    shape = (6, 6, 6)
    views = workloads.random_cone_views(99, 40, shape, 3, 3)
    g = oracle_mod.Geometry(shape, views, 3, 3)
    axes = {oracle_mod.ray_info(g, v, 1, 1)[0] for v in range(40)}
    assert axes == {0, 1, 2}


# ---------------------------------------------------------------------------
# P7b: fine-step quadrature of the trilinear interpolant along the ray agrees
# with the GJP sum for a smooth field (the GJP is a unit-step quadrature of the
# same interpolant), converging as the grid is refined.
# ---------------------------------------------------------------------------
def test_fine_quadrature_smooth_field(oracle_mod):
    from scipy.interpolate import RegularGridInterpolator
    errs = []
    for N in (16, 32):
        shape = (N, N, N)
        idx = (np.indices(shape) - 0.5 * (N - 1)) / N
        vol = np.exp(-((idx ** 2).sum(0)) / (2 * 0.15 ** 2))
        pad = np.pad(vol, 1)
        axes = [np.arange(-1, N + 1, dtype=np.float64)] * 3
        T = RegularGridInterpolator(axes, pad, method="linear", bounds_error=False,
                                    fill_value=0.0)
        rng = np.random.default_rng(6)
        rel = []
        for _ in range(8):
            gsl = rng.uniform(-0.5, 0.5, size=2)
            dvec = np.array([1.0, gsl[0], gsl[1]])
            mid = np.array([0.5 * (N - 1), 0.5 * (N - 1) + rng.uniform(-0.1, 0.1) * N,
                            0.5 * (N - 1) + rng.uniform(-0.1, 0.1) * N])
            g = _one_ray(oracle_mod, shape, mid, dvec)
            got = oracle_mod.forward(g, vol)[0, 0, 0]
            t = np.linspace(-N, N, 40001)
            P = mid[None, :] + t[:, None] * dvec[None, :]
            quad = np.trapezoid(T(P), t) * np.linalg.norm(dvec)
            rel.append(abs(got - quad) / quad)
        errs.append(max(rel))
    assert errs[0] < 0.02
    assert errs[1] < errs[0]


# ---------------------------------------------------------------------------
# P8: convergence to the analytic line integrals of a rasterised ellipsoid
# phantom (the paper's quality benchmark, Sec. IV-A): first-order convergence
# under grid refinement, chords clipped to the grid box.
# ---------------------------------------------------------------------------
def test_analytic_ellipsoid_convergence(oracle_mod):
    import workloads
    from oracle import phantom
    errs = []
    for N in (32, 64, 128):
        shape = (N, N, N)
        ells = workloads.random_ellipsoids(12, shape, n=12)
        vol = workloads.rasterize(ells, shape, dtype=np.float64)
        n_det = int(1.5 * N)
        views = oracle_mod.views_circular_cone(8, 4.0 * N, 6.0 * N, 1.0, 1.0, n_det, n_det)
        g = oracle_mod.Geometry(shape, views, n_det, n_det)
        rays = workloads.sample_rays(1, 3000, 8, n_det, n_det)
        got = oracle_mod.forward_rays(g, vol, rays)
        want = phantom.line_integrals(ells, g, rays, clip=True)
        errs.append(np.linalg.norm(got - want) / np.linalg.norm(want))
    assert errs[1] <= 0.10
    assert errs[1] / errs[0] <= 0.7
    assert errs[2] / errs[1] <= 0.7


# ---------------------------------------------------------------------------
# P9 / P10: the adjoint. The dot-product identity <Ax, y> = <x, A^T y>, and
# central differences of L(x) = 0.5 ||Ax - b||^2 (exact for a quadratic up to
# rounding) against the gradient A^T (Ax - b), on cone and parallel beams.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("beam", [0, 1])
def test_dot_product_identity(oracle_mod, beam):
    import workloads
    shape = (14, 12, 10)
    n_views, n_u, n_v = 5, 16, 13
    if beam == 0:
        views = workloads.random_cone_views(21, n_views, shape, n_u, n_v)
    else:
        views = workloads.random_parallel_views(21, n_views, shape, n_u, n_v)
    g = oracle_mod.Geometry(shape, views, n_u, n_v, beam=beam)
    rng = np.random.default_rng(22)
    for y_kind in ("uniform", "normal"):
        x = rng.uniform(0, 1, size=shape)
        y = (rng.uniform(0, 1, size=(n_views, n_u, n_v)) if y_kind == "uniform"
             else rng.normal(size=(n_views, n_u, n_v)))
        lhs = float((oracle_mod.forward(g, x) * y).sum())
        rhs = float((x * oracle_mod.adjoint(g, y)).sum())
        assert lhs == pytest.approx(rhs, rel=1e-13)


def test_finite_differences_of_quadratic_loss(oracle_mod):
    import workloads
    shape = (10, 10, 10)
    n_views, n_u, n_v = 4, 14, 14
    views = workloads.random_cone_views(31, n_views, shape, n_u, n_v)
    g = oracle_mod.Geometry(shape, views, n_u, n_v)
    rng = np.random.default_rng(32)
    x = rng.uniform(0, 1, size=shape)
    b = rng.uniform(0, 5, size=(n_views, n_u, n_v))

    def loss(z):
        r = oracle_mod.forward(g, z) - b
        return 0.5 * float((r * r).sum())

    grad = oracle_mod.adjoint(g, oracle_mod.forward(g, x) - b)
    eps = 0.5
    for flat in rng.choice(x.size, size=12, replace=False):
        e = np.zeros(x.size)
        e[flat] = eps
        e = e.reshape(shape)
        fd = (loss(x + e) - loss(x - e)) / (2 * eps)
        assert fd == pytest.approx(grad.reshape(-1)[flat], rel=1e-9, abs=1e-9)


# ---------------------------------------------------------------------------
# P11 / P12: a 90-degree rotation about the rotation axis (an index
# permutation of the volume, an exact component swap of the view vectors)
# leaves the projections unchanged; the operator is linear.
# ---------------------------------------------------------------------------
def test_rotation_by_90_degrees(oracle_mod):
    import workloads
    N = 12
    shape = (N, N, 9)
    n_views, n_u, n_v = 4, 15, 11
    views = workloads.random_cone_views(41, n_views, shape, n_u, n_v)
    rng = np.random.default_rng(42)
    vol = rng.uniform(0, 1, size=shape)
    # rotation (x, y, z) -> (-y, x, z) about the grid centre
    rot = np.empty_like(vol)
    for a in range(N):
        for b in range(N):
            rot[a, b] = vol[b, N - 1 - a]
    rv = views.copy()
    for j in range(4):
        x, y = views[:, 3 * j].copy(), views[:, 3 * j + 1].copy()
        rv[:, 3 * j], rv[:, 3 * j + 1] = -y, x
    g0 = oracle_mod.Geometry(shape, views, n_u, n_v)
    g1 = oracle_mod.Geometry(shape, rv, n_u, n_v)
    np.testing.assert_allclose(oracle_mod.forward(g1, rot), oracle_mod.forward(g0, vol),
                               rtol=1e-11, atol=1e-11)


def test_linearity(oracle_mod):
    import workloads
    shape = (9, 8, 7)
    views = workloads.random_cone_views(51, 3, shape, 9, 8)
    g = oracle_mod.Geometry(shape, views, 9, 8)
    rng = np.random.default_rng(52)
    x, z = rng.normal(size=shape), rng.normal(size=shape)
    lhs = oracle_mod.forward(g, 2.5 * x - 0.75 * z)
    rhs = 2.5 * oracle_mod.forward(g, x) - 0.75 * oracle_mod.forward(g, z)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# Special cases of the setup step (Eq. 3 ties, degenerate rays, rays that miss
# the grid) and the sample count.
# ---------------------------------------------------------------------------
def test_argmax_tie_goes_to_lowest_axis(oracle_mod):
    shape = (8, 8, 8)
    g = _one_ray(oracle_mod, shape, [3.5, 3.5, 3.5], [1.0, -1.0, 0.5])
    assert oracle_mod.ray_info(g, 0, 0, 0)[0] == 0
    g = _one_ray(oracle_mod, shape, [3.5, 3.5, 3.5], [0.25, -1.0, 1.0])
    assert oracle_mod.ray_info(g, 0, 0, 0)[0] == 1
    g = _one_ray(oracle_mod, shape, [3.5, 3.5, 3.5], [1.0, 1.0, 1.0])
    assert oracle_mod.ray_info(g, 0, 0, 0)[0] == 0


def test_degenerate_and_missing_rays(oracle_mod):
    shape = (6, 6, 6)
    vol = np.ones(shape)
    # cone beam with the source exactly on the only pixel: r = 0 -> value 0
    views = np.zeros((1, 12))
    views[0, 0:3] = [0.25, 0.5, -0.75]
    views[0, 3:6] = [0.25, 0.5, -0.75]
    views[0, 6:9] = [1.0, 0.0, 0.0]
    views[0, 9:12] = [0.0, 1.0, 0.0]
    g = oracle_mod.Geometry(shape, views, 1, 1)
    assert oracle_mod.forward(g, vol)[0, 0, 0] == 0.0
    assert oracle_mod.ray_info(g, 0, 0, 0)[0] == -1
    # a ray passing beside the grid
    g = _one_ray(oracle_mod, shape, [0.0, 7.5, 2.0], [1.0, 0.0, 0.0])
    assert oracle_mod.forward(g, vol)[0, 0, 0] == 0.0
    assert oracle_mod.count_samples(g) == 0


def test_sample_count_axis_aligned(oracle_mod):
    # n_u x n_v axis-parallel rays at transverse positions inside (-1, N):
    # every ray has exactly N_m samples; rays outside have none.
    shape = (6, 7, 8)
    views = parallel_rays_views(shape, (1.0, 0.0, 0.0), (0.0, -1.5, -1.25), (0, 1.0, 0),
                                (0, 0, 1.0))
    n_u, n_v = 10, 11  # y from -1.5 .. 7.5, z from -1.25 .. 8.75
    g = oracle_mod.Geometry(shape, views, n_u, n_v, beam=oracle_mod.PARALLEL)
    ys = -1.5 + np.arange(n_u)
    zs = -1.25 + np.arange(n_v)
    inside = ((ys > -1) & (ys < shape[1])).sum() * ((zs > -1) & (zs < shape[2])).sum()
    assert oracle_mod.count_samples(g) == inside * shape[0]
