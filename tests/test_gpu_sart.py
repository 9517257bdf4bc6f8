"""GPU SART (Sec. IV-B reconstruction) against the oracle's FP64 SART, and the
C-ABI elementwise steps against numpy.

Tolerance: each subset update applies the FP32 forward and adjoint (each
within 1e-5 relative L2 of FP64) and two elementwise steps; the update is a
relaxed projection (non-expansive for 0 < lam < 2), so the deviations add up
at most linearly over the updates: 12 updates x (2 x 1e-5) < 3e-4. The bound
used is 3e-4.
"""
import ctypes

import numpy as np
import pytest

import workloads
from gpu_helpers import cuda, note, rel_l2

pytestmark = pytest.mark.gpu

TOL_SART = 3e-4


@pytest.fixture(scope="module")
def gjp():
    import paper_1609_00958_amd as m
    return m


def _problem(oracle_mod, clip=False):
    shape = (26, 22, 18)
    cfg = workloads.WorkloadConfig("s", shape, 16, 34, 24, beam="cone", sod=90.0, sdd=180.0,
                                   pitch_u=1.5, pitch_v=1.5, clip_cylinder=clip)
    og = oracle_mod.geometry_for(cfg)
    x_true = workloads.rasterize(workloads.random_ellipsoids(97, shape), shape)
    b = oracle_mod.forward(og, x_true).astype(np.float32)
    return cfg, og, b


@pytest.mark.parametrize("n_subsets,lam,nonneg,n_iter,clip",
                         [(4, 0.9, False, 3, False), (16, 1.0, True, 1, False),
                          (4, 1.0, False, 2, True)])
def test_sart_matches_oracle(gjp, oracle_mod, n_subsets, lam, nonneg, n_iter, clip):
    import torch
    from oracle import sart as osart
    dev = cuda()
    cfg, og, b = _problem(oracle_mod, clip)
    G = gjp.Geometry.from_config(cfg)
    note(f"sart subsets={n_subsets} lam={lam} nonneg={nonneg} clip={clip}")
    x = gjp.sart(G, torch.from_numpy(b).to(dev), n_iter, n_subsets, lam=lam,
                 nonneg=nonneg).cpu().numpy()
    want = osart.sart_projector(og, b.astype(np.float64), n_iter, n_subsets, lam=lam,
                                nonneg=nonneg)
    assert rel_l2(x, want) <= TOL_SART
    if nonneg:
        assert x.min() >= 0.0


def test_sart_parallel_beam(gjp, oracle_mod):
    import torch
    from oracle import sart as osart
    dev = cuda()
    shape = (24, 24, 12)
    cfg = workloads.WorkloadConfig("p", shape, 18, 30, 14, beam="parallel", pitch_u=0.9,
                                   pitch_v=1.0)
    og = oracle_mod.geometry_for(cfg)
    x_true = workloads.rasterize(workloads.random_ellipsoids(96, shape), shape)
    b = oracle_mod.forward(og, x_true).astype(np.float32)
    G = gjp.Geometry.from_config(cfg)
    note("sart parallel")
    x = gjp.sart(G, torch.from_numpy(b).to(dev), 2, 6, lam=0.8).cpu().numpy()
    want = osart.sart_projector(og, b.astype(np.float64), 2, 6, lam=0.8)
    assert rel_l2(x, want) <= TOL_SART


def test_sart_reduces_residual(gjp, oracle_mod):
    import torch
    dev = cuda()
    cfg, og, b = _problem(oracle_mod)
    G = gjp.Geometry.from_config(cfg)
    bd = torch.from_numpy(b).to(dev)
    s = gjp.SART(G, 4)
    res = []
    x = None
    for _ in range(3):
        x = s.run(bd, 1, x0=x)
        res.append(float(torch.linalg.vector_norm(bd - gjp.forward(x, G))))
    assert res[1] < res[0] and res[2] < res[1]


def test_sart_elementwise_steps(gjp):
    import torch
    from paper_1609_00958_amd import _lib
    dev = cuda()
    rng = np.random.default_rng(98)
    n = 100003
    b = rng.normal(size=n).astype(np.float32)
    ax = rng.normal(size=n).astype(np.float32)
    w = rng.uniform(0.0, 2.0, size=n).astype(np.float32)
    w[::7] = 0.0
    tb, tax, tw = (torch.from_numpy(a).to(dev) for a in (b, ax, w))
    out = torch.empty_like(tax)
    L = _lib.lib()
    stream = int(torch.cuda.current_stream().cuda_stream)
    _lib.check(L.gjp_sart_residual(n, tb.data_ptr(), tax.data_ptr(), tw.data_ptr(),
                                   out.data_ptr(), stream))
    want = np.where(w > 0, (b - ax) / np.where(w > 0, w, np.float32(1)), np.float32(0))
    assert np.array_equal(out.cpu().numpy(), want.astype(np.float32))
    x = rng.normal(size=n).astype(np.float32)
    bp = rng.normal(size=n).astype(np.float32)
    c = rng.uniform(0.0, 3.0, size=n).astype(np.float32)
    c[::5] = 0.0
    tx, tbp, tc = (torch.from_numpy(a).to(dev) for a in (x, bp, c))
    lam = np.float32(0.7)
    _lib.check(L.gjp_sart_update(n, tx.data_ptr(), tbp.data_ptr(), tc.data_ptr(), float(lam), 1,
                                 stream))
    upd = np.where(c > 0, x + (lam * bp) / np.where(c > 0, c, np.float32(1)), x)
    want = np.maximum(upd.astype(np.float32), np.float32(0))
    assert np.array_equal(tx.cpu().numpy(), want)
    # argument errors are reported before any launch
    assert L.gjp_sart_update(-1, None, None, None, 1.0, 0, None) == _lib.GJP_EINVAL
    assert L.gjp_sart_residual(5, None, None, None, None, None) == _lib.GJP_EINVAL
