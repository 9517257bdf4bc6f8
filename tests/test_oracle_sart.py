"""Pins of the oracle's SART (Sec. IV-B reconstruction; the update, subset
order and relaxation readings are stated in oracle/sart.py).

* hand-derived steps on 2x2 systems (one subset, two subsets);
* the golden-ratio subset order for n = 10 and that it is a permutation;
* with the projector: the true volume is a fixed point for consistent data,
  and iterations reduce the data residual of a consistent problem.
"""
import numpy as np
import pytest

import oracle
from oracle import sart as osart


def _mat_ops(A, rows):
    A = np.asarray(A, dtype=np.float64)
    fwd = [lambda x, r=r: A[r] @ x for r in rows]
    adj = [lambda y, r=r: A[r].T @ y for r in rows]
    return fwd, adj


def test_one_subset_step_by_hand():
    # A = [[2, 0], [1, 1]], b = [4, 3], x0 = 0, lam = 1:
    # row sums (2, 2) -> r = (2, 1.5); A^T r = (5.5, 1.5); column sums (3, 1)
    A = [[2.0, 0.0], [1.0, 1.0]]
    fwd, adj = _mat_ops(A, [np.array([0, 1])])
    x = osart.sart(fwd, adj, [np.array([4.0, 3.0])], np.zeros(2), n_iter=1)
    np.testing.assert_allclose(x, [11.0 / 6.0, 1.5], rtol=0, atol=1e-15)


def test_two_subsets_by_hand():
    # subset 0 = row 0: r = 4/2 = 2, A^T r = (4, 0), column sums (2, 0) -> x = (2, 0)
    # subset 1 = row 1: r = (3 - 2)/2 = 0.5, A^T r = (0.5, 0.5), sums (1, 1) -> (2.5, 0.5)
    A = [[2.0, 0.0], [1.0, 1.0]]
    fwd, adj = _mat_ops(A, [np.array([0]), np.array([1])])
    b = [np.array([4.0]), np.array([3.0])]
    x = osart.sart(fwd, adj, b, np.zeros(2), n_iter=1, order=[0, 1])
    np.testing.assert_allclose(x, [2.5, 0.5], rtol=0, atol=1e-15)
    # relaxation scales the first update; the second sees the relaxed state
    x = osart.sart(fwd, adj, b, np.zeros(2), n_iter=1, lam=0.5, order=[0, 1])
    # (1, 0) then r = (3 - 1)/2 = 1 -> + 0.5 * (1, 1)
    np.testing.assert_allclose(x, [1.5, 0.5], rtol=0, atol=1e-15)


def test_subset_order():
    assert osart.subset_order(10) == [0, 7, 4, 1, 8, 5, 2, 9, 6, 3]
    assert osart.subset_order(1) == [0]
    for n in (2, 3, 12, 45, 360):
        assert sorted(osart.subset_order(n)) == list(range(n))


def _small_problem(seed=5):
    shape = (14, 12, 10)
    views = oracle.views_circular_cone(16, 60.0, 120.0, 1.6, 1.6, 22, 16)
    g = oracle.Geometry(shape, views, 22, 16)
    rng = np.random.default_rng(seed)
    x_true = rng.uniform(0.0, 1.0, size=shape)
    return g, x_true, oracle.forward(g, x_true)


def test_projector_fixed_point():
    g, x_true, b = _small_problem()
    x = osart.sart_projector(g, b, n_iter=1, n_subsets=4, x0=x_true)
    np.testing.assert_allclose(x, x_true, rtol=0, atol=1e-12)


def test_projector_residual_decreases():
    g, x_true, b = _small_problem()
    res = []
    for k in range(4):
        x = osart.sart_projector(g, b, n_iter=k, n_subsets=4)
        res.append(np.linalg.norm(b - oracle.forward(g, x)))
    assert all(r2 < r1 for r1, r2 in zip(res, res[1:]))
    assert res[-1] < 0.3 * res[0]
