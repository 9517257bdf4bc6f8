"""FP64 SART on top of the oracle projector (test infrastructure only).

The paper reconstructs with SART (Sec. IV-B, Andersen and Kak), which enforces
consistency with each observed projection image in turn through the forward
model A. The relaxation factor, the subset order and the backprojector are not
given; the readings taken here (and by the GPU path) are:

* the views are split into ``n_subsets`` interleaved subsets (subset s holds
  views s, s + n_subsets, ...), visited in a stride order that spreads
  consecutive updates over the circle (``subset_order``);
* one update for subset S:
      x <- x + lam * A_S^T( (b_S - A_S x) / (A_S 1) ) / (A_S^T 1)
  where a zero row sum (A_S 1) or column sum (A_S^T 1) makes that term zero;
* the backprojector is the exact adjoint A^T;
* optional clamping of x to x >= 0 after each update (off by default).

``sart`` is written for any linear operator given as callables, so it can be
pinned on small explicit matrices as well as run with the projector.
"""
from __future__ import annotations

from typing import Callable, Sequence

import numpy as np

import oracle


def subset_order(n_subsets: int):
    """Visit order of the subsets: a golden-ratio stride k * p mod n, p the
    first integer at or above round(0.618 n) coprime with n, so consecutive
    updates use views far apart on the circle."""
    import math
    if n_subsets <= 1:
        return [0]
    p = int(round(n_subsets * 0.6180339887498949))
    while math.gcd(p, n_subsets) != 1:
        p += 1
    return [(k * p) % n_subsets for k in range(n_subsets)]


def sart(forward: Sequence[Callable], adjoint: Sequence[Callable], b: Sequence[np.ndarray],
         x0: np.ndarray, n_iter: int, lam: float = 1.0, nonneg: bool = False,
         order: Sequence[int] | None = None) -> np.ndarray:
    """Generic SART: forward[s](x) = A_s x, adjoint[s](y) = A_s^T y, b[s] the
    data of subset s. Returns x after n_iter passes over all subsets."""
    n = len(forward)
    order = list(range(n)) if order is None else list(order)
    x = np.array(x0, dtype=np.float64, copy=True)
    row = [forward[s](np.ones_like(x)) for s in range(n)]
    col = [adjoint[s](np.ones_like(np.asarray(b[s], dtype=np.float64))) for s in range(n)]
    for _ in range(n_iter):
        for s in order:
            r = np.asarray(b[s], dtype=np.float64) - forward[s](x)
            r = np.where(row[s] > 0, r / np.where(row[s] > 0, row[s], 1.0), 0.0)
            bp = adjoint[s](r)
            x = x + lam * np.where(col[s] > 0, bp / np.where(col[s] > 0, col[s], 1.0), 0.0)
            if nonneg:
                x = np.maximum(x, 0.0)
    return x


def subsets(n_views: int, n_subsets: int):
    return [np.arange(s, n_views, n_subsets) for s in range(n_subsets)]


def sart_projector(g: "oracle.Geometry", b: np.ndarray, n_iter: int, n_subsets: int,
                   lam: float = 1.0, x0: np.ndarray | None = None,
                   nonneg: bool = False) -> np.ndarray:
    """SART with the oracle projector: b has the shape of g's sinogram."""
    import dataclasses
    subs = subsets(g.n_views, n_subsets)
    geoms = [dataclasses.replace(g, views=g.views[idx]) for idx in subs]
    fwd = [lambda x, gs=gs: oracle.forward(gs, x) for gs in geoms]
    adj = [lambda y, gs=gs: oracle.adjoint(gs, y) for gs in geoms]
    bs = [np.asarray(b)[idx] for idx in subs]
    x0 = np.zeros(tuple(g.shape)) if x0 is None else x0
    return sart(fwd, adj, bs, x0, n_iter, lam=lam, nonneg=nonneg,
                order=subset_order(n_subsets))
