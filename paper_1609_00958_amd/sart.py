"""SART reconstruction (Sec. IV-B, after Andersen and Kak) on the library's
forward projector and its exact adjoint.

For a subset S of the views one update is
    x <- x + lam * A_S^T( (b_S - A_S x) / (A_S 1) ) / (A_S^T 1)
with zero row or column sums giving zero terms. The views are split into
interleaved subsets (subset s holds views s, s + n_subsets, ...), visited in a
golden-ratio stride order; each iteration visits every subset once. The
projections and both elementwise steps run in the library's kernels
(gjp_forward_project, gjp_back_project, gjp_sart_residual, gjp_sart_update);
this module only schedules them. The per-subset row and column sums are
computed once (A_S 1 and A_S^T 1) and kept on the device: memory is one
sinogram plus n_subsets volumes in FP32.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from ._lib import check, lib
from .projector import Geometry, back, forward


def visit_order(n: int):
    """k * p mod n with p the first integer >= round(0.618 n) coprime to n."""
    if n <= 1:
        return [0]
    p = int(round(n * (math.sqrt(5.0) - 1.0) / 2.0))
    while math.gcd(p, n) != 1:
        p += 1
    return [(k * p) % n for k in range(n)]


class SART:
    def __init__(self, geom: Geometry, n_subsets: int, lam: float = 1.0,
                 nonneg: bool = False, device=None):
        import torch
        if not 1 <= n_subsets <= geom.n_views:
            raise ValueError("n_subsets must lie in [1, n_views]")
        self.geom = geom
        self.lam = float(lam)
        self.nonneg = bool(nonneg)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.subsets = [np.arange(s, geom.n_views, n_subsets) for s in range(n_subsets)]
        self.order = visit_order(n_subsets)
        self.geoms = [Geometry(geom.shape, geom.views[idx], geom.n_u, geom.n_v,
                               beam=geom.beam, voxel_size=geom.voxel_size, center=geom.center,
                               weight=geom.weight, clip_cylinder=geom.clip_cylinder)
                      for idx in self.subsets]
        ones_v = torch.ones(geom.shape, dtype=torch.float32, device=self.device)
        self.row = [forward(ones_v, g) for g in self.geoms]
        self.col = []
        for g in self.geoms:
            ones_s = torch.ones(g.sino_shape, dtype=torch.float32, device=self.device)
            self.col.append(back(ones_s, g))
        self._idx = [torch.from_numpy(idx).to(self.device) for idx in self.subsets]

    def run(self, b, n_iter: int, x0: Optional[object] = None):
        """n_iter SART iterations from x0 (zeros if None); b is the full
        sinogram (n_views, n_u, n_v), float32 on the device."""
        import torch
        if tuple(b.shape) != self.geom.sino_shape or b.dtype != torch.float32:
            raise ValueError("b must be a float32 sinogram of the geometry")
        x = torch.zeros(self.geom.shape, dtype=torch.float32, device=self.device) \
            if x0 is None else x0.detach().to(self.device, torch.float32).clone()
        bs = [b.index_select(0, i).contiguous() for i in self._idx]
        L = lib()
        stream = int(torch.cuda.current_stream(self.device).cuda_stream)
        nvox = x.numel()
        for _ in range(int(n_iter)):
            for s in self.order:
                g = self.geoms[s]
                ax = forward(x, g)
                check(L.gjp_sart_residual(ax.numel(), bs[s].data_ptr(), ax.data_ptr(),
                                          self.row[s].data_ptr(), ax.data_ptr(), stream))
                bp = back(ax, g)
                check(L.gjp_sart_update(nvox, x.data_ptr(), bp.data_ptr(),
                                        self.col[s].data_ptr(), self.lam,
                                        1 if self.nonneg else 0, stream))
        return x


def sart(geom: Geometry, b, n_iter: int, n_subsets: int, lam: float = 1.0, x0=None,
         nonneg: bool = False):
    """SART reconstruction of b (see SART)."""
    return SART(geom, n_subsets, lam=lam, nonneg=nonneg, device=b.device).run(b, n_iter, x0)
