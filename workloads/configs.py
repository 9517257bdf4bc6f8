"""The five workload configurations, described by their parameters.

All cone-beam configurations use a circular trajectory about the third
(fastest) grid axis with unit voxels and the grid centred at the origin.
Where a configuration does not fix a distance or pitch, the choice below is
a stated reading: source-to-centre distance 4N, source-to-detector 1.5x that
(magnification 1.5), detector pitch 1 voxel.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class WorkloadConfig:
    name: str
    shape: tuple
    n_views: int
    n_u: int
    n_v: int
    beam: str = "cone"           # "cone" | "parallel"
    sod: float = 0.0             # source to rotation axis (cone)
    sdd: float = 0.0             # source to detector (cone)
    pitch_u: float = 1.0
    pitch_v: float = 1.0
    phantom: str = "random"      # "sl" | "random"
    phantom_seed: int = 0
    n_ellipsoids: int = 12
    note: str = ""
    clip_cylinder: bool = False  # sample range clipped to the inscribed cylinder

    def phantom_ellipsoids(self):
        from .phantoms import random_ellipsoids, sl_stand_in
        if self.phantom == "sl":
            return sl_stand_in(self.shape)
        return random_ellipsoids(self.phantom_seed, self.shape, n=self.n_ellipsoids)

    @property
    def n_rays(self) -> int:
        return self.n_views * self.n_u * self.n_v


def _cone(name, n, n_views, n_det, phantom, seed, note=""):
    sod = 4.0 * n
    return WorkloadConfig(name=name, shape=(n, n, n), n_views=n_views, n_u=n_det, n_v=n_det,
                          beam="cone", sod=sod, sdd=1.5 * sod, pitch_u=1.0, pitch_v=1.0,
                          phantom=phantom, phantom_seed=seed, note=note)


CONFIGS = {
    # 64^3 stand-in phantom, 64 views, 64x64 detector, SOD 256 / SDD 512; pitch 2 so
    # that the 64-pixel detector covers the grid magnified by 2.
    "c1": WorkloadConfig(name="c1", shape=(64, 64, 64), n_views=64, n_u=64, n_v=64,
                         beam="cone", sod=256.0, sdd=512.0, pitch_u=2.0, pitch_v=2.0,
                         phantom="sl", note="plain FP32 forward; oracle-sized"),
    "c2": _cone("c2", 256, 360, 384, "random", 2, "FP32 forward + adjoint; dot test"),
    # The paper's speed geometry (Sec. IV-C, Table I): 512^3 box, sample range
    # clipped to the inscribed cylinder, 512^2 detector, 10 degree cone (the
    # detector half-width subtends 5 degrees: SOD = 256 / tan 5deg voxels at
    # magnification 2 with pitch 2, i.e. one voxel per pixel at the axis),
    # 360 views, FP32.
    "t1": WorkloadConfig(name="t1", shape=(512, 512, 512), n_views=360, n_u=512, n_v=512,
                         beam="cone", sod=256.0 / math.tan(math.radians(5.0)),
                         sdd=2.0 * 256.0 / math.tan(math.radians(5.0)), pitch_u=2.0,
                         pitch_v=2.0, phantom="sl", clip_cylinder=True,
                         note="paper's projection-speed geometry"),
    "c3": _cone("c3", 512, 720, 768, "sl", 0, "differentiable projector, 20 GD steps"),
    "c5a": _cone("c5a", 1024, 1440, 1536, "random", 5, "BF16/FP16 storage"),
    "c5b": WorkloadConfig(name="c5b", shape=(2048, 2048, 2048), n_views=64, n_u=3072, n_v=3072,
                          beam="cone", sod=8192.0, sdd=12288.0, pitch_u=1.0, pitch_v=1.0,
                          phantom="random", phantom_seed=5, note="2048^3 FP32, 64 views"),
}


def config(name: str) -> WorkloadConfig:
    return CONFIGS[name]


def batched_instances(seed: int = 4, n: int = 32) -> List[WorkloadConfig]:
    """The uneven batched workload: n instances with per-axis edges in
    [96, 320], 90-360 views, square detectors of 128^2 to 512^2, cone or
    parallel beam with probability 1/2, 12 random ellipsoids each."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        shape = tuple(int(x) for x in rng.integers(96, 321, size=3))
        n_views = int(rng.integers(90, 361))
        n_det = int(rng.integers(128, 513))
        beam = "cone" if rng.uniform() < 0.5 else "parallel"
        inplane = math.hypot(shape[0], shape[1])
        if beam == "cone":
            sod = 4.0 * max(shape)
            sdd = 1.5 * sod
            mag = sdd / sod
            pu = mag * inplane * 1.05 / n_det
            pv = mag * shape[2] * 1.05 / n_det
        else:
            sod = sdd = 0.0
            pu = inplane * 1.05 / n_det
            pv = shape[2] * 1.05 / n_det
        out.append(WorkloadConfig(name=f"c4_{k}", shape=shape, n_views=n_views, n_u=n_det,
                                  n_v=n_det, beam=beam, sod=sod, sdd=sdd, pitch_u=pu,
                                  pitch_v=pv, phantom="random", phantom_seed=1000 + k))
    return out
