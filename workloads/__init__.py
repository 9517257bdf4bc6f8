"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module generates inputs only: ellipsoid phantoms and their rasterised
volumes, scan trajectories described by their parameters, random ray
geometries and random arrays. It contains none of the projector's arithmetic
(no ray setup, no sampling, no interpolation) and imports neither the GPU
library nor the oracle.

Ellipsoid phantoms stand in for the paper's benchmark object (a 3D
Shepp-Logan-type sum of uniform ellipsoids, Sec. IV-A). The published table
of that phantom is not reproduced here: ``sl_stand_in`` is a nested
10-ellipsoid "head-like" phantom with parameters chosen for this project.
"""
from .phantoms import (  # noqa: F401
    Ellipsoid,
    random_ellipsoids,
    sl_stand_in,
    rasterize,
    rasterize_torch,
)
from .configs import CONFIGS, WorkloadConfig, config  # noqa: F401
from .geometry import random_cone_views, random_parallel_views, sample_rays  # noqa: F401
