import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long-running GPU parity at full workload size")


def grid_point(shape, p_grid):
    """World coordinates of a grid-coordinate point (unit voxels, centred grid)."""
    return np.asarray(p_grid, dtype=np.float64) - 0.5 * (np.asarray(shape, dtype=np.float64) - 1)


def parallel_rays_views(shape, direction, det00_grid, du, dv):
    """One parallel-beam view: rays along `direction`, pixel (iu, iv) through
    grid point det00_grid + iu du + iv dv (du, dv in grid units)."""
    v = np.zeros((1, 12), dtype=np.float64)
    v[0, 0:3] = direction
    v[0, 3:6] = grid_point(shape, det00_grid)
    v[0, 6:9] = du
    v[0, 9:12] = dv
    return v


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.lib()
    return oracle
