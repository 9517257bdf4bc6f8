"""Shared helpers of the GPU parity tests (no arithmetic of the method here)."""
import sys

import numpy as np


def rel_l2(got, want) -> float:
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return float(np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300))


def assert_parity(got, want, tol, elem=None):
    """Relative L2 error <= tol over the compared values, and every element
    within elem * max|want| (default: the same factor as tol). An all-zero
    reference requires an all-zero result."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape, (got.shape, want.shape)
    scale = float(np.abs(want).max()) if want.size else 0.0
    if scale == 0.0:
        assert not np.any(got), f"reference is zero, result has {int(np.count_nonzero(got))} non-zeros"
        return
    err = rel_l2(got, want)
    assert err <= tol, f"relative L2 error {err:.3e} > {tol:.1e}"
    worst = float(np.abs(got - want).max())
    lim = (tol if elem is None else elem) * scale
    assert worst <= lim, f"max element error {worst:.3e} > {lim:.3e} ({worst / scale:.2e} of max)"


def note(msg: str) -> None:
    """Name the case before a GPU step (flushed, so it survives a crash)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no HIP device")
    return torch.device("cuda:0")
