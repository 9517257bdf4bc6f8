"""Shared helpers of the GPU parity tests (no arithmetic of the method here)."""
import sys

import numpy as np


def rel_l2(got, want) -> float:
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return float(np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300))


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
