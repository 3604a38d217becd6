"""Helpers shared by the GPU tests (no oracle arithmetic here)."""
import sys

import numpy as np
import torch


def require_gpu():
    import pytest
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_fro(got: np.ndarray, ref: np.ndarray):
    """Per-cell relative Frobenius error ||got - ref||_F / ||ref||_F -> (max, median)."""
    cells = ref.shape[0]
    g = got.reshape(cells, -1).astype(np.float64)
    r = ref.reshape(cells, -1)
    num = np.linalg.norm(g - r, axis=1)
    den = np.linalg.norm(r, axis=1)
    den = np.where(den == 0, 1.0, den)
    e = num / den
    return float(e.max()), float(np.median(e))


def to_dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()
