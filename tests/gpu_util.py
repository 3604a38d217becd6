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


def every_cell_errors(kind, dim, q, coords, coeffs, outputs, chunk=32768, lam=1.0, mu=1.0):
    """Per-cell relative Frobenius error of every cell of each device output in `outputs`
    (name -> torch tensor [cells, ...]) against the oracle, which runs once per chunk of cells
    and is shared by all outputs.  Returns name -> (max, median, cells); also asserts that
    every output value is finite."""
    import oracle

    cells = coords.shape[1]
    errs = {name: np.empty(cells) for name in outputs}
    for c0 in range(0, cells, chunk):
        c1 = min(cells, c0 + chunk)
        ref = oracle.tabulate(kind, dim, q, np.ascontiguousarray(coords[:, c0:c1]),
                              None if coeffs is None else np.ascontiguousarray(coeffs[:, c0:c1]), lam=lam, mu=mu)
        r = ref.reshape(c1 - c0, -1)
        den = np.linalg.norm(r, axis=1)
        den = np.where(den == 0, 1.0, den)
        for name, out in outputs.items():
            g = out[c0:c1].reshape(c1 - c0, -1).cpu().numpy().astype(np.float64)
            assert np.all(np.isfinite(g)), (name, c0)
            errs[name][c0:c1] = np.linalg.norm(g - r, axis=1) / den
    return {name: (float(e.max()), float(np.median(e)), cells) for name, e in errs.items()}
