"""Elasticity at lambda != mu on the GPU (test case 4, Sec. 3.3): every kernel path against
the oracle at the same Lame parameters -- FP64 tensor kernels (persistent and per-tile) and
the quadrature kernel to 1e-12, split BF16 x6 to 1e-6 -- and the homogeneous-strain energy
identity v^T A^K u = |K| (2 mu sym(B_v) : sym(B_u) + lambda tr B_v tr B_u) for linear fields
checked on the GPU's own output, which does not go through the oracle at all."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1112_0402_amd import meshgen
from paper_1112_0402_amd.forms import Form
from tests.gpu_util import rel_fro, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu

LAME = [(0.7, 1.3), (0.0, 0.5), (1.7, 0.3)]  # (lambda, mu); mu = 1/2, lambda = 0: the paper's strain-strain term


def _mesh(dim, q):
    n = 11 if dim == 2 else 5  # 242 / 750 cells: several tiles and a ragged tail
    return meshgen.make_workload("elasticity", dim, q, n, 41 + q)


@pytest.mark.parametrize("lam,mu", LAME)
@pytest.mark.parametrize("dim,q", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_lame_parameters_every_path(dim, q, lam, mu):
    require_gpu()
    wl = _mesh(dim, q)
    ref = oracle.tabulate("elasticity", dim, q, wl.coords, lam=lam, mu=mu)
    X = to_dev(wl.coords)
    paths = [("tensor", "fp64", {}, 1e-12), ("tensor", "fp64", dict(persistent=-1), 1e-12),
             ("quadrature", "fp64", {}, 1e-12), ("tensor", "bf16x6", {}, 1e-6)]
    if dim == 3 and q == 2:
        paths.append(("tensor", "fp64", dict(persistent=1), 1e-12))
    for kernel, precision, extra, tol in paths:
        f = Form("elasticity", dim, q, precision=precision, kernel=kernel, lam=lam, mu=mu, **extra)
        got = f.tabulate(X)
        torch.cuda.synchronize()
        e = rel_fro(got.cpu().numpy(), ref)[0]
        say(f"[lame] {kernel} {precision} {extra} d={dim} q={q} lambda={lam} mu={mu}: max {e:.2e} "
            f"(persistent waves {f.info['persistent_waves']})")
        assert e <= tol


@pytest.mark.parametrize("kernel", ["tensor", "quadrature"])
def test_energy_identity_on_gpu_output(kernel):
    require_gpu()
    dim, q, lam, mu = 3, 2, 0.7, 1.3
    wl = _mesh(dim, q)
    A = Form("elasticity", dim, q, kernel=kernel, lam=lam, mu=mu).tabulate(to_dev(wl.coords))
    torch.cuda.synchronize()
    A = A.cpu().numpy()
    rng = np.random.default_rng(3)
    bary = oracle.nodes(dim, q).astype(np.float64) / q
    for c in rng.choice(wl.cells, size=40, replace=False):
        cell = wl.coords[:, c].reshape(dim + 1, dim)
        vol = abs(np.linalg.det(cell[1:] - cell[0])) / math.factorial(dim)
        P = bary @ cell
        B_u, B_v = rng.standard_normal((dim, dim)), rng.standard_normal((dim, dim))
        u = (P @ B_u.T + rng.standard_normal(dim)).T.reshape(-1)
        v = (P @ B_v.T + rng.standard_normal(dim)).T.reshape(-1)
        su, sv = 0.5 * (B_u + B_u.T), 0.5 * (B_v + B_v.T)
        want = vol * (2 * mu * np.sum(sv * su) + lam * np.trace(B_u) * np.trace(B_v))
        scale = vol * (2 * mu + dim * lam) * np.linalg.norm(B_u) * np.linalg.norm(B_v)
        assert abs(v @ A[c] @ u - want) <= 1e-12 * scale
