"""GPU parity of the operator action (matrix-free use of the tensor representation):
per cell, y_K = A^K x_K against the oracle's element tensors times the same x_K; globally,
y = A x against the oracle-assembled CSR matrix times x."""
import numpy as np
import pytest
import torch

import oracle
from oracle.assemble import assemble
from paper_1112_0402_amd import capi, meshgen
from paper_1112_0402_amd.forms import Assembly, Form
from tests.gpu_util import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-12

# (kind, dim, q, mesh n): persistent forms (n_I >= 576: elasticity and NS in 3D, Laplacian
# 3D P4) and tile-kernel forms, meshes of several tiles with a ragged tail
CASES = [("elasticity", 3, 2, 5), ("ns", 3, 2, 5), ("laplace", 3, 4, 4), ("wlaplace", 3, 3, 5), ("mass", 2, 1, 11),
         ("laplace", 2, 1, 11), ("elasticity", 2, 3, 9), ("ns", 2, 2, 9), ("mass", 3, 3, 4), ("laplace", 2, 4, 9)]


def _x(cells, n, seed):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(cells, n))


def _action_err(y, A, x):
    """max over cells of ||y - A x|| / (||A||_F ||x||)"""
    ref = np.einsum("cij,cj->ci", A, x)
    num = np.linalg.norm(y - ref, axis=1)
    den = np.linalg.norm(A.reshape(len(A), -1), axis=1) * np.linalg.norm(x, axis=1)
    return float((num / np.where(den == 0, 1.0, den)).max(initial=0.0))


@pytest.mark.parametrize("kind,dim,q,n", CASES)
def test_local_action_matches_oracle(kind, dim, q, n):
    require_gpu()
    wl = meshgen.make_workload(kind, dim, q, n, 21)
    f = Form(kind, dim, q)
    nd = f.info["n_dofs"]
    x = _x(wl.cells, nd, 5)
    y = f.apply(to_dev(wl.coords), to_dev(x), to_dev(wl.coeffs))
    again = f.apply(to_dev(wl.coords), to_dev(x), to_dev(wl.coeffs))
    torch.cuda.synchronize()
    assert torch.equal(y, again)
    A = oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs).reshape(wl.cells, nd, nd)
    e = _action_err(y.cpu().numpy(), A, x)
    say(f"[action] {kind} d={dim} q={q} ({wl.cells} cells, persistent {f.info['persistent_waves']}): max {e:.2e}")
    assert e <= TOL


@pytest.mark.parametrize("kind,dim,q", [("elasticity", 3, 2), ("laplace", 3, 4), ("ns", 3, 2)])
def test_action_persistent_and_tile_kernels_agree(kind, dim, q):
    """The persistent kernel's action (I/O waves multiply the staged tile) and the tile
    kernel's agree to rounding, and both equal the tabulated element tensors times x."""
    require_gpu()
    wl = meshgen.make_workload(kind, dim, q, 7, 8, max_cells=1999)
    X, C = to_dev(wl.coords), to_dev(wl.coeffs)
    fp, ft = Form(kind, dim, q), Form(kind, dim, q, persistent=-1)
    nd = fp.info["n_dofs"]
    x = _x(wl.cells, nd, 9)
    yp = fp.apply(X, to_dev(x), C).cpu().numpy()
    yt = ft.apply(X, to_dev(x), C).cpu().numpy()
    A = fp.tabulate(X, C).cpu().numpy().reshape(wl.cells, nd, nd)
    assert _action_err(yp, A, x) <= 1e-14 * nd
    assert _action_err(yt, A, x) <= 1e-14 * nd


def test_action_edge_cases():
    require_gpu()
    f = Form("elasticity", 3, 2)
    empty = torch.empty((12, 0), dtype=torch.float64, device="cuda")
    y = f.apply(empty, torch.empty((0, 30), dtype=torch.float64, device="cuda"))
    assert y.shape == (0, 30)
    # a single cell (one partial tile) and 17 cells (a full tile plus one)
    for cells in (1, 17):
        wl = meshgen.make_workload("elasticity", 3, 2, 2, 3, max_cells=cells)
        x = _x(cells, 30, cells)
        yv = f.apply(to_dev(wl.coords), to_dev(x)).cpu().numpy()
        A = oracle.tabulate("elasticity", 3, 2, wl.coords).reshape(cells, 30, 30)
        assert _action_err(yv, A, x) <= TOL
    with pytest.raises(capi.FFCError):
        Form("laplace", 3, 2, precision="bf16x3").apply(to_dev(wl.coords[:, :1].copy()), torch.zeros(
            (1, 10), dtype=torch.float64, device="cuda"))
    with pytest.raises(capi.FFCError):
        Form("laplace", 3, 2, kernel="quadrature").apply(to_dev(wl.coords[:, :1].copy()), torch.zeros(
            (1, 10), dtype=torch.float64, device="cuda"))


def test_config2_full_size_action_sampled():
    """750,000-cell elasticity (the benchmarked mesh): sampled cells against the oracle."""
    require_gpu()
    wl = meshgen.config2()
    f = Form("elasticity", 3, 2)
    x = _x(wl.cells, 30, 2)
    y = f.apply(to_dev(wl.coords), to_dev(x)).cpu().numpy()
    rng = np.random.default_rng(2)
    idx = np.unique(np.concatenate([[0, 1, wl.cells - 2, wl.cells - 1], rng.choice(wl.cells, 2000, replace=False)]))
    A = oracle.tabulate("elasticity", 3, 2, wl.coords[:, idx]).reshape(len(idx), 30, 30)
    e = _action_err(y[idx], A, x[idx])
    say(f"[action cfg2] sampled max {e:.2e}")
    assert e <= TOL


@pytest.mark.parametrize("kind,dim,q,n", [("laplace", 2, 1, 9), ("laplace", 3, 2, 3), ("elasticity", 3, 2, 3),
                                          ("wlaplace", 3, 2, 3), ("ns", 2, 2, 6), ("laplace", 3, 4, 2)])
def test_global_operator_matches_assembled_matrix(kind, dim, q, n):
    """y = A x without forming A equals the oracle-assembled CSR matrix times x; two runs
    are bitwise equal (fixed summation order)."""
    require_gpu()
    wl = meshgen.make_workload(kind, dim, q, n, 11)
    comps = dim if kind in ("elasticity", "ns") else 1
    dm, ng = meshgen.lagrange_dofmap(wl.meta["cells"], q, comps)
    form = Form(kind, dim, q)
    asm = Assembly(dm, ng)
    x = np.random.default_rng(4).uniform(-1.0, 1.0, size=ng)
    X, C, xd = to_dev(wl.coords), to_dev(wl.coeffs), to_dev(x)
    y = asm.apply(form, X, xd, C)
    y2 = asm.apply(form, X, xd, C)
    torch.cuda.synchronize()
    assert torch.equal(y, y2)
    K = assemble(oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs), dm, ng)
    ref = K @ x
    scale = abs(K).max() * np.abs(x).max() * max(np.diff(K.indptr).max(), 1)
    e = float(np.abs(y.cpu().numpy() - ref).max() / scale)
    say(f"[operator] {kind} d={dim} q={q}: {ng} dofs, max error {e:.2e}")
    assert e <= TOL


def test_global_operator_graph_replay():
    """The matrix-free y = A x (gather, per-cell action, fixed-order sum) and its
    allocation-free entry point, each captured in a graph and replayed three times with eager
    work between the replays: every replay equals the eager result bit for bit."""
    require_gpu()
    s = torch.cuda.Stream()
    wl = meshgen.make_workload("elasticity", 3, 2, 5, 12)
    dm, ng = meshgen.lagrange_dofmap(wl.meta["cells"], 2, 3)
    form = Form("elasticity", 3, 2, stream=s)
    asm = Assembly(dm, ng, stream=s)
    X, xd = to_dev(wl.coords), to_dev(np.random.default_rng(6).uniform(-1.0, 1.0, size=ng))
    y = torch.empty(ng, dtype=torch.float64, device="cuda")
    y2 = torch.empty_like(y)
    work = torch.empty(2 * asm.cells * asm.n_local, dtype=torch.float64, device="cuda")

    def noalloc():
        capi.check(capi.lib().ffc_operator_apply_noalloc(asm._h, form.handle, X.data_ptr(), None, xd.data_ptr(),
                                                         y2.data_ptr()))

    with torch.cuda.stream(s):
        asm.apply(form, X, xd, y=y, work=work)
        noalloc()
    torch.cuda.synchronize()
    eager, eager2 = y.clone(), y2.clone()
    assert torch.equal(eager, eager2)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        asm.apply(form, X, xd, y=y, work=work)
        noalloc()
    other = Form("mass", 2, 1)
    ow = to_dev(meshgen.make_workload("mass", 2, 1, 20, 13).coords)
    for rep in range(3):
        y.fill_(float("nan"))
        y2.fill_(float("nan"))
        other.tabulate(ow)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, eager), rep
        assert torch.equal(y2, eager2), rep
