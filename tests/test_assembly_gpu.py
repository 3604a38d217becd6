"""GPU parity of global assembly (Algorithm 2's insertion step): the library's CSR pattern
equals the oracle's, and its values equal the oracle assembly of oracle element tensors."""
import numpy as np
import pytest
import torch

import oracle
from oracle.assemble import assemble
from paper_1112_0402_amd import meshgen
from paper_1112_0402_amd.forms import Assembly, Form
from tests.gpu_util import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu

CASES = [("laplace", 2, 1, 9), ("laplace", 2, 3, 5), ("laplace", 3, 2, 3), ("laplace", 3, 4, 2), ("mass", 3, 3, 2),
         ("wlaplace", 3, 2, 3), ("elasticity", 3, 2, 3), ("ns", 2, 2, 6), ("elasticity", 2, 3, 4)]


def _setup(kind, dim, q, n, seed=11):
    wl = meshgen.make_workload(kind, dim, q, n, seed)
    comps = dim if kind in ("elasticity", "ns") else 1
    dm, ng = meshgen.lagrange_dofmap(wl.meta["cells"], q, comps)
    return wl, dm, ng


def _row_err(vals, ref):
    """max over rows of max |v - r| / max |r| of the row"""
    ref = ref.tocsr()
    err = 0.0
    for r in range(ref.shape[0]):
        a, b = ref.indptr[r], ref.indptr[r + 1]
        scale = max(abs(ref.data[a:b]).max(initial=0.0), 1e-300)
        err = max(err, abs(vals[a:b] - ref.data[a:b]).max(initial=0.0) / scale)
    return err


@pytest.mark.parametrize("kind,dim,q,n", CASES)
def test_assembly_matches_oracle(kind, dim, q, n):
    require_gpu()
    wl, dm, ng = _setup(kind, dim, q, n)
    form = Form(kind, dim, q)
    T = form.tabulate(to_dev(wl.coords), to_dev(wl.coeffs))
    asm = Assembly(dm, ng)
    vals = asm.assemble(T)
    torch.cuda.synchronize()
    ref = assemble(oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs), dm, ng)
    rp, ci = asm.pattern()
    assert np.array_equal(rp, ref.indptr) and np.array_equal(ci, ref.indices)
    again = asm.assemble(T)  # fixed summation order: reproducible to the bit
    torch.cuda.synchronize()
    assert torch.equal(vals, again)
    e = _row_err(vals.cpu().numpy(), ref)
    say(f"[assembly] {kind} d={dim} q={q}: {ng} dofs, nnz {asm.nnz}, max row error {e:.2e}")
    assert e <= 1e-12


def test_assembly_of_split_output_accumulate_and_graph_replay():
    """FP32 element tensors (split BF16 output) are added in FP64; accumulate adds onto the
    existing values; a captured graph replays the assembly (fill kernel, no memset)."""
    require_gpu()
    wl, dm, ng = _setup("wlaplace", 3, 3, 2)
    T = Form("wlaplace", 3, 3, precision="bf16x6").tabulate(to_dev(wl.coords), to_dev(wl.coeffs))
    torch.cuda.synchronize()
    ref = assemble(T.cpu().numpy().astype(np.float64), dm, ng)
    s = torch.cuda.Stream()
    asm = Assembly(dm, ng, stream=s)
    with torch.cuda.stream(s):
        v = asm.assemble(T)
        torch.cuda.synchronize()
        assert _row_err(v.cpu().numpy(), ref) <= 1e-12
        asm.assemble(T, values=v, accumulate=True)
        torch.cuda.synchronize()
        assert _row_err(v.cpu().numpy() / 2, ref) <= 1e-12
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        asm.assemble(T, values=v)
    for rep in range(3):
        v.fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.replay()
        torch.cuda.synchronize()
        assert _row_err(v.cpu().numpy(), ref) <= 1e-12, rep


def test_assembly_edge_cases():
    require_gpu()
    from paper_1112_0402_amd import capi

    # no cells: an empty pattern, assembly is a no-op
    asm = Assembly(np.zeros((0, 3), dtype=np.int32), 5)
    assert asm.nnz == 0
    rp, ci = asm.pattern()
    assert np.array_equal(rp, np.zeros(6)) and ci.size == 0
    asm.assemble(torch.empty((0, 3, 3), dtype=torch.float64, device="cuda"), torch.empty(0, dtype=torch.float64,
                                                                                           device="cuda"))
    # one cell: the pattern is the full n x n block of its dofs, values are its tensor
    wl, dm, ng = _setup("laplace", 2, 2, 1)
    dm1 = dm[:1]
    T = Form("laplace", 2, 2).tabulate(to_dev(np.ascontiguousarray(wl.coords[:, :1])))
    a1 = Assembly(dm1, ng)
    v = a1.assemble(T)
    torch.cuda.synchronize()
    ref = assemble(T.cpu().numpy(), dm1, ng)
    assert np.allclose(v.cpu().numpy(), ref.data, rtol=0, atol=0)
    # a dof index out of range is refused before anything runs
    bad = dm1.copy()
    bad[0, 0] = ng
    with pytest.raises(capi.FFCError):
        Assembly(bad, ng)


def test_config2_full_size_assembly_sampled_rows():
    """Elasticity P2, 750,000 cells (the bench's element tensors): the assembled values of
    300 sampled rows against a brute-force sum over the cells incident to each row."""
    require_gpu()
    wl = meshgen.config2()
    dm, ng = meshgen.lagrange_dofmap(wl.meta["cells"], 2, 3)
    T = Form("elasticity", 3, 2).tabulate(to_dev(wl.coords))
    asm = Assembly(dm, ng)
    v = asm.assemble(T)
    torch.cuda.synchronize()
    rp, ci = asm.pattern()
    vals = v.cpu().numpy()
    rng = np.random.default_rng(4)
    rows = rng.choice(ng, size=300, replace=False)
    n = dm.shape[1]
    order = np.argsort(dm.reshape(-1), kind="stable")  # (cell, local) slots grouped by dof
    starts = np.searchsorted(dm.reshape(-1)[order], np.arange(ng + 1))
    worst = 0.0
    for r in rows:
        slots = order[starts[r]:starts[r + 1]]
        cells, loc = slots // n, slots % n
        expect = {}
        Tc = T[torch.from_numpy(cells).cuda()].cpu().numpy()
        for k, (c, i) in enumerate(zip(cells, loc)):
            for j in range(n):
                col = int(dm[c, j])
                expect[col] = expect.get(col, 0.0) + Tc[k, i, j]
        cols = ci[rp[r]:rp[r + 1]]
        assert sorted(expect) == list(cols)
        got = vals[rp[r]:rp[r + 1]]
        ref = np.array([expect[c] for c in cols])
        worst = max(worst, abs(got - ref).max() / abs(ref).max())
    say(f"[assembly cfg2] {ng} dofs, nnz {asm.nnz}, max sampled row error {worst:.2e}")
    assert worst <= 1e-12
