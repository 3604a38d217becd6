"""GPU parity of the linear form L(v) = int f v dx (rank-1 element vectors and the assembled
load vector) against the oracle's quadrature of f v on the physical cell."""
import numpy as np
import pytest

import oracle
from paper_1112_0402_amd import meshgen
from paper_1112_0402_amd.forms import Assembly, SourceForm
from tests.gpu_util import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,q,n", [(2, 1, 11), (2, 3, 9), (3, 2, 5), (3, 3, 4), (2, 4, 7)])
def test_source_element_vectors_and_load_vector(dim, q, n):
    require_gpu()
    wl = meshgen.make_workload("mass", dim, q, n, 17)
    cells_v = wl.meta["cells"]
    dm, ng = meshgen.lagrange_dofmap(cells_v, q, 1)
    fg = np.random.default_rng(3).normal(size=ng)          # f as a global P_q function
    fl = np.ascontiguousarray(fg[dm])                        # its dofs on each cell
    L = SourceForm(dim, q)
    b = L.tabulate(to_dev(wl.coords), to_dev(fl)).cpu().numpy()
    ref = oracle.source_vector(dim, q, wl.coords, fl)
    e = float((np.linalg.norm(b - ref, axis=1) / np.linalg.norm(ref, axis=1)).max())
    bg = Assembly(dm, ng).apply(L.mass, to_dev(wl.coords), to_dev(fg)).cpu().numpy()
    refg = np.zeros(ng)
    np.add.at(refg, dm, ref)
    eg = float(np.abs(bg - refg).max() / np.abs(refg).max())
    say(f"[source] d={dim} q={q} ({wl.cells} cells): element max {e:.2e}, load vector {eg:.2e}")
    assert e <= 1e-12 and eg <= 1e-12
