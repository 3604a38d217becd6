"""The quadrature comparison kernel on cell counts that leave a partial last block (a block
holds up to 8 cells; more for elasticity, as many as give every thread a 2 x 2 block of
function pairs, and for elements below 8 dofs, as many as give every thread one entry;
fewer when one cell's tables fill the LDS): every entry of every cell is written, nothing
past the last cell is, and the values match the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1112_0402_amd import meshgen
from paper_1112_0402_amd.forms import Form
from tests.gpu_util import rel_fro, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,dim,q", [("elasticity", 3, 2), ("elasticity", 2, 1), ("elasticity", 2, 3),
                                        ("mass", 3, 3), ("laplace", 3, 3), ("wlaplace", 2, 2), ("ns", 2, 2),
                                        ("laplace", 2, 1)])
@pytest.mark.parametrize("cells", [1, 13, 67])
def test_quadrature_partial_blocks(kind, dim, q, cells):
    require_gpu()
    wl = meshgen.make_workload(kind, dim, q, 6 if dim == 3 else 9, 17, max_cells=cells)
    f = Form(kind, dim, q, kernel="quadrature")
    n_I = f.info["n_entries"]
    # one spare cell past the end, filled with NaN: must stay untouched
    buf = torch.full((cells + 1, n_I), float("nan"), dtype=torch.float64, device="cuda")
    f.tabulate(to_dev(wl.coords), to_dev(wl.coeffs), out=buf[:cells])
    torch.cuda.synchronize()
    got = buf.cpu().numpy()
    assert np.isnan(got[cells]).all()
    assert np.isfinite(got[:cells]).all()
    ref = oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs)
    emax, _ = rel_fro(got[:cells], ref)
    say(f"[quadrature] {kind} d={dim} q={q} cells={cells}: max {emax:.2e}")
    assert emax <= 1e-12
