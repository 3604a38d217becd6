"""The allocation-free operator entry point (ffc_operator_apply_noalloc, scratch in a fixed
library-owned device array) against ffc_operator_apply (caller's work buffer), called through
the C-ABI: two calls in a row on different meshes, the second smaller, each bitwise equal to
the existing entry point's result; sizes beyond the array are refused before anything runs."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1112_0402_amd import capi, meshgen
from paper_1112_0402_amd.forms import Assembly, Form
from tests.gpu_util import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


def _case(kind, dim, q, n, seed, comps):
    wl = meshgen.make_workload(kind, dim, q, n, seed)
    dm, ng = meshgen.lagrange_dofmap(wl.meta["cells"], q, comps)
    return wl, Assembly(dm, ng), Form(kind, dim, q)


def _noalloc(asm, form, X, C, x, y):
    return capi.lib().ffc_operator_apply_noalloc(asm._h, form.handle, X.data_ptr(),
                                                  None if C is None else C.data_ptr(), x.data_ptr(), y.data_ptr())


def test_noalloc_operator_matches_operator_apply_twice():
    require_gpu()
    # first call: elasticity P2 on 10,368 tets (311,040 local dofs, 622,080 scratch doubles);
    # second call: a smaller mesh and another form (weighted Laplacian P2 on 750 tets)
    for kind, q, n, comps in (("elasticity", 2, 12, 3), ("wlaplace", 2, 5, 1)):
        wl, asm, form = _case(kind, 3, q, n, 70 + n, comps)
        X, C = to_dev(wl.coords), to_dev(wl.coeffs)
        x = torch.from_numpy(np.random.default_rng(n).standard_normal(asm.n_rows)).cuda()
        ref = asm.apply(form, X, x, C)
        y = torch.full((asm.n_rows,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        capi.check(_noalloc(asm, form, X, C, x, y))
        torch.cuda.synchronize()
        say(f"[noalloc] {kind} P{q}: {wl.cells} cells, {asm.n_rows} dofs, max |y - ref| "
            f"{float((y - ref).abs().max()):.1e}")
        assert torch.equal(y, ref)


def test_noalloc_operator_refuses_beyond_its_scratch():
    require_gpu()
    wl, asm, form = _case("elasticity", 3, 2, 37, 5, 3)  # 303,918 cells: 2 * cells * 30 > 2^24
    assert 2 * wl.cells * form.n > (1 << 24)
    X = to_dev(wl.coords)
    x = torch.zeros(asm.n_rows, dtype=torch.float64, device="cuda")
    y = torch.full((asm.n_rows,), 7.0, dtype=torch.float64, device="cuda")
    assert _noalloc(asm, form, X, None, x, y) == capi.FFC_E_UNSUPPORTED
    assert b"2^24" in capi.lib().ffc_last_error()
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())  # nothing ran
