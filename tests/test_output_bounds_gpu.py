"""Output placement: element tensors written into a view of a NaN-filled buffer, 16-byte
aligned or not (an unaligned output takes the direct-store tile launch), with guard elements
on both sides of the view.  The guards must stay untouched (no write before or past the
output), every entry must be written, FP64 must be bitwise the same for both placements, and
sampled cells must match the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1112_0402_amd import capi, meshgen
from paper_1112_0402_amd.forms import Form
from tests.gpu_util import rel_fro, require_gpu, to_dev
from tests.test_gpu_parity import ALL_FORMS, FP64_TOL, split_tol

pytestmark = pytest.mark.gpu

GUARD = 8  # guard elements on each side of the output view


def _placed(form, cells, shift):
    """View of `cells` element tensors starting GUARD + shift elements into a NaN buffer."""
    n_el = cells * form.n_I
    buf = torch.full((n_el + 2 * GUARD + 1,), float("nan"), dtype=form.out_dtype, device="cuda")
    return buf, buf[GUARD + shift:GUARD + shift + n_el].view(cells, form.n, form.n)


def _guards_intact(buf, cells, form, shift):
    b = buf.cpu().numpy()
    n_el = cells * form.n_I
    return np.isnan(b[:GUARD + shift]).all() and np.isnan(b[GUARD + shift + n_el:]).all()


_FORMS = {}


def _check(kind, dim, q, precision, cells):
    wl = meshgen.make_workload(kind, dim, q, 11 if dim == 2 else 5, 77, max_cells=cells)
    key = (kind, dim, q, precision)
    if key not in _FORMS:
        _FORMS[key] = Form(kind, dim, q, precision=precision)
    f = _FORMS[key]
    X, C = to_dev(wl.coords), to_dev(wl.coeffs)
    got = {}
    for shift in (0, 1):  # 0: 16-byte aligned (GUARD elements are 32 or 64 bytes), 1: not
        buf, o = _placed(f, wl.cells, shift)
        assert (o.data_ptr() % 16 == 0) == (shift == 0)
        f.tabulate(X, C, out=o)
        torch.cuda.synchronize()
        assert _guards_intact(buf, wl.cells, f, shift), (kind, dim, q, precision, shift, "write outside the output")
        a = o.cpu().numpy()
        assert not np.isnan(a).any(), (kind, dim, q, precision, shift, "entries left unwritten")
        got[shift] = a
    if precision == "fp64":
        assert np.array_equal(got[0], got[1]), (kind, dim, q)
    idx = np.unique(np.r_[0, wl.cells - 1, np.arange(1, wl.cells, max(1, wl.cells // 7))])
    ref = oracle.tabulate(kind, dim, q, np.ascontiguousarray(wl.coords[:, idx]),
                          None if wl.coeffs is None else np.ascontiguousarray(wl.coeffs[:, idx]))
    tol = FP64_TOL if precision == "fp64" else split_tol(precision, kind, dim, q)
    for shift in (0, 1):
        assert rel_fro(got[shift][idx], ref)[0] <= tol, (kind, dim, q, precision, shift)


@pytest.mark.parametrize("kind,dim,q", ALL_FORMS)
def test_output_placement_fp64(kind, dim, q):
    require_gpu()
    for cells in (1, 17, 241):
        _check(kind, dim, q, "fp64", cells)


@pytest.mark.parametrize("kind,dim,q", [("laplace", 2, 4), ("mass", 3, 3), ("wlaplace", 3, 3), ("elasticity", 3, 2),
                                        ("ns", 2, 2), ("ns", 3, 2), ("laplace", 3, 1), ("elasticity", 2, 1)])
@pytest.mark.parametrize("precision", ["bf16x3", "bf16x6"])
def test_output_placement_split(kind, dim, q, precision):
    require_gpu()
    for cells in (1, 33, 241):
        _check(kind, dim, q, precision, cells)


@pytest.mark.parametrize("kind,dim,q", ALL_FORMS)
def test_action_placement(kind, dim, q):
    """The operator action y_K = A^K x_K into a view of a NaN buffer with guards, aligned and
    not: guards untouched, every value written, both placements bitwise equal, and y equal
    to the oracle's element tensors applied to x."""
    require_gpu()
    key = (kind, dim, q, "fp64")
    if key not in _FORMS:
        _FORMS[key] = Form(kind, dim, q)
    f = _FORMS[key]
    if 16 * f.n_I * 8 > 160 * 1024:
        # a 16-cell tile of element tensors does not fit the LDS: the action refuses the form
        wl = meshgen.make_workload(kind, dim, q, 11 if dim == 2 else 5, 78, max_cells=5)
        with pytest.raises(capi.FFCError) as ei:
            f.apply(to_dev(wl.coords), torch.zeros((wl.cells, f.n), dtype=torch.float64, device="cuda"),
                    to_dev(wl.coeffs))
        assert ei.value.code == capi.FFC_E_UNSUPPORTED
        return
    for cells in (1, 17, 241):
        wl = meshgen.make_workload(kind, dim, q, 11 if dim == 2 else 5, 78, max_cells=cells)
        X, C = to_dev(wl.coords), to_dev(wl.coeffs)
        xh = np.random.default_rng(cells).standard_normal((wl.cells, f.n))
        x = torch.from_numpy(xh).cuda()
        got = {}
        for shift in (0, 1):
            n_el = wl.cells * f.n
            buf = torch.full((n_el + 2 * GUARD + 1,), float("nan"), dtype=torch.float64, device="cuda")
            y = buf[GUARD + shift:GUARD + shift + n_el].view(wl.cells, f.n)
            f.apply(X, x, C, y=y)
            torch.cuda.synchronize()
            b = buf.cpu().numpy()
            assert np.isnan(b[:GUARD + shift]).all() and np.isnan(b[GUARD + shift + n_el:]).all(), (kind, dim, q, cells)
            got[shift] = y.cpu().numpy()
            assert not np.isnan(got[shift]).any(), (kind, dim, q, cells)
        assert np.array_equal(got[0], got[1]), (kind, dim, q, cells)
        ref = np.einsum("cij,cj->ci", oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs), xh)
        assert np.abs(got[0] - ref).max() <= FP64_TOL * max(np.abs(ref).max(), 1e-300), (kind, dim, q, cells)


@pytest.mark.parametrize("kind,dim,q", [("piola", 2, 1), ("piola", 3, 1), ("nedelec", 2, 1), ("nedelec", 3, 1),
                                        ("curved", 2, 1), ("curved", 2, 2), ("curved", 3, 1), ("curved", 3, 2)])
def test_output_placement_other_kinds(kind, dim, q):
    """The same placement checks for the Piola-mapped and curvilinear forms (FP64)."""
    require_gpu()
    f = Form(kind, dim, q)
    for cells in (1, 17, 241):
        if kind == "curved":
            wl = meshgen.curved_workload(dim, q, 11 if dim == 2 else 5, 79, max_cells=cells)
        else:
            wl = meshgen.make_workload(kind, dim, q, 11 if dim == 2 else 5, 79, max_cells=cells)
        X = to_dev(wl.coords)
        got = {}
        for shift in (0, 1):
            buf, o = _placed(f, wl.cells, shift)
            f.tabulate(X, out=o)
            torch.cuda.synchronize()
            assert _guards_intact(buf, wl.cells, f, shift), (kind, dim, q, cells, shift)
            got[shift] = o.cpu().numpy()
            assert not np.isnan(got[shift]).any(), (kind, dim, q, cells, shift)
        assert np.array_equal(got[0], got[1]), (kind, dim, q, cells)
        ref = (oracle.curved_laplace(dim, q, wl.coords) if kind == "curved"
               else oracle.piola_mass(dim, wl.coords) if kind == "piola" else oracle.nedelec_mass(dim, wl.coords))
        assert rel_fro(got[0], ref)[0] <= FP64_TOL, (kind, dim, q, cells)
