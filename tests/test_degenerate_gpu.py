"""Validation mode (ffc_check_cells): a cell whose affine map is not invertible has no
element tensor (Sec. 3.2).  The check flags |det J| <= tol * h^d, h the longest edge, and
non-finite det J; the expected sets come from the construction of the planted cells and
from NumPy determinants of the same coordinates, with tol chosen far from every cell's
ratio so the two evaluations cannot disagree."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1112_0402_amd import capi, meshgen
from paper_1112_0402_amd.forms import check_cells
from tests.gpu_util import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


def _ratios(coords, dim):
    """|det J| / h^d per cell, in NumPy (FP64)."""
    x = coords.reshape(dim + 1, dim, -1)  # [vertex][component][cell]
    J = np.stack([x[b + 1] - x[0] for b in range(dim)], axis=-1)  # [component][cell][b]
    J = np.moveaxis(J, 1, 0)  # [cell][component][b]
    det = np.abs(np.linalg.det(J))
    h2 = np.zeros(x.shape[-1])
    for v in range(dim + 1):
        for w in range(v + 1, dim + 1):
            h2 = np.maximum(h2, ((x[w] - x[v]) ** 2).sum(axis=0))
    return det / h2 ** (dim / 2)


@pytest.mark.parametrize("dim", [2, 3])
def test_well_shaped_mesh_passes(dim):
    require_gpu()
    wl = meshgen.make_workload("laplace", dim, 1, 150 if dim == 2 else 20, 3)
    r = _ratios(wl.coords, dim)
    tol = 0.1 * r.min()
    assert check_cells(to_dev(wl.coords), dim, tol) == (0, -1)
    L = capi.lib()
    cnt, first = ctypes.c_int64(), ctypes.c_int64()
    X = to_dev(wl.coords)
    assert L.ffc_check_cells(dim, wl.cells, X.data_ptr(), tol, ctypes.byref(cnt), ctypes.byref(first), None) == 0
    say(f"[degenerate] d={dim} {wl.cells} cells, min |det J|/h^d {r.min():.3e}: none flagged at tol {tol:.1e}")


@pytest.mark.parametrize("dim", [2, 3])
def test_planted_degenerate_cells(dim):
    """Collapsed cells (a vertex on another: det J = 0 exactly), flattened cells (a vertex
    moved into the opposite facet's plane: det J at rounding level), slivers (ratio ~1e-6),
    and a NaN coordinate, planted across several workgroups and a ragged last one."""
    require_gpu()
    wl = meshgen.make_workload("laplace", dim, 1, 200 if dim == 2 else 25, 5, max_cells=70001)
    X = wl.coords.copy()
    n = wl.cells
    x = X.reshape(dim + 1, dim, n)
    collapsed = [5, 300, 40001, n - 1]
    for c in collapsed:
        x[dim, :, c] = x[0, :, c]
    flat = [17, 1024, 65535]
    for c in flat:  # last vertex into the plane (line) of the others
        x[dim, :, c] = x[0, :, c] + 0.3 * (x[1, :, c] - x[0, :, c]) + (0.45 * (x[2, :, c] - x[0, :, c]) if dim == 3 else 0)
    sliver = [777, 20000]
    for c in sliver:  # last vertex a tiny distance off that plane
        e = x[1, :, c] - x[0, :, c]
        base = x[0, :, c] + 0.4 * e + (0.35 * (x[2, :, c] - x[0, :, c]) if dim == 3 else 0)
        if dim == 2:
            nrm = np.array([-e[1], e[0]])
        else:
            nrm = np.cross(e, x[2, :, c] - x[0, :, c])
        x[dim, :, c] = base + 1e-6 * np.linalg.norm(e) * nrm / np.linalg.norm(nrm)
    nan_cell = 999
    x[1, 0, nan_cell] = np.nan
    Xd = to_dev(X)
    r = _ratios(X, dim)
    good = np.ones(n, bool)
    good[collapsed + flat + sliver + [nan_cell]] = False
    assert r[good].min() > 1e-3 and np.all(r[flat] < 1e-13) and np.all((r[sliver] > 1e-8) & (r[sliver] < 1e-5))
    # tol = 0: the collapsed cells (det exactly 0, the NaN one); flattened cells may round to +-tiny
    cnt, first = check_cells(Xd, dim, 0.0)
    assert first == 5 and len(collapsed) + 1 <= cnt <= len(collapsed) + 1 + len(flat)
    # tol between the flattened and the sliver ratios: collapsed + flat + NaN
    assert check_cells(Xd, dim, 1e-11) == (len(collapsed) + len(flat) + 1, 5)
    # tol between the sliver ratios and the well-shaped cells: every planted cell
    assert check_cells(Xd, dim, 1e-4) == (len(collapsed) + len(flat) + len(sliver) + 1, 5)
    # the C call reports FFC_E_DEGENERATE with the count in its message; a prefix without
    # planted cells passes
    L = capi.lib()
    c1, f1 = ctypes.c_int64(), ctypes.c_int64()
    assert L.ffc_check_cells(dim, n, Xd.data_ptr(), 1e-4, ctypes.byref(c1), ctypes.byref(f1), None) == capi.FFC_E_DEGENERATE
    assert (c1.value, f1.value) == (10, 5) and b"10 degenerate" in L.ffc_last_error()
    assert check_cells(to_dev(np.ascontiguousarray(X[:, :5])), dim, 1e-4) == (0, -1)
    say(f"[degenerate] d={dim}: {c1.value} flagged of {n}, first {f1.value}")
