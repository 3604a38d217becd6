"""Pins for the H(div) example (lowest-order Raviart-Thomas mass matrix under the Piola
map, Sec. 3.4): the oracle against exact rationals and closed relations, and the library's
compile step through A^0 : G_K against the oracle.  CPU only."""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_1112_0402_amd import capi, meshgen


def _rational_cell(dim, seed):
    rnd = random.Random(seed)
    base = [[0] * dim] + [[1 if k == v else 0 for k in range(dim)] for v in range(dim)]
    scale = Fraction(rnd.randint(20, 40), 37)
    return [[Fraction(c) * scale + Fraction(rnd.randint(-6, 6), 53) for c in v] for v in base]


def _soa(verts):
    return np.ascontiguousarray(np.asarray([[float(c) for c in v] for v in verts]).reshape(-1, 1))


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_oracle_matches_exact_rationals(dim, seed):
    verts = _rational_cell(dim, seed)
    ref = np.array([[float(x) for x in row] for row in exact.piola_mass(verts)])
    got = oracle.piola_mass(dim, _soa(verts))[0]
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_constant_fields_are_reproduced(dim):
    """A constant field c is the RT combination sum_i F_i(c) psi_i with facet fluxes
    F_i(c) = -d |K| c . grad(lambda_i); hence sum_i M_ji F_i(c) = int_K c . psi_j
    = c . (centroid - x^j) / d."""
    verts = np.array([[float(x) for x in v] for v in _rational_cell(dim, 9)])
    M = oracle.piola_mass(dim, _soa(verts))[0]
    T = np.vstack([verts.T, np.ones(dim + 1)])   # [x; 1] per vertex
    grad_lam = np.linalg.inv(T)[:, :dim]         # row i = grad lambda_i
    vol = abs(np.linalg.det(verts[1:] - verts[0])) / math.factorial(dim)
    for c in np.eye(dim).tolist() + [[0.3, -1.1, 0.7][:dim]]:
        c = np.array(c)
        flux = -dim * vol * grad_lam @ c
        rhs = (verts.mean(axis=0) - verts) @ c / dim
        assert np.allclose(M @ flux, rhs, rtol=0, atol=1e-14 * np.abs(rhs).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_scaling_symmetry_definiteness(dim):
    verts = np.array([[float(x) for x in v] for v in _rational_cell(dim, 4)])
    M = oracle.piola_mass(dim, _soa(verts))[0]
    M2 = oracle.piola_mass(dim, _soa(2.5 * verts))[0]
    assert np.allclose(M2, 2.5 ** (2 - dim) * M, rtol=1e-13, atol=0)
    assert np.allclose(M, M.T, rtol=0, atol=1e-15 * np.abs(M).max())
    assert np.linalg.eigvalsh(M).min() > 0


@pytest.mark.parametrize("dim", [2, 3])
def test_compile_step_times_geometry_matches_oracle(dim):
    """The library's A^0 (alpha = a1 * d + a2) contracted with G = (J^T J) / |det J|
    (numpy, from the documented conventions) equals the oracle, orientation included."""
    wl = meshgen.make_workload("piola", dim, 1, 2, seed=23)
    A0 = capi.reference_tensor("piola", dim, 1)
    cells = wl.cells
    X = wl.coords.T.reshape(cells, dim + 1, dim)
    J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))
    G = np.einsum("cka,ckb->cab", J, J) / np.abs(np.linalg.det(J))[:, None, None]
    AK = G.reshape(cells, -1) @ A0.T
    ref = oracle.piola_mass(dim, wl.coords).reshape(cells, -1)
    assert (np.linalg.norm(AK - ref, axis=1) / np.linalg.norm(ref, axis=1)).max() < 1e-12
    # reversed orientation (two vertices swapped) permutes the basis consistently
    Xr = X.copy()
    Xr[:, [1, 2]] = X[:, [2, 1]]
    cr = np.ascontiguousarray(Xr.reshape(cells, -1).T)
    Mr = oracle.piola_mass(dim, cr)
    p = [0, 2, 1] + list(range(3, dim + 1))
    Mp = ref.reshape(cells, dim + 1, dim + 1)[:, p][:, :, p]
    assert np.abs(Mr - Mp).max() <= 1e-13 * np.abs(Mp).max()


def test_unsupported_uses_are_rejected():
    L = capi.lib()
    nI, na = ctypes_pair()
    d = capi.make_desc("piola", 2, 2)
    assert L.ffc_compile_reference_tensor(d, nI, na, None) == capi.FFC_E_UNSUPPORTED


def ctypes_pair():
    import ctypes
    a, b = ctypes.c_int64(), ctypes.c_int64()
    return ctypes.byref(a), ctypes.byref(b)
