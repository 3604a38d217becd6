"""Pins for the H(curl) example (lowest-order Nedelec mass matrix under the covariant Piola
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
@pytest.mark.parametrize("seed", [1, 2])
def test_oracle_matches_exact_rationals(dim, seed):
    verts = _rational_cell(dim, seed)
    ref = np.array([[float(x) for x in row] for row in exact.nedelec_mass(verts)])
    got = oracle.nedelec_mass(dim, _soa(verts))[0]
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_constant_fields_are_reproduced(dim):
    """A constant field c is the Whitney combination sum_e circ_e(c) phi_e with the edge
    circulations circ_(a,b)(c) = c . (x^b - x^a); hence sum_e M_je circ_e(c) = int_K c . phi_j
    = c . |K| (grad lambda_b - grad lambda_a) / (d + 1) for edge j = (a, b)."""
    verts = np.array([[float(x) for x in v] for v in _rational_cell(dim, 4)])
    M = oracle.nedelec_mass(dim, _soa(verts))[0]
    T = np.vstack([verts.T, np.ones(dim + 1)])
    gl = np.linalg.inv(T)[:, :dim]
    vol = abs(np.linalg.det(verts[1:] - verts[0])) / math.factorial(dim)
    edges = oracle.NEDELEC_EDGES[dim]
    for c in np.eye(dim).tolist() + [[0.3, -1.1, 0.7][:dim]]:
        c = np.array(c)
        circ = np.array([c @ (verts[b] - verts[a]) for a, b in edges])
        rhs = np.array([c @ (gl[b] - gl[a]) * vol / (dim + 1) for a, b in edges])
        assert np.allclose(M @ circ, rhs, rtol=0, atol=1e-14 * np.abs(rhs).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_scaling_symmetry_definiteness(dim):
    verts = np.array([[float(x) for x in v] for v in _rational_cell(dim, 6)])
    M = oracle.nedelec_mass(dim, _soa(verts))[0]
    M2 = oracle.nedelec_mass(dim, _soa(2.5 * verts))[0]
    assert np.allclose(M2, 2.5 ** (dim - 2) * M, rtol=1e-13, atol=0)
    assert np.abs(M - M.T).max() <= 1e-15 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 0


@pytest.mark.parametrize("dim", [2, 3])
def test_compile_step_times_geometry_matches_oracle(dim):
    """The library's A^0 (alpha = a1 * d + a2) contracted with the Laplacian's
    G = |det J| g g^T (numpy, from the documented conventions) equals the oracle."""
    wl = meshgen.make_workload("nedelec", dim, 1, 2, seed=23)
    A0 = capi.reference_tensor("nedelec", dim, 1)
    cells = wl.cells
    X = wl.coords.T.reshape(cells, dim + 1, dim)
    J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))
    g = np.linalg.inv(J)
    G = np.einsum("cak,cbk->cab", g, g) * np.abs(np.linalg.det(J))[:, None, None]
    AK = G.reshape(cells, -1) @ A0.T
    ref = oracle.nedelec_mass(dim, wl.coords).reshape(cells, -1)
    assert (np.linalg.norm(AK - ref, axis=1) / np.linalg.norm(ref, axis=1)).max() < 1e-12
