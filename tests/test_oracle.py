"""Pins for the oracle: closed forms, the paper's printed reference-tensor values, exact
rational integration and invariants.  CPU only."""
import itertools
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _coords_of(verts):
    """SoA coordinates [(d+1)*d][1] of one cell given [d+1][d] vertices."""
    v = np.asarray(verts, dtype=np.float64)
    return np.ascontiguousarray(v.reshape(-1, 1))


def _soa(cells_verts):
    """SoA coordinates [(d+1)*d][cells] from [cells][d+1][d]."""
    v = np.asarray(cells_verts, dtype=np.float64)
    return np.ascontiguousarray(v.reshape(v.shape[0], -1).T)


REF = {2: [[0, 0], [1, 0], [0, 1]], 3: [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]}


# ------------------------------------------------------------------ quadrature ---

@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("m", [1, 2, 3, 5])
def test_simplex_rule_integrates_monomials(dim, m):
    """Collapsed Gauss-Legendre rule vs the Dirichlet integral int_K0 X^a = a!/(|a|+d)!,
    for every monomial of total degree <= 2m - 1 - (d - 1)."""
    pts, wts = oracle.simplex_rule(dim, m)
    pmax = 2 * m - 1 - (dim - 1)
    if pmax < 0:
        pytest.skip("rule exact for no degree at this m (the Duffy Jacobian needs more points)")
    for a in itertools.product(range(pmax + 1), repeat=dim):
        if sum(a) > pmax:
            continue
        exact_val = math.prod(math.factorial(x) for x in a) / math.factorial(sum(a) + dim)
        approx = np.sum(wts * np.prod(pts ** np.array(a), axis=1))
        assert abs(approx - exact_val) <= 1e-15 + 1e-13 * exact_val, (a, approx, exact_val)


# ----------------------------------------------------------------------- basis ---

@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_lagrange_property_and_partition_of_unity(dim, q):
    nd = oracle.nodes(dim, q)
    assert len(nd) == math.comb(q + dim, dim)
    assert np.all(nd.sum(axis=1) == q)
    assert len({tuple(r) for r in nd}) == len(nd)
    X = nd[:, 1:].astype(np.float64) / q  # Cartesian reference coordinates of the nodes
    phi, dphi = oracle.basis(dim, q, X)
    assert np.allclose(phi, np.eye(len(nd)), atol=1e-13)
    rng = np.random.default_rng(0)
    Y = rng.dirichlet(np.ones(dim + 1), size=7)[:, 1:]
    phi, dphi = oracle.basis(dim, q, Y)
    assert np.allclose(phi.sum(axis=1), 1.0, atol=1e-13)
    assert np.allclose(dphi.sum(axis=1), 0.0, atol=1e-11)
    # gradients vs central differences
    h = 1e-6
    for b in range(dim):
        e = np.zeros(dim)
        e[b] = h
        fp, _ = oracle.basis(dim, q, Y + e)
        fm, _ = oracle.basis(dim, q, Y - e)
        assert np.allclose((fp - fm) / (2 * h), dphi[:, :, b], atol=1e-6)


def test_dof_order_p3_triangle():
    """The written dof convention: vertices, edge 0 = (1,2), edge 1 = (0,2), edge 2 = (0,1)
    each from the lower to the higher vertex, then the bubble."""
    expected = [(3, 0, 0), (0, 3, 0), (0, 0, 3),
                (0, 2, 1), (0, 1, 2),
                (2, 0, 1), (1, 0, 2),
                (2, 1, 0), (1, 2, 0),
                (1, 1, 1)]
    assert [tuple(r) for r in oracle.nodes(2, 3)] == expected
    assert [tuple(r) for r in exact.node_list(2, 3)] == expected


def test_dof_order_p2_tet():
    expected = [(2, 0, 0, 0), (0, 2, 0, 0), (0, 0, 2, 0), (0, 0, 0, 2),
                (0, 0, 1, 1), (0, 1, 0, 1), (0, 1, 1, 0), (1, 0, 0, 1), (1, 0, 1, 0), (1, 1, 0, 0)]
    assert [tuple(r) for r in oracle.nodes(3, 2)] == expected
    assert [tuple(r) for r in exact.node_list(3, 2)] == expected


@pytest.mark.parametrize("dim,q", [(2, 4), (3, 3), (3, 4)])
def test_dof_order_agrees_between_oracle_evaluators(dim, q):
    assert [tuple(r) for r in oracle.nodes(dim, q)] == list(exact.node_list(dim, q))


# ---------------------------------------------------------------- closed forms ---

def test_p1_laplacian_reference_triangle_golden():
    gold = np.loadtxt(os.path.join(GOLDEN, "p1_laplacian_reference_triangle.txt"))
    A = oracle.tabulate("laplace", 2, 1, _coords_of(REF[2]))[0]
    assert np.max(np.abs(A - gold)) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_p1_mass_closed_form(dim):
    """P1 mass: |K|/12 (1 + delta_ij) in 2D, |K|/20 (1 + delta_ij) in 3D."""
    rng = np.random.default_rng(5)
    v = np.array(REF[dim], dtype=float) * 0.7 + rng.uniform(-0.1, 0.1, size=(dim + 1, dim))
    vol = abs(np.linalg.det(v[1:] - v[0])) / math.factorial(dim)
    A = oracle.tabulate("mass", dim, 1, _coords_of(v))[0]
    denom = 12.0 if dim == 2 else 20.0
    expect = vol / denom * (np.ones((dim + 1, dim + 1)) + np.eye(dim + 1))
    assert np.max(np.abs(A - expect)) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_p1_laplacian_closed_form(dim):
    """P1 Laplacian: |K| grad(lambda_i) . grad(lambda_j) with the barycentric gradients
    read off the inverse of [[x^0..x^d],[1..1]]."""
    rng = np.random.default_rng(6)
    v = np.array(REF[dim], dtype=float) * 1.3 + rng.uniform(-0.2, 0.2, size=(dim + 1, dim))
    M = np.vstack([v.T, np.ones(dim + 1)])
    grads = np.linalg.inv(M)[:, :dim]
    vol = abs(np.linalg.det(M)) / math.factorial(dim)
    A = oracle.tabulate("laplace", dim, 1, _coords_of(v))[0]
    assert np.allclose(A, vol * grads @ grads.T, rtol=0, atol=1e-14)


def test_paper_p3_triangle_reference_values():
    """Fit the reference-tensor coefficients of entries 0, 1, 2, 99 of the P3 triangle
    Poisson tensor from oracle element tensors on three cells and compare with the values
    printed in the paper's generated-code listing.  G is symmetric, so c_01 + c_10 is
    what the data determine."""
    rows = np.loadtxt(os.path.join(GOLDEN, "poisson_p3_triangle_reference_tensor.txt"))
    cells = [
        [[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]],
        [[0.1, 0.2], [1.3, 0.1], [0.4, 0.9]],
        [[0.0, 0.0], [0.8, 0.3], [-0.2, 1.1]],
        [[0.3, -0.1], [1.0, 0.4], [0.1, 0.7]],
    ]
    A = oracle.tabulate("laplace", 2, 3, _soa(cells)).reshape(len(cells), -1)
    feats = []
    for v in cells:
        v = np.asarray(v)
        J = (v[1:] - v[0]).T
        g = np.linalg.inv(J)
        det = np.linalg.det(J)
        G = det * g @ g.T
        feats.append([G[0, 0], G[0, 1] + G[1, 0], G[1, 1]])
    feats = np.array(feats)
    for row in rows:
        k = int(row[0])
        c00, c01, c10, c11 = row[1:]
        sol, *_ = np.linalg.lstsq(feats, A[:, k], rcond=None)
        # with symmetric G only c01 + c10 is identified (each printed G01/G10 pair is
        # the same value up to rounding, so it is split evenly between the two)
        expect = np.array([c00, 0.5 * (c01 + c10), c11])
        assert np.allclose(sol, expect, rtol=0, atol=1e-12), (k, sol, expect)


# ------------------------------------------------------------ exact rationals ---

def _rational_cell(dim, seed):
    rnd = random.Random(seed)
    base = REF[dim]
    scale = Fraction(rnd.randint(20, 40), 37)
    return [[Fraction(c) * scale + Fraction(rnd.randint(-6, 6), 53) for c in v] for v in base]


def _compare_exact(kind, dim, q, seed, coeffs=None, tol=2e-14):
    verts = _rational_cell(dim, seed)
    E = np.array([[float(x) for x in row] for row in exact.element_tensor(kind, verts, q, coeffs)])
    coords = _coords_of([[float(c) for c in v] for v in verts])
    C = None if coeffs is None else np.array([float(c) for c in coeffs]).reshape(-1, 1)
    A = oracle.tabulate(kind, dim, q, coords, C)[0]
    err = np.max(np.abs(A - E)) / np.max(np.abs(E))
    assert err < tol, (kind, dim, q, err)


@pytest.mark.parametrize("dim,q", [(2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2), (3, 3)])
def test_mass_and_laplace_vs_exact(dim, q):
    _compare_exact("mass", dim, q, seed=10 * dim + q)
    _compare_exact("laplace", dim, q, seed=100 + 10 * dim + q)


@pytest.mark.parametrize("dim,q", [(2, 2), (3, 3)])
def test_wlaplace_vs_exact(dim, q):
    w = [Fraction(k + 2, 3 + k) for k in range(dim + 1)]
    _compare_exact("wlaplace", dim, q, seed=7, coeffs=w)


@pytest.mark.parametrize("dim,q", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_elasticity_vs_exact(dim, q):
    _compare_exact("elasticity", dim, q, seed=11 + dim + q)


@pytest.mark.parametrize("dim", [2, 3])
def test_ns_vs_exact(dim):
    rnd = random.Random(3)
    w = [Fraction(rnd.randint(-9, 9), 7) for _ in range(dim * (dim + 1))]
    _compare_exact("ns", dim, 2, seed=21 + dim, coeffs=w)


def test_exact_p4_triangle_laplace_and_p4_tet_mass():
    _compare_exact("laplace", 2, 4, seed=99)
    _compare_exact("mass", 3, 4, seed=98)


# ------------------------------------------------------------------ invariants ---

def _jittered_cells(dim, ncell, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    base = np.array(REF[dim], dtype=float)
    out = []
    for _ in range(ncell):
        R = np.linalg.qr(rng.standard_normal((dim, dim)))[0]
        v = (base @ R.T) * rng.uniform(0.3, 2.0) + rng.uniform(-1, 1, size=dim)
        v = v + rng.uniform(-scale, scale, size=v.shape) * 0.3
        # keep positive orientation
        if np.linalg.det(v[1:] - v[0]) < 0:
            v[[1, 2]] = v[[2, 1]]
        out.append(v)
    return np.array(out)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("q", [1, 2, 3])
def test_symmetry_rowsums_mass_total(dim, q):
    cells = _jittered_cells(dim, 5, seed=q)
    X = _soa(cells)
    vol = np.abs(np.linalg.det(cells[:, 1:] - cells[:, :1])) / math.factorial(dim)
    M = oracle.tabulate("mass", dim, q, X)
    L = oracle.tabulate("laplace", dim, q, X)
    w = np.random.default_rng(1).uniform(0.5, 2.0, size=(dim + 1, len(cells)))
    W = oracle.tabulate("wlaplace", dim, q, X, w)
    for T in (M, L, W):
        assert np.allclose(T, T.transpose(0, 2, 1), atol=1e-13 * np.abs(T).max())
    assert np.allclose(L.sum(axis=2), 0.0, atol=1e-12 * np.abs(L).max())
    assert np.allclose(W.sum(axis=2), 0.0, atol=1e-12 * np.abs(W).max())
    assert np.allclose(M.sum(axis=(1, 2)), vol, rtol=1e-13)
    # w == 1 reduces the weighted Laplacian to the Laplacian; linear in w
    ones = np.ones((dim + 1, len(cells)))
    assert np.allclose(oracle.tabulate("wlaplace", dim, q, X, ones), L, atol=1e-13 * np.abs(L).max())
    W2 = oracle.tabulate("wlaplace", dim, q, X, 2.0 * w + 0.5 * ones)
    assert np.allclose(W2, 2.0 * W + 0.5 * L, atol=1e-12 * np.abs(W2).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_translation_scaling_rotation(dim):
    cells = _jittered_cells(dim, 3, seed=4)
    X = _soa(cells)
    shift = np.array([0.37, -1.2, 2.5][:dim])
    s = 1.7
    R = np.linalg.qr(np.random.default_rng(2).standard_normal((dim, dim)))[0]
    if np.linalg.det(R) < 0:
        R[:, 0] *= -1
    for kind, q, power in (("mass", 2, dim), ("laplace", 3, dim - 2)):
        A = oracle.tabulate(kind, dim, q, X)
        At = oracle.tabulate(kind, dim, q, _soa(cells + shift))
        As = oracle.tabulate(kind, dim, q, _soa(cells * s))
        Ar = oracle.tabulate(kind, dim, q, _soa(cells @ R.T))
        tol = 1e-12 * np.abs(A).max()
        assert np.allclose(At, A, atol=tol)
        assert np.allclose(As, s ** power * A, atol=tol * s ** max(power, 0) * 10)
        assert np.allclose(Ar, A, atol=tol)


def _nodal_points(cell, dim, q):
    nd = oracle.nodes(dim, q).astype(float) / q  # barycentric
    return nd @ cell  # physical node coordinates [n, d]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("q", [1, 2])
def test_elasticity_rigid_body_kernel_and_rotation(dim, q):
    cells = _jittered_cells(dim, 3, seed=8)
    A = oracle.tabulate("elasticity", dim, q, _soa(cells))
    ns = len(oracle.nodes(dim, q))
    scale = np.abs(A).max()
    for c, cell in enumerate(cells):
        P = _nodal_points(cell, dim, q)
        modes = []
        for k in range(dim):  # translations
            u = np.zeros((dim, ns))
            u[k] = 1.0
            modes.append(u.reshape(-1))
        pairs = [(0, 1)] if dim == 2 else [(0, 1), (0, 2), (1, 2)]
        for a, b in pairs:  # infinitesimal rotations, exact in P_q for q >= 1
            u = np.zeros((dim, ns))
            u[a] = -P[:, b]
            u[b] = P[:, a]
            modes.append(u.reshape(-1))
        for u in modes:
            assert np.max(np.abs(A[c] @ u)) < 1e-12 * scale * (1 + np.abs(u).max())
    # rotating the cell rotates the vector dofs: A(RK) = (R x I) A(K) (R x I)^T
    R = np.linalg.qr(np.random.default_rng(3).standard_normal((dim, dim)))[0]
    if np.linalg.det(R) < 0:
        R[:, 0] *= -1
    Ar = oracle.tabulate("elasticity", dim, q, _soa(cells @ R.T))
    T = np.kron(R, np.eye(ns))
    for c in range(len(cells)):
        assert np.allclose(Ar[c], T @ A[c] @ T.T, atol=1e-12 * scale)


@pytest.mark.parametrize("dim", [2, 3])
def test_ns_constant_trial_fields_and_linearity(dim):
    cells = _jittered_cells(dim, 3, seed=9)
    X = _soa(cells)
    rng = np.random.default_rng(4)
    w1 = rng.standard_normal((dim * (dim + 1), len(cells)))
    w2 = rng.standard_normal((dim * (dim + 1), len(cells)))
    A1 = oracle.tabulate("ns", dim, 2, X, w1)
    A2 = oracle.tabulate("ns", dim, 2, X, w2)
    A12 = oracle.tabulate("ns", dim, 2, X, 3.0 * w1 - w2)
    scale = np.abs(A12).max()
    assert np.allclose(A12, 3.0 * A1 - A2, atol=1e-12 * scale)
    assert np.max(np.abs(oracle.tabulate("ns", dim, 2, X, np.zeros_like(w1)))) == 0.0
    ns = len(oracle.nodes(dim, 2))
    for k in range(dim):
        u = np.zeros((dim, ns))
        u[k] = 1.0
        assert np.max(np.abs(A1 @ u.reshape(-1))) < 1e-12 * scale
    # w = constant vector c, u = linear field x_j e_k: (w.grad)u = c_j e_k, so A u = M-ish
    # load: int v . c_j e_k = c_j * (row sums of the mass matrix of the k block)
    c = rng.standard_normal(dim)
    wc = np.repeat(c, dim + 1)[:, None] * np.ones((1, len(cells)))
    Ac = oracle.tabulate("ns", dim, 2, X, wc)
    M = oracle.tabulate("mass", dim, 2, X)
    for cc, cell in enumerate(cells):
        P = _nodal_points(cell, dim, 2)
        for j in range(dim):
            for k in range(dim):
                u = np.zeros((dim, ns))
                u[k] = P[:, j]
                got = (Ac[cc] @ u.reshape(-1)).reshape(dim, ns)
                want = np.zeros((dim, ns))
                want[k] = c[j] * M[cc].sum(axis=1)
                assert np.allclose(got, want, atol=1e-12 * scale)


def test_orientation_reversal_unchanged():
    cells = _jittered_cells(3, 2, seed=12)
    X = _soa(cells)
    rev = cells[:, [0, 2, 1, 3]]  # swapping two vertices flips the sign of det J
    # swapping vertices 1 and 2 permutes the dofs; compare P1, where dofs are vertices
    A = oracle.tabulate("laplace", 3, 1, X)
    B = oracle.tabulate("laplace", 3, 1, _soa(rev))
    perm = [0, 2, 1, 3]
    assert np.allclose(B, A[:, perm][:, :, perm], atol=1e-13 * np.abs(A).max())


# --------------------------------------------------------- badly shaped cells ---

@pytest.mark.parametrize("shape", ["needle", "sliver"])
@pytest.mark.parametrize("kind,dim,q", [("mass", 3, 1), ("laplace", 3, 2), ("laplace", 2, 2)])
def test_oracle_accuracy_on_badly_shaped_cells(kind, dim, q, shape):
    """The oracle against exact rationals of the same binary coordinates on needles and
    slivers: within 1e-12 up to Jacobian condition number 100, and within 1e-11 at 1000
    (its cofactor inverse loses digits on 3D needles, ~4e-12 measured).  This is why the GPU
    tests on such cells compare with exact arithmetic rather than with the oracle."""
    from paper_1112_0402_amd import meshgen

    for aspect, tol in ((10.0, 1e-12), (100.0, 1e-12), (1000.0, 1e-11)):
        c = meshgen.badly_shaped(dim, 12, aspect, shape, seed=5)
        O = oracle.tabulate(kind, dim, q, c)
        E = np.array([[[float(x) for x in r] for r in exact.element_tensor(
            kind, [[Fraction(float(c[v * dim + k, i])) for k in range(dim)] for v in range(dim + 1)], q)]
            for i in range(c.shape[1])])
        err = np.linalg.norm((O - E).reshape(len(E), -1), axis=1) / np.linalg.norm(E.reshape(len(E), -1), axis=1)
        assert err.max() <= tol, (aspect, err.max())
