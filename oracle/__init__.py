"""Element-tensor oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check (``__graft_entry__.smoke``) and the CPU-baseline leg of
``bench.py`` import this package.  The product path (the HIP library and its Python
binding) never imports, links or executes anything here, and this package never imports
the product.

Two independent evaluators of the element tensor A^K (element matrix, Sec. 2.2; element
tensor of a multilinear form, Sec. 3.1):

* ``tabulate`` -- plain C, FP64, OpenMP over cells: the defining integral on the
  physical cell by a collapsed Gauss-Legendre product rule that is exact for the
  integrand's polynomial degree (``ffc_oracle.c`` states every convention);
* ``exact.element_tensor`` -- pure-Python exact rational arithmetic on one cell with
  rational vertices (the pin for ``tabulate``).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

KINDS = {"mass": 0, "laplace": 1, "wlaplace": 2, "elasticity": 3, "ns": 4}

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ffc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP) into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_tabulate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_longlong, dp, dp, dp, ctypes.c_int]
        L.oracle_tabulate.restype = ctypes.c_int
        L.oracle_n_dofs.argtypes = [ctypes.c_int] * 3
        L.oracle_n_dofs.restype = ctypes.c_int
        L.oracle_n_coeffs.argtypes = [ctypes.c_int] * 2
        L.oracle_n_coeffs.restype = ctypes.c_int
        L.oracle_simplex_rule.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.oracle_simplex_rule.restype = ctypes.c_int
        L.oracle_nodes.argtypes = [ctypes.c_int, ctypes.c_int, ip]
        L.oracle_nodes.restype = ctypes.c_int
        L.oracle_basis.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.oracle_basis.restype = ctypes.c_int
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def n_dofs(kind: str, dim: int, degree: int) -> int:
    return lib().oracle_n_dofs(KINDS[kind], dim, degree)


def n_coeffs(kind: str, dim: int) -> int:
    return lib().oracle_n_coeffs(KINDS[kind], dim)


def max_threads() -> int:
    return lib().oracle_max_threads()


def tabulate(kind: str, dim: int, degree: int, coords, coeffs=None, lam: float = 1.0, mu: float = 1.0,
             nthreads: int = 0) -> np.ndarray:
    """Element tensors [cells, n, n] (row = test function) in FP64."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    assert coords.ndim == 2 and coords.shape[0] == (dim + 1) * dim
    cells = coords.shape[1]
    n = n_dofs(kind, dim, degree)
    if n < 0:
        raise ValueError(f"unsupported form {kind} dim={dim} degree={degree}")
    nc = n_coeffs(kind, dim)
    cptr = None
    if nc:
        if coeffs is None:
            raise ValueError(f"form {kind} needs {nc} coefficients per cell")
        coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
        assert coeffs.shape == (nc, cells)
        cptr = _dp(coeffs)
    out = np.empty((cells, n, n), dtype=np.float64)
    rc = lib().oracle_tabulate(KINDS[kind], dim, degree, lam, mu, cells, _dp(coords), cptr, _dp(out), nthreads)
    if rc != 0:
        raise RuntimeError(f"oracle_tabulate failed ({rc})")
    return out


def simplex_rule(dim: int, m: int):
    pts = np.zeros((m ** dim, dim))
    wts = np.zeros(m ** dim)
    npts = lib().oracle_simplex_rule(dim, m, _dp(pts), _dp(wts))
    assert npts == m ** dim
    return pts, wts


def nodes(dim: int, degree: int) -> np.ndarray:
    buf = np.zeros((64, 4), dtype=np.int32)
    nn = lib().oracle_nodes(dim, degree, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return buf[:nn, : dim + 1].copy()


def basis(dim: int, degree: int, X) -> tuple[np.ndarray, np.ndarray]:
    X = np.ascontiguousarray(np.atleast_2d(X), dtype=np.float64)
    npts = X.shape[0]
    nn = len(nodes(dim, degree))
    phi = np.zeros((npts, nn))
    dphi = np.zeros((npts, nn, dim))
    lib().oracle_basis(dim, degree, npts, _dp(X), _dp(phi), _dp(dphi))
    return phi, dphi


def source_vector(dim: int, degree: int, coords, f) -> np.ndarray:
    """Element vectors of the linear form L(v) = int_K f v dx (the right-hand side of the
    Poisson form file, Sec. 5.5), f in the same Lagrange P_q space as v given by its nodal
    values f [cells, n] in the dof order: b[c, i] = sum_q w_q |det J| phi_i(X_q) f(X_q) on the
    physical cell (affine map of Sec. 3.2), with a collapsed rule exact for degree 2q."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cells = coords.shape[1]
    f = np.asarray(f, dtype=np.float64).reshape(cells, -1)
    X = coords.reshape(dim + 1, dim, cells)          # [vertex][component][cell]
    J = np.transpose(X[1:] - X[0], (2, 1, 0))        # [cell][k][b] = x^{b+1}_k - x^0_k
    adet = np.abs(np.linalg.det(J))
    pts, wts = simplex_rule(dim, degree + 2)
    phi, _ = basis(dim, degree, pts)                 # [point][dof]
    fq = f @ phi.T                                   # f at the points, [cell][point]
    return adet[:, None] * ((fq * wts) @ phi)


def piola_mass(dim: int, coords) -> np.ndarray:
    """Mass matrices [cells, d+1, d+1] of the lowest-order Raviart-Thomas space (the H(div)
    example of Sec. 3.4), written on the physical cell: basis psi_i(x) = (x - x^i) / (d |K|),
    the field of unit flux through the facet opposite vertex i, M_ij = int_K psi_i . psi_j dx
    by a collapsed rule exact for degree 2, mapped to K (weights |det J|)."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cells = coords.shape[1]
    X = coords.reshape(dim + 1, dim, cells)          # [vertex][component][cell]
    J = np.transpose(X[1:] - X[0], (2, 1, 0))        # [cell][k][b] = x^{b+1}_k - x^0_k
    adet = np.abs(np.linalg.det(J))
    vol = adet / math.factorial(dim)
    pts, wts = simplex_rule(dim, 3)
    xq = X[0].T[:, None, :] + np.einsum("ckb,qb->cqk", J, pts)          # [cell][point][k]
    psi = (xq[:, None, :, :] - np.transpose(X, (2, 0, 1))[:, :, None, :]) / (dim * vol)[:, None, None, None]
    return np.einsum("ciqk,cjqk,q->cij", psi, psi, wts) * adet[:, None, None]


def collapsed_rule(dim: int, m: int):
    """Collapsed Gauss-Jacobi rule on the reference simplex, m points per direction: the
    direction collapsed k times carries the Jacobi weight (1 - s)^k on [0, 1] (scipy's
    Gauss-Jacobi nodes on [-1, 1] mapped to [0, 1]).  Exact for degree 2m - 1."""
    from scipy.special import roots_jacobi

    rules = []
    for a in range(dim):
        t, w = roots_jacobi(m, a, 0)
        rules.append(((1.0 + t) / 2.0, w / 2.0 ** (a + 1)))
    pts, wts = [], []
    if dim == 2:
        for i in range(m):
            for j in range(m):
                s1, s2 = rules[0][0][i], rules[1][0][j]
                pts.append((s1 * (1 - s2), s2))
                wts.append(rules[0][1][i] * rules[1][1][j])
    else:
        for i in range(m):
            for j in range(m):
                for k in range(m):
                    s1, s2, s3 = rules[0][0][i], rules[1][0][j], rules[2][0][k]
                    pts.append((s1 * (1 - s2) * (1 - s3), s2 * (1 - s3), s3))
                    wts.append(rules[0][1][i] * rules[1][1][j] * rules[2][1][k])
    return np.array(pts), np.array(wts)


def curved_laplace(dim: int, degree: int, coords, m: int | None = None) -> np.ndarray:
    """Element matrices [cells, n, n] of int grad u . grad v on cells with P2 geometry (the
    curvilinear elements of Sec. 3.4): x(X) = sum_k x_k Psi_k(X) over the P2 nodes, and the
    integral taken as the sum over the points of the collapsed rule with m = degree + 1
    points per direction, w_p |det J| (J^{-T} grad Phi_i) . (J^{-T} grad Phi_j) at X_p.
    coords: SoA [n_geo * d][cells], nodes in the P2 dof order."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cells = coords.shape[1]
    m = degree + 1 if m is None else m
    pts, wts = collapsed_rule(dim, m)
    _, dpsi = basis(dim, 2, pts)          # [p][k][b]
    _, dphi = basis(dim, degree, pts)     # [p][i][b]
    ng = dpsi.shape[1]
    x = coords.reshape(ng, dim, cells)    # [k][j][c]
    J = np.einsum("kjc,pkb->cpjb", x, dpsi)
    det = np.linalg.det(J)                # [c][p]
    Jinv = np.linalg.inv(J)               # [c][p][b][j]
    grad = np.einsum("cpbj,pib->cpij", Jinv, dphi)   # physical gradients [c][p][i][j]
    return np.einsum("cpij,cpkj,p,cp->cik", grad, grad, wts, np.abs(det))


NEDELEC_EDGES = {2: ((1, 2), (0, 2), (0, 1)), 3: ((2, 3), (1, 3), (1, 2), (0, 3), (0, 2), (0, 1))}


def nedelec_mass(dim: int, coords) -> np.ndarray:
    """Mass matrices [cells, n_edges, n_edges] of the lowest-order Nedelec (Whitney edge)
    space (the H(curl) side of Sec. 3.4), written on the physical cell: edge (a, b), a < b,
    carries phi = lambda_a grad lambda_b - lambda_b grad lambda_a with the physical
    barycentric coordinates; M_ij = int_K phi_i . phi_j by a collapsed rule exact for degree 3,
    mapped to K (weights |det J|)."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cells = coords.shape[1]
    X = np.transpose(coords.reshape(dim + 1, dim, cells), (2, 0, 1))   # [c][v][k]
    T = np.concatenate([np.transpose(X, (0, 2, 1)), np.ones((cells, 1, dim + 1))], axis=1)  # [x; 1]
    gl = np.linalg.inv(T)[:, :, :dim]                                    # [c][v][k] = d lambda_v / d x_k
    adet = np.abs(np.linalg.det(X[:, 1:, :] - X[:, :1, :]))
    pts, wts = collapsed_rule(dim, 2)
    lam = np.concatenate([1.0 - pts.sum(axis=1, keepdims=True), pts], axis=1)  # [p][v] (affine: same in K)
    phi = np.stack([lam[None, :, a, None] * gl[:, None, b, :] - lam[None, :, b, None] * gl[:, None, a, :]
                    for a, b in NEDELEC_EDGES[dim]], axis=1)                 # [c][e][p][k]
    return np.einsum("cipk,cjpk,p->cij", phi, phi, wts) * adet[:, None, None]
