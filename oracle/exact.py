"""Exact rational element tensors on one cell -- TEST INFRASTRUCTURE ONLY (a pin for the
C oracle; the product never imports this).

Everything is done in ``fractions.Fraction`` arithmetic on polynomials in the barycentric
coordinates lambda_0..lambda_d of the physical cell K, so no quadrature and no floating
point is involved:

* Lagrange P_q basis by the barycentric product formula at the equispaced nodes
  (Sec. 5.3: nodes given by point evaluation), nodes listed in the dof order written out
  in ``ffc_oracle.c`` (re-implemented here, not imported);
* physical derivatives from the barycentric gradients, which are the first d columns of
  the inverse of the (d+1)x(d+1) matrix [[x^0 ... x^d], [1 ... 1]];
* the integral of a barycentric monomial over a simplex (the Dirichlet integral):
  int_K lambda^a dx = d! |K| prod(a_v!) / (|a| + d)!,  with d! |K| = |det [[x^v],[1]]|.

The element tensor is the defining integral A^K_{i1 i2} = a_K(phi_{i1}, phi_{i2})
(element matrix, Sec. 2.2; test cases 1-4, Sec. 3.3), row = test function.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import factorial


# ------------------------------------------------------------ polynomial algebra ----
# A polynomial is a dict {exponent tuple (len d+1): Fraction}.

def padd(p, r, s=Fraction(1)):
    out = dict(p)
    for k, v in r.items():
        out[k] = out.get(k, Fraction(0)) + s * v
        if out[k] == 0:
            del out[k]
    return out


def pmul(p, r):
    out = {}
    for k1, v1 in p.items():
        for k2, v2 in r.items():
            k = tuple(a + b for a, b in zip(k1, k2))
            out[k] = out.get(k, Fraction(0)) + v1 * v2
    return {k: v for k, v in out.items() if v != 0}


def pscale(p, s):
    return {k: v * s for k, v in p.items() if v * s != 0}


def pdiff(p, v):
    out = {}
    for k, c in p.items():
        if k[v] > 0:
            kk = list(k)
            kk[v] -= 1
            kk = tuple(kk)
            out[kk] = out.get(kk, Fraction(0)) + c * k[v]
    return {k: c for k, c in out.items() if c != 0}


def const(d, c):
    return {tuple([0] * (d + 1)): Fraction(c)} if c != 0 else {}


def lam(d, v):
    e = [0] * (d + 1)
    e[v] = 1
    return {tuple(e): Fraction(1)}


# ------------------------------------------------------------------ the element ----

def _interior(q, s):
    """Points strictly inside the sub-simplex with sorted vertex list s, ascending
    lexicographically in (b_1, ..., b_m)."""
    m = len(s) - 1
    pts = []

    def rec(prefix):
        if len(prefix) == m:
            b0 = q - sum(prefix)
            if b0 >= 1:
                pts.append((b0,) + tuple(prefix))
            return
        for b in range(1, q):
            rec(prefix + [b])

    rec([])
    return pts


@lru_cache(maxsize=None)
def node_list(d, q):
    nodes = []
    for v in range(d + 1):
        a = [0] * (d + 1)
        a[v] = q
        nodes.append(tuple(a))
    if d == 2:
        subs = [(1, 2), (0, 2), (0, 1), (0, 1, 2)]
    else:
        subs = [(2, 3), (1, 3), (1, 2), (0, 3), (0, 2), (0, 1),
                (1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2), (0, 1, 2, 3)]
    for s in subs:
        for b in _interior(q, s):
            a = [0] * (d + 1)
            for vert, bv in zip(s, b):
                a[vert] = bv
            nodes.append(tuple(a))
    return tuple(nodes)


@lru_cache(maxsize=None)
def basis_polys(d, q):
    """Lagrange basis as barycentric polynomials: prod_v prod_{k<a_v} (q lam_v - k)/(k+1)."""
    out = []
    for a in node_list(d, q):
        p = const(d, 1)
        for v in range(d + 1):
            for k in range(a[v]):
                factor = padd(pscale(lam(d, v), Fraction(q, k + 1)), const(d, Fraction(-k, k + 1)))
                p = pmul(p, factor)
        out.append(p)
    return tuple(out)


def _inverse(M):
    """Exact inverse of a small square Fraction matrix by Gauss-Jordan."""
    n = len(M)
    A = [list(map(Fraction, row)) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(M)]
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        pv = A[col][col]
        A[col] = [x / pv for x in A[col]]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [x - f * y for x, y in zip(A[r], A[col])]
    return [row[n:] for row in A]


def _det(M):
    n = len(M)
    A = [list(map(Fraction, row)) for row in M]
    det = Fraction(1)
    for col in range(n):
        piv = next((r for r in range(col, n) if A[r][col] != 0), None)
        if piv is None:
            return Fraction(0)
        if piv != col:
            A[col], A[piv] = A[piv], A[col]
            det = -det
        det *= A[col][col]
        for r in range(col + 1, n):
            f = A[r][col] / A[col][col]
            A[r] = [x - f * y for x, y in zip(A[r], A[col])]
    return det


class Cell:
    """An affine simplex with rational vertices x[v][k]."""

    def __init__(self, verts):
        self.verts = [[Fraction(c) for c in v] for v in verts]
        self.d = len(self.verts) - 1
        d = self.d
        M = [[self.verts[v][k] for v in range(d + 1)] for k in range(d)] + [[Fraction(1)] * (d + 1)]
        self.absdet = abs(_det(M))  # = d! |K|
        Minv = _inverse(M)
        # lambda = Minv [x; 1]  ->  d lambda_v / d x_k = Minv[v][k]
        self.dlam = [[Minv[v][k] for k in range(d)] for v in range(d + 1)]

    def integrate(self, p):
        d = self.d
        total = Fraction(0)
        for a, c in p.items():
            num = 1
            for av in a:
                num *= factorial(av)
            total += c * Fraction(num, factorial(sum(a) + d))
        return total * self.absdet

    def grad(self, p):
        """Physical gradient of a barycentric polynomial: list of d polynomials."""
        d = self.d
        dl = [pdiff(p, v) for v in range(d + 1)]
        out = []
        for k in range(d):
            g = {}
            for v in range(d + 1):
                if self.dlam[v][k] != 0 and dl[v]:
                    g = padd(g, dl[v], self.dlam[v][k])
            out.append(g)
        return out


def p1_field(d, values):
    """P1 function with given vertex values: sum_t w_t lambda_t."""
    p = {}
    for t, w in enumerate(values):
        p = padd(p, lam(d, t), Fraction(w))
    return p


def element_tensor(kind, verts, degree, coeffs=None, lam_=1, mu=1):
    """Exact element tensor as a list of lists of Fractions (row = test function).
    coeffs: wlaplace -> d+1 vertex values; ns -> d*(d+1) values, index comp*(d+1)+vertex."""
    K = Cell(verts)
    d = K.d
    basis = basis_polys(d, degree)
    ns = len(basis)
    grads = [K.grad(p) for p in basis]
    lam_ = Fraction(lam_)
    mu = Fraction(mu)

    if kind in ("mass", "laplace", "wlaplace"):
        w = p1_field(d, coeffs) if kind == "wlaplace" else None
        A = [[Fraction(0)] * ns for _ in range(ns)]
        for i in range(ns):
            for j in range(ns):
                if kind == "mass":
                    integrand = pmul(basis[i], basis[j])
                else:
                    integrand = {}
                    for k in range(d):
                        integrand = padd(integrand, pmul(grads[i][k], grads[j][k]))
                    if w is not None:
                        integrand = pmul(integrand, w)
                A[i][j] = K.integrate(integrand)
        return A

    n = d * ns
    A = [[Fraction(0)] * n for _ in range(n)]
    if kind == "elasticity":
        # strain of phi_s e_c: eps_ab = (delta_ac d_b phi + delta_bc d_a phi) / 2
        def strain(c, s):
            E = [[{} for _ in range(d)] for _ in range(d)]
            for a in range(d):
                for b in range(d):
                    e = {}
                    if a == c:
                        e = padd(e, grads[s][b], Fraction(1, 2))
                    if b == c:
                        e = padd(e, grads[s][a], Fraction(1, 2))
                    E[a][b] = e
            return E

        strains = {(c, s): strain(c, s) for c in range(d) for s in range(ns)}
        for c1 in range(d):
            for s1 in range(ns):
                ev = strains[(c1, s1)]
                for c2 in range(d):
                    for s2 in range(ns):
                        eu = strains[(c2, s2)]
                        tr = {}
                        for a in range(d):
                            tr = padd(tr, eu[a][a])
                        integrand = {}
                        for a in range(d):
                            for b in range(d):
                                sig = pscale(eu[a][b], 2 * mu)
                                if a == b:
                                    sig = padd(sig, tr, lam_)
                                integrand = padd(integrand, pmul(sig, ev[a][b]))
                        A[c1 * ns + s1][c2 * ns + s2] = K.integrate(integrand)
        return A

    if kind == "ns":
        wk = [p1_field(d, coeffs[k * (d + 1):(k + 1) * (d + 1)]) for k in range(d)]
        for c1 in range(d):
            for s1 in range(ns):
                for s2 in range(ns):
                    # (w . grad) phi_s2, same for every component
                    conv = {}
                    for k in range(d):
                        conv = padd(conv, pmul(wk[k], grads[s2][k]))
                    val = K.integrate(pmul(basis[s1], conv))
                    A[c1 * ns + s1][c1 * ns + s2] = val
        return A
    raise ValueError(kind)


def source_vector(verts, degree, fvals):
    """Exact element vector of L(v) = int_K f v dx for f = sum_a f_a phi_a in the same P_q
    space (nodal values f_a in the dof order): b_i = int_K phi_i f, as Fractions."""
    K = Cell(verts)
    basis = basis_polys(K.d, degree)
    fp = {}
    for a, fa in enumerate(fvals):
        fp = padd(fp, basis[a], Fraction(fa))
    return [K.integrate(pmul(basis[i], fp)) for i in range(len(basis))]


def piola_mass(verts):
    """Exact lowest-order Raviart-Thomas mass matrix on a rational cell: psi_i =
    (x - x^i) / (d |K|) with x = sum_v lambda_v x^v, M_ij = int_K psi_i . psi_j, as Fractions."""
    K = Cell(verts)
    d = K.d
    vol = K.absdet / factorial(d)
    comp = [[{} for _ in range(d)] for _ in range(d + 1)]  # comp[i][k] = x_k - x^i_k
    for i in range(d + 1):
        for k in range(d):
            p = {}
            for v in range(d + 1):
                p = padd(p, lam(d, v), K.verts[v][k] - K.verts[i][k])
            comp[i][k] = p
    M = [[Fraction(0)] * (d + 1) for _ in range(d + 1)]
    for i in range(d + 1):
        for j in range(d + 1):
            s = Fraction(0)
            for k in range(d):
                s += K.integrate(pmul(comp[i][k], comp[j][k]))
            M[i][j] = s / (d * vol) ** 2
    return M


def nedelec_mass(verts):
    """Exact lowest-order Nedelec (Whitney edge) mass matrix on a rational cell: edge (a, b)
    in the P2 edge order carries lambda_a grad lambda_b - lambda_b grad lambda_a, as Fractions."""
    K = Cell(verts)
    d = K.d
    edges = ((1, 2), (0, 2), (0, 1)) if d == 2 else ((2, 3), (1, 3), (1, 2), (0, 3), (0, 2), (0, 1))
    comps = []
    for a, b in edges:
        comps.append([padd(pscale(lam(d, a), K.dlam[b][k]), pscale(lam(d, b), -K.dlam[a][k])) for k in range(d)])
    n = len(edges)
    return [[sum((K.integrate(pmul(comps[i][k], comps[j][k])) for k in range(d)), Fraction(0)) for j in range(n)]
            for i in range(n)]
