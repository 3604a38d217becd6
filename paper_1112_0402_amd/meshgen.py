"""Seeded synthetic meshes and coefficient fields.

This module only generates inputs: vertex coordinates, cell connectivity, the per-cell
structure-of-arrays gathers the tabulation entry points take, and random coefficient
values.  It holds none of the element-tensor arithmetic, so both the HIP path and the
oracle can be fed from it.

Meshes follow the workloads of the paper's benchmarks (Sec. 6: affine simplices, one
million elements per timing) generalised to jittered structured grids:

* 2D: the unit square cut into n x n squares, each split along its (0,0)-(1,1) diagonal
  into two positively oriented triangles;
* 3D: the unit cube cut into n^3 cubes, each split into the six Kuhn tetrahedra (vertex
  chains along the axes in the order of a permutation), reordered to positive orientation;
* every coordinate of every interior vertex is moved by an independent U(-0.2h, 0.2h).

Layouts handed to the library:
* coords: float64 SoA ``[(d+1)*d][cells]``, ``coords[(v*d + k)*cells + c]`` = coordinate k
  of local vertex v of cell c;
* coeffs: float64 SoA ``[n_coeff][cells]``: P1 scalar field -> one value per local vertex;
  P1 vector field -> ``coeffs[(comp*(d+1) + vertex)*cells + c]``.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

JITTER = 0.2


def _grid_vertices(n: int, dim: int, rng: np.random.Generator, jitter: float = JITTER):
    h = 1.0 / n
    axes = [np.arange(n + 1, dtype=np.float64) * h] * dim
    grid = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, dim)
    idx = np.stack(np.meshgrid(*[np.arange(n + 1)] * dim, indexing="ij"), axis=-1).reshape(-1, dim)
    interior = np.all((idx > 0) & (idx < n), axis=1)
    noise = rng.uniform(-jitter * h, jitter * h, size=grid.shape)
    grid = grid + noise * interior[:, None]
    return grid, idx


def unit_square(n: int, seed: int, jitter: float = JITTER):
    """Jittered unit square, 2 n^2 triangles. Returns (vertices [nv,2], cells [nc,3])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    verts, _ = _grid_vertices(n, 2, rng, jitter)

    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    i, j = i.reshape(-1), j.reshape(-1)
    v00, v10 = i * (n + 1) + j, (i + 1) * (n + 1) + j
    v01, v11 = v00 + 1, v10 + 1
    cells = np.empty((2 * n * n, 3), dtype=np.int64)
    cells[0::2] = np.stack([v00, v10, v11], axis=1)
    cells[1::2] = np.stack([v00, v11, v01], axis=1)
    return verts, cells


_PERMS = list(itertools.permutations(range(3)))


def _perm_parity(p):
    inv = 0
    for a in range(3):
        for b in range(a + 1, 3):
            inv += p[a] > p[b]
    return inv % 2


def unit_cube(n: int, seed: int, jitter: float = JITTER, max_cells: int | None = None):
    """Jittered unit cube, 6 n^3 Kuhn tetrahedra. Returns (vertices [nv,3], cells [nc,4])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    verts, _ = _grid_vertices(n, 3, rng, jitter)
    stride = np.array([(n + 1) * (n + 1), n + 1, 1], dtype=np.int64)
    corners = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), axis=-1).reshape(-1, 3)
    base = corners @ stride
    local = []
    for p in _PERMS:
        chain = [np.zeros(3, dtype=np.int64)]
        cur = np.zeros(3, dtype=np.int64)
        for ax in p:
            cur = cur.copy()
            cur[ax] += 1
            chain.append(cur)
        offs = [int(c @ stride) for c in chain]
        if _perm_parity(p) == 1:  # odd permutation: negative orientation, swap two vertices
            offs[2], offs[3] = offs[3], offs[2]
        local.append(offs)
    local = np.array(local, dtype=np.int64)  # [6,4]
    cells = (base[:, None, None] + local[None, :, :]).reshape(-1, 4)
    if max_cells is not None:
        cells = cells[:max_cells]
    return verts, cells


def soa_coords(verts: np.ndarray, cells: np.ndarray) -> np.ndarray:
    """Per-cell SoA coordinates [(d+1)*d][cells], contiguous float64."""
    d = verts.shape[1]
    g = verts[cells]  # [nc, d+1, d]
    return np.ascontiguousarray(g.reshape(cells.shape[0], (d + 1) * d).T)


def signed_volumes_ok(verts: np.ndarray, cells: np.ndarray) -> bool:
    """Input validation: every cell positively oriented."""
    g = verts[cells]
    e = g[:, 1:, :] - g[:, :1, :]
    return bool(np.all(np.linalg.det(e) > 0))


def p1_scalar_coeffs(cells: np.ndarray, vertex_values: np.ndarray) -> np.ndarray:
    """Gather a P1 scalar field given at mesh vertices: SoA [d+1][cells]."""
    return np.ascontiguousarray(vertex_values[cells].T)


def p1_vector_coeffs(cells: np.ndarray, vertex_values: np.ndarray) -> np.ndarray:
    """Gather a P1 vector field [nv, d]: SoA [d*(d+1)][cells], index comp*(d+1)+vertex."""
    nc, nv1 = cells.shape
    d = vertex_values.shape[1]
    g = vertex_values[cells]  # [nc, d+1, d]
    return np.ascontiguousarray(g.transpose(2, 1, 0).reshape(d * nv1, nc))


# --------------------------------------------------------------------------- forms ---

FORM_KINDS = ("mass", "laplace", "wlaplace", "elasticity", "ns", "piola", "nedelec")


@dataclass
class Workload:
    """One mesh with one form: everything a tabulation call needs, on the host."""

    kind: str
    dim: int
    degree: int
    coords: np.ndarray
    coeffs: np.ndarray | None
    lam: float = 1.0
    mu: float = 1.0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return int(self.coords.shape[1])


def _mesh(dim: int, n: int, seed: int, max_cells: int | None = None):
    if dim == 2:
        v, c = unit_square(n, seed)
        if max_cells is not None:
            c = c[:max_cells]
        return v, c
    return unit_cube(n, seed, max_cells=max_cells)


def make_workload(kind, dim, degree, n, seed, max_cells=None, name="", coeff_seed=None, jitter=JITTER):
    """Mesh of side n (2 n^2 or 6 n^3 cells, optionally cut to max_cells) with the
    coefficient field the form needs: wlaplace w ~ U(0.5, 2) per vertex, ns w ~ N(0, 1)
    per vertex and component.  meta holds the topology (cells [nc, d+1] vertex indices,
    n_vertices) for building local-to-global maps."""
    if dim == 2:
        verts, cells = unit_square(n, seed, jitter)
        if max_cells is not None:
            cells = cells[:max_cells]
    else:
        verts, cells = unit_cube(n, seed, jitter, max_cells=max_cells)
    coords = soa_coords(verts, cells)
    rng = np.random.Generator(np.random.PCG64(seed + 7919 if coeff_seed is None else coeff_seed))
    coeffs = None
    if kind == "wlaplace":
        coeffs = p1_scalar_coeffs(cells, rng.uniform(0.5, 2.0, size=verts.shape[0]))
    elif kind == "ns":
        coeffs = p1_vector_coeffs(cells, rng.standard_normal(size=(verts.shape[0], dim)))
    return Workload(kind, dim, degree, coords, coeffs, name=name,
                    meta={"cells": cells, "n_vertices": int(verts.shape[0])})


# ------------------------------------------------------------ local-to-global maps ---
# Topology only (no element arithmetic): a Lagrange node of a cell is named by its
# barycentric lattice index a (a_v >= 0, sum = q) over the cell's vertices; the same
# node seen from any cell sharing it has the same set {(global vertex, a_v) : a_v > 0},
# which serves as its global key.  The local node order is the element tensor's: the
# vertices, then the nodes inside the edges (triangle: edge k opposite vertex k;
# tetrahedron: (2,3), (1,3), (1,2), (0,3), (0,2), (0,1)), the faces (face k opposite
# vertex k), the interior; inside a sub-simplex with local vertices s_0 < ... < s_m,
# ascending lexicographically in the weights of s_1, ..., s_m.

def _lattice_nodes(dim: int, q: int):
    nodes = []
    for v in range(dim + 1):
        a = [0] * (dim + 1)
        a[v] = q
        nodes.append(a)
    if dim == 2:
        subs = [(1, 2), (0, 2), (0, 1), (0, 1, 2)]
    else:
        subs = [(2, 3), (1, 3), (1, 2), (0, 3), (0, 2), (0, 1), (1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2),
                (0, 1, 2, 3)]
    for s in subs:
        m = len(s) - 1
        for tail in itertools.product(range(1, q), repeat=m):  # ascending lexicographic
            b0 = q - sum(tail)
            if b0 >= 1:
                a = [0] * (dim + 1)
                a[s[0]] = b0
                for vert, bv in zip(s[1:], tail):
                    a[vert] = bv
                nodes.append(a)
    return np.array(nodes, dtype=np.int64)


def lagrange_dofmap(cells: np.ndarray, degree: int, components: int = 1):
    """Local-to-global map of the degree-q Lagrange space on a simplicial mesh: (dofmap
    int32 [nc, components * n_s], n_global).  Vector spaces are component-blocked: local
    dof (c, s) = c * n_s + s, global dof = c * N_s + (scalar global dof)."""
    nc, nv1 = cells.shape
    dim = nv1 - 1
    nodes = _lattice_nodes(dim, degree)
    n_s = nodes.shape[0]
    keys = np.full((nc, n_s, 2 * nv1), -1, dtype=np.int64)
    for p, a in enumerate(nodes):
        sup = np.nonzero(a)[0]
        g = cells[:, sup]                        # global vertices carrying the node
        order = np.argsort(g, axis=1, kind="stable")
        gs = np.take_along_axis(g, order, axis=1)
        ws = a[sup][order]
        keys[:, p, 0:2 * len(sup):2] = gs
        keys[:, p, 1:2 * len(sup):2] = ws
    flat = keys.reshape(nc * n_s, 2 * nv1)
    _, inv = np.unique(flat, axis=0, return_inverse=True)
    n_global = int(inv.max()) + 1 if inv.size else 0
    scalar = inv.reshape(nc, n_s).astype(np.int64)
    if components == 1:
        return scalar.astype(np.int32), n_global
    blocks = [scalar + c * n_global for c in range(components)]
    return np.concatenate(blocks, axis=1).astype(np.int32), n_global * components


def config1():
    """2D Poisson, P1 triangles, 64 x 64 squares -> 8192 cells, seed 1."""
    return make_workload("laplace", 2, 1, 64, 1, name="poisson2d_p1_8192")


def config2():
    """3D elasticity (lambda = mu = 1), vector P2 tets, 6 * 50^3 = 750,000 cells, seed 2."""
    return make_workload("elasticity", 3, 2, 50, 2, name="elasticity3d_p2_750k")


def config3():
    """3D weighted Laplacian, P3 tets, w in P1 ~ U(0.5, 2), 6 * 63^3 = 1,500,282 cells, seed 3."""
    return make_workload("wlaplace", 3, 3, 63, 3, name="wlaplace3d_p3_1.5M")


# 16 form variants of the mixed batch, mesh k gets variant k mod 16.
BATCH_VARIANTS = (
    [("laplace", 2, q) for q in (1, 2, 3, 4)]
    + [("laplace", 3, q) for q in (1, 2, 3, 4)]
    + [("mass", 2, q) for q in (1, 2, 3)]
    + [("mass", 3, q) for q in (1, 2, 3)]
    + [("ns", 2, 2), ("ns", 3, 2)]
)


def batch_sizes(n_meshes: int = 64, lo: float = 1e3, hi: float = 5e5, seed: int = 4):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [int(round(math.exp(x))) for x in rng.uniform(math.log(lo), math.log(hi), size=n_meshes)]


def config4(n_meshes: int = 64, lo: float = 1e3, hi: float = 5e5, seed: int = 4, scale: float = 1.0):
    """Mixed batch: n_meshes meshes of log-uniform sizes, variants round-robin. `scale`
    shrinks every mesh (for quick tests) without changing the variant mix."""
    out = []
    for k, size in enumerate(batch_sizes(n_meshes, lo, hi, seed)):
        size = max(1, int(round(size * scale)))
        kind, dim, q = BATCH_VARIANTS[k % len(BATCH_VARIANTS)]
        if dim == 2:
            n = max(1, math.ceil(math.sqrt(size / 2.0)))
        else:
            n = max(1, math.ceil((size / 6.0) ** (1.0 / 3.0)))
        out.append(make_workload(kind, dim, q, n, seed * 1000 + k, max_cells=size,
                                 name=f"mesh{k}_{kind}{dim}d_p{q}"))
    return out


# ------------------------------------------------------------------ curved cells ---
# P2 geometry: each cell carries its vertices and its edge midpoints, the midpoints moved by
# a smooth displacement field that depends on the position only (so neighbours agree and
# the mesh stays conforming).  Edge order = the P2 dof order: triangle (1,2), (0,2), (0,1);
# tetrahedron (2,3), (1,3), (1,2), (0,3), (0,2), (0,1).

P2_EDGES = {2: ((1, 2), (0, 2), (0, 1)), 3: ((2, 3), (1, 3), (1, 2), (0, 3), (0, 2), (0, 1))}


def _bump(x: np.ndarray) -> np.ndarray:
    """Smooth displacement direction field on the unit square / cube, |value| <= 1."""
    d = x.shape[-1]
    s = np.sin(np.pi * x)
    base = np.prod(s, axis=-1)
    out = np.empty_like(x)
    for k in range(d):
        out[..., k] = base * np.cos(np.pi * (k + 1) * x[..., (k + 1) % d])
    return out


def curved_workload(dim: int, degree: int, n: int, seed: int, amplitude: float = 0.1, straight: bool = False,
                    max_cells: int | None = None, jitter: float = 0.1, name: str = "") -> Workload:
    """A jittered mesh of side n with P2 geometry: coords SoA [n_geo * d][cells] (vertices
    moved by up to jitter * h, then edge midpoints displaced by amplitude * h * bump(midpoint);
    straight=True keeps the midpoints on the straight edges, i.e. affine cells).  The
    defaults keep every Jacobian well conditioned (condition number below ~20 at every
    quadrature point); the affine workloads' 0.2 h jitter combined with curved edges can
    bring an occasional cell close to degenerate."""
    if dim == 2:
        verts, cells = unit_square(n, seed, jitter)
        if max_cells is not None:
            cells = cells[:max_cells]
    else:
        verts, cells = unit_cube(n, seed, jitter, max_cells=max_cells)
    h = 1.0 / n
    X = verts[cells]  # [nc, d+1, d]
    nodes = [X[:, v, :] for v in range(dim + 1)]
    for a, b in P2_EDGES[dim]:
        m = 0.5 * (X[:, a, :] + X[:, b, :])
        if not straight:
            m = m + amplitude * h * _bump(m)
        nodes.append(m)
    P = np.stack(nodes, axis=1)  # [nc, n_geo, d]
    coords = np.ascontiguousarray(P.reshape(P.shape[0], -1).T)
    return Workload("curved", dim, degree, coords, None, name=name,
                    meta={"cells": cells, "n_vertices": int(verts.shape[0])})


# ------------------------------------------------------------- badly shaped cells ---
# Single cells whose Jacobian J = R1 diag(s) R2 (R1, R2 random rotations) has condition
# number `aspect`: needles (s = (1, 1/a, ..., 1/a): one long edge direction) and slivers
# (s = (1, ..., 1, 1/a): a flat cell), each translated by U(-1, 1) per coordinate so that
# the edge vectors are formed by cancelling subtractions, as in a mesh away from the origin.

def badly_shaped(dim: int, cells: int, aspect: float, shape: str, seed: int) -> np.ndarray:
    """SoA coordinates [(d+1)*d][cells] of positively oriented needles or slivers."""
    if shape not in ("needle", "sliver"):
        raise ValueError(shape)
    rng = np.random.Generator(np.random.PCG64(seed))
    base = np.eye(dim + 1, dim, -1)  # vertex 0 at the origin, vertex k at e_k
    out = np.empty((cells, dim + 1, dim))
    for c in range(cells):
        R1 = np.linalg.qr(rng.standard_normal((dim, dim)))[0]
        R2 = np.linalg.qr(rng.standard_normal((dim, dim)))[0]
        s = np.ones(dim)
        if shape == "needle":
            s[1:] = 1.0 / aspect
        else:
            s[-1] = 1.0 / aspect
        v = base @ (R1 @ np.diag(s) @ R2).T + rng.uniform(-1.0, 1.0, size=dim)
        if np.linalg.det(v[1:] - v[0]) < 0:
            v[[1, 2]] = v[[2, 1]]
        out[c] = v
    return np.ascontiguousarray(out.reshape(cells, -1).T)
