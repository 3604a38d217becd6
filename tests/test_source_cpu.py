"""Pins for the oracle's linear form L(v) = int_K f v dx (rank-1 element vectors, the
right-hand side of the Poisson form file, Sec. 5.5).  CPU only."""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact


def _rational_cell(dim, seed):
    rnd = random.Random(seed)
    base = [[0] * dim] + [[1 if k == v else 0 for k in range(dim)] for v in range(dim)]
    scale = Fraction(rnd.randint(20, 40), 37)
    return [[Fraction(c) * scale + Fraction(rnd.randint(-6, 6), 53) for c in v] for v in base]


def _soa(verts):
    return np.ascontiguousarray(np.asarray([[float(c) for c in v] for v in verts]).reshape(-1, 1))


def _volume(verts):
    d = len(verts) - 1
    J = np.array([[float(verts[b + 1][k] - verts[0][k]) for b in range(d)] for k in range(d)])
    return abs(np.linalg.det(J)) / math.factorial(d)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("q", [1, 2, 3])
def test_source_vector_matches_exact_rationals(dim, q):
    verts = _rational_cell(dim, 10 * dim + q)
    ns = len(oracle.nodes(dim, q))
    rnd = random.Random(q)
    f = [Fraction(rnd.randint(-20, 20), 11) for _ in range(ns)]
    ref = np.array([float(x) for x in exact.source_vector(verts, q, f)])
    got = oracle.source_vector(dim, q, _soa(verts), np.array([[float(x) for x in f]]))[0]
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_source_vector_p1_closed_form(dim):
    """P1: b_i = |K| / ((d+1)(d+2)) * (f_i + sum_j f_j)."""
    verts = _rational_cell(dim, 5)
    f = np.array([0.3, -1.2, 2.5, 0.7][: dim + 1])
    b = oracle.source_vector(dim, 1, _soa(verts), f[None])[0]
    vol = _volume(verts)
    assert np.allclose(b, vol / ((dim + 1) * (dim + 2)) * (f + f.sum()), rtol=1e-14, atol=0)


@pytest.mark.parametrize("dim,q", [(2, 2), (3, 3), (2, 4)])
def test_source_vector_constant_and_linearity(dim, q):
    """f = 1 integrates to |K| in total (partition of unity); L is linear in f."""
    verts = _rational_cell(dim, 7)
    X = _soa(verts)
    ns = len(oracle.nodes(dim, q))
    one = oracle.source_vector(dim, q, X, np.ones((1, ns)))[0]
    assert abs(one.sum() - _volume(verts)) <= 1e-14 * _volume(verts)
    rng = np.random.default_rng(q)
    f, g = rng.normal(size=(1, ns)), rng.normal(size=(1, ns))
    lhs = oracle.source_vector(dim, q, X, 2.0 * f - 3.0 * g)
    rhs = 2.0 * oracle.source_vector(dim, q, X, f) - 3.0 * oracle.source_vector(dim, q, X, g)
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-14 * np.abs(rhs).max())
