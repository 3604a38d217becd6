"""CPU checks of the selector's reference network, heuristic, regret and tuning DB."""
import math

import numpy as np

from paper_1112_0402_amd import selector, tune


def _rand_params(n_in, h, n_out, seed=0):
    rng = np.random.default_rng(seed)
    n = n_in * h + h + h * h + h + h * n_out + n_out
    return rng.normal(0, 0.5, size=n)


def test_reference_backward_matches_finite_differences():
    n_in, h, n_out = 6, 8, 5
    p = _rand_params(n_in, h, n_out)
    rng = np.random.default_rng(1)
    x = rng.normal(size=(7, n_in))
    dy = rng.normal(size=(7, n_out))
    g = selector.ref_backward(p, x, dy, n_in, h, n_out)
    eps = 1e-6
    for k in rng.choice(p.size, size=40, replace=False):
        e = np.zeros_like(p)
        e[k] = eps
        fp = (selector.ref_forward(p + e, x, n_in, h, n_out)[0] * dy).sum()
        fm = (selector.ref_forward(p - e, x, n_in, h, n_out)[0] * dy).sum()
        assert abs((fp - fm) / (2 * eps) - g[k]) < 1e-6 * (1 + abs(g[k]))


def test_reference_mse():
    y = np.array([[1.0, 2.0], [3.0, 5.0]])
    t = np.array([[0.0, 2.0], [3.0, 1.0]])
    m = np.array([[1.0, 1.0], [0.0, 1.0]])
    loss, dy = selector.ref_mse(y, t, m)
    assert math.isclose(loss, (1 + 0 + 16) / 3)
    assert np.allclose(dy, 2 * (y - t) * m / 3)


def test_heuristic_follows_paper_complexity_model():
    # mass: speedup (2q)^d > 1 -> tensor representation for every q >= 1
    for d in (2, 3):
        for q in (1, 2, 3):
            assert selector.heuristic_choice("mass", d, q) == 0
    assert selector.heuristic_choice("laplace", 3, 2) == 0


def test_regret_and_features():
    recs = [{"ms": [2.0, 1.0, 4.0, 1.0, 1.0, 3.0]}, {"ms": [1.0, 2.0, 2.0, 2.0, 2.0, 0.5]}]
    r = selector.regret(recs, [0, 5])
    assert np.allclose(r, [1.0, 0.0])
    f = selector.features("laplace", 3, 2, 1024, 100, 9)
    assert f.shape == (selector.N_FEATURES,) and f[5] == 10 and np.isclose(f[6], 10 + np.log2(100))


def test_targets_are_relative_to_the_default_launch():
    recs = [{"kind": "mass", "dim": 2, "degree": 1, "cells": 64, "n_I": 9, "n_alpha": 1,
             "ms": [2.0, 1.0, None, 4.0]}]
    X, T, M = selector.records_to_arrays(recs)
    assert np.allclose(T[0], [0.0, np.log(0.5), 0.0, np.log(2.0)])
    assert np.array_equal(M[0], [1, 1, 0, 1])


def test_tune_db_roundtrip(tmp_path):
    db = tune.TuneDB(str(tmp_path / "db.json"))
    db.put(tune.shape_key("laplace", 3, 2, "fp64", 1 << 14), {"candidate": 2, "ms": 0.1})
    db.put(tune.shape_key("laplace", 3, 2, "fp64", 1 << 18), {"candidate": 0, "ms": 0.5})
    db2 = tune.TuneDB(str(tmp_path / "db.json"))
    assert db2.lookup("laplace", 3, 2, "fp64", 20000)["candidate"] == 2
    assert db2.lookup("laplace", 3, 2, "fp64", 300000)["candidate"] == 0
    assert db2.lookup("mass", 3, 2, "fp64", 300000) is None


def test_candidate_lists():
    assert tune.CANDIDATES_FP64[-1]["kernel"] == "quadrature"
    assert all(c["kernel"] == "tensor" for c in tune.CANDIDATES_SPLIT)
    assert len(tune.default_sweep_shapes()) == 18 * 6


def test_decision_margin():
    """A candidate replaces the default (index 0) only when predicted faster by more than
    the margin; the allowed set restricts the choice; margin 0 is the plain argmin."""
    sel = selector.Selector.__new__(selector.Selector)
    sel.margin = 0.02
    lg = math.log1p
    assert sel.decide(np.array([0.0, -lg(0.01), 0.3])) == 0           # 1% predicted gain: keep the default
    assert sel.decide(np.array([0.0, -lg(0.05), -lg(0.03)])) == 1     # 5% gain: take the best
    assert sel.decide(np.array([0.0, -lg(0.05), -lg(0.03)]), allowed=[0, 2]) == 2
    assert sel.decide(np.array([0.1, 0.0, 0.2])) == 1                 # the default predicted slower
    sel.margin = 0.0
    assert sel.decide(np.array([0.0, -1e-9, 0.3])) == 1
    assert selector.DECISION_MARGIN == 0.02


def test_selector_file_carries_the_margin():
    """The shipped selector file is format 2 and states the decision margin the library's
    automatic choice applies."""
    tok = open(selector.DEFAULT_FILE).read().split()
    assert tok[:2] == ["ffc_selector", "2"]
    i = tok.index("margin")
    assert tok[i - 2] == "tmu" and float(tok[i + 1]) == selector.DECISION_MARGIN
