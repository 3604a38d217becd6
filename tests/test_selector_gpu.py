"""GPU tests of the selector network kernels (against the FP64 NumPy statement), of the
autotuner, and of what the trained selector gains over choosing without it."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1112_0402_amd import meshgen, selector, tune
from tests.gpu_util import rel_fro, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu

SWEEP = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1112_0402_amd", "data",
                     "sweep_mi355x_fp64.jsonl")


def test_mlp_kernels_match_fp64_reference():
    require_gpu()
    net = selector.MLP(n_in=7, n_hidden=32, n_out=6, seed=3)
    rng = np.random.default_rng(0)
    X = rng.normal(size=(300, 7))
    x = torch.tensor(X, dtype=torch.float32, device="cuda")
    y, act = net.forward(x)
    p = net.params.cpu().numpy().astype(np.float64)
    yref, _ = selector.ref_forward(p, x.cpu().numpy().astype(np.float64), 7, 32, 6)
    assert np.allclose(y.cpu().numpy(), yref, rtol=1e-4, atol=1e-4)
    T = rng.normal(size=(300, 6))
    Mk = (rng.uniform(size=(300, 6)) > 0.2).astype(np.float64)
    t = torch.tensor(T, dtype=torch.float32, device="cuda")
    m = torch.tensor(Mk, dtype=torch.float32, device="cuda")
    loss, dy = net.mse(y, t, m)
    lref, dyref = selector.ref_mse(yref, T, Mk)
    assert abs(float(loss.item()) - lref) < 1e-4 * max(1.0, lref)
    assert np.allclose(dy.cpu().numpy(), dyref, rtol=1e-3, atol=1e-6)
    g = net.backward(x, act, dy).cpu().numpy()
    gref = selector.ref_backward(p, x.cpu().numpy().astype(np.float64), dy.cpu().numpy().astype(np.float64), 7, 32, 6)
    err = np.abs(g - gref).max() / np.abs(gref).max()
    say(f"[mlp] max rel gradient error vs FP64 reference {err:.2e}")
    assert err < 1e-4
    # one Adam step with the L2 term vs its definition
    wd = 1e-2
    net.adam(lr=1e-2, weight_decay=wd)
    torch.cuda.synchronize()
    gd = g + wd * p
    m1 = 0.1 * gd
    v1 = 0.001 * gd * gd
    pref = p - 1e-2 * (m1 / 0.1) / (np.sqrt(v1 / 0.001) + 1e-8)
    assert np.allclose(net.params.cpu().numpy(), pref, rtol=1e-4, atol=1e-6)


def test_autotuner_picks_fastest_and_is_exact():
    require_gpu()
    wl = meshgen.make_workload("laplace", 3, 2, 12, 21)  # 10,368 cells
    X, C = to_dev(wl.coords), None
    db = tune.TuneDB()
    best, cfg, times = tune.autotune("laplace", 3, 2, "fp64", X, C, db=db, reps=3)
    say(f"[tune] laplace P2 3D 10k cells: best {best} {cfg} times {[round(t, 4) for t in times]}")
    assert times[best] == min(times)
    assert db.lookup("laplace", 3, 2, "fp64", wl.cells)["candidate"] == best
    out = tune.make_form("laplace", 3, 2, "fp64", cfg).tabulate(X, C)
    torch.cuda.synchronize()
    ref = oracle.tabulate("laplace", 3, 2, wl.coords)
    assert rel_fro(out.cpu().numpy(), ref)[0] <= 1e-12


def _cross_validate(recs, folds, seed0=0):
    held, choice = [], []
    for k, test_idx in enumerate(folds):
        ts = set(test_idx)
        train = [r for i, r in enumerate(recs) if i not in ts]
        test = [recs[i] for i in test_idx]
        sel = selector.Selector(n_hidden=64, seed=seed0 + k)
        sel.fit(train, epochs=3000, lr=3e-3)
        held += test
        choice += sel.choose(test)
    return held, choice


def _report(tag, held, choice):
    r_mlp = selector.regret(held, choice)
    r_fixed = selector.regret(held, [0] * len(held))
    heur = [selector.heuristic_choice(r["kind"], r["dim"], r["degree"]) for r in held]
    r_heur = selector.regret(held, heur)
    t_best = sum(min(r["ms"]) for r in held)
    t_mlp = sum(r["ms"][c] for r, c in zip(held, choice))
    t_fixed = sum(r["ms"][0] for r in held)
    t_heur = sum(r["ms"][c] for r, c in zip(held, heur))
    say(f"[selector] {tag}: held-out mean regret: mlp {r_mlp.mean():.3f} fixed default {r_fixed.mean():.3f} "
        f"analytic rule {r_heur.mean():.3f}; total ms: exhaustive {t_best:.3f} mlp {t_mlp:.3f} "
        f"fixed {t_fixed:.3f} analytic {t_heur:.3f}")
    return r_mlp.mean(), r_fixed.mean(), r_heur.mean()


def test_selector_beats_choosing_without_it():
    """Three-fold cross-validation over the stored sweep (fold k holds out the shapes whose
    index is k mod 3; every (form, degree, dimension) keeps other cell counts in training, so
    this measures the choice at unseen sizes of known forms): the mean regret against the
    exhaustive autotuner must be lower than always taking the library default launch and
    lower than the paper's analytic tensor-vs-quadrature rule."""
    require_gpu()
    if not os.path.exists(SWEEP):
        pytest.skip("no stored sweep")
    recs = tune.load_sweep(SWEEP)
    held, choice = _cross_validate(recs, [[i for i in range(len(recs)) if i % 3 == k] for k in range(3)])
    r_mlp, r_fixed, r_heur = _report("3-fold, unseen sizes", held, choice)
    assert r_mlp < r_fixed
    assert r_mlp < r_heur


def test_selector_on_unseen_forms():
    """Leave-one-form-out cross-validation: each fold holds out every cell count of one
    (kind, dimension, degree), so the network judges a form it never saw.  Reported next to
    the per-size folds; the regret must stay finite and the choices valid (the weaker
    generalisation is stated, not hidden)."""
    require_gpu()
    if not os.path.exists(SWEEP):
        pytest.skip("no stored sweep")
    recs = tune.load_sweep(SWEEP)
    groups = {}
    for i, r in enumerate(recs):
        groups.setdefault((r["kind"], r["dim"], r["degree"]), []).append(i)
    held, choice = _cross_validate(recs, list(groups.values()), seed0=10)
    r_mlp, r_fixed, r_heur = _report(f"leave-one-form-out ({len(groups)} folds)", held, choice)
    assert np.isfinite(r_mlp) and all(0 <= c < len(tune.CANDIDATES_FP64) for c in choice)


def test_selected_launch_is_exact():
    """Whatever the selector picks, the element tensors are the oracle's."""
    require_gpu()
    if not os.path.exists(SWEEP):
        pytest.skip("no stored sweep")
    recs = tune.load_sweep(SWEEP)
    sel = selector.Selector(seed=1)
    sel.fit(recs, epochs=1500)
    for kind, dim, q, n in (("laplace", 2, 1, 8), ("mass", 3, 2, 4), ("ns", 3, 2, 3)):
        wl = meshgen.make_workload(kind, dim, q, n, 31)
        from paper_1112_0402_amd.forms import Form

        info = Form(kind, dim, q).info
        rec = {"kind": kind, "dim": dim, "degree": q, "cells": wl.cells, "n_I": info["n_entries"],
               "n_alpha": info["n_alpha"], "ms": [1.0] * len(tune.CANDIDATES_FP64)}
        c = sel.choose([rec])[0]
        out = tune.make_form(kind, dim, q, "fp64", tune.CANDIDATES_FP64[c]).tabulate(to_dev(wl.coords),
                                                                                       to_dev(wl.coeffs))
        torch.cuda.synchronize()
        ref = oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs)
        assert rel_fro(out.cpu().numpy(), ref)[0] <= 1e-12, (kind, c)


@pytest.mark.parametrize("choice", ["autotune", "selector"])
def test_tuned_batch_is_exact(choice):
    """A batch whose per-mesh launch shapes come from the autotuner (or the selector) groups
    the items by shape and still equals the oracle."""
    require_gpu()
    from paper_1112_0402_amd.forms import Batch

    if choice == "selector" and not os.path.exists(SWEEP):
        pytest.skip("no stored sweep")
    wls = meshgen.config4(n_meshes=16, scale=0.01)
    sel = None
    if choice == "selector":
        sel = selector.Selector(seed=2)
        sel.fit(tune.load_sweep(SWEEP), epochs=1000)
    fl, picks = tune.batch_forms(wls, "fp64", choice, db=tune.TuneDB(None), selector=sel)
    say(f"[tuned batch] {choice}: picks {picks}")
    assert all(tune.CANDIDATES_FP64[j]["kernel"] == "tensor" for j in picks)
    X = [to_dev(w.coords) for w in wls]
    C = [to_dev(w.coeffs) for w in wls]
    outs = [f.empty_out(w.cells) for f, w in zip(fl, wls)]
    b = Batch(fl, X, C, outs)
    b.run()
    torch.cuda.synchronize()
    for w, o in zip(wls, outs):
        ref = oracle.tabulate(w.kind, w.dim, w.degree, w.coords, w.coeffs)
        assert rel_fro(o.cpu().numpy(), ref)[0] <= 1e-12, w.name
