"""FFC_KERNEL_AUTO through the C-ABI: the library evaluates the trained selector network on
the host at form creation and dispatches each tabulation to the launch it picks for that
cell count.  The picks equal those of the Python selector (the same network evaluated by
the library's GPU MLP kernels) wherever the two best predictions are not a near tie, the
results equal the oracle whichever launch is taken, and without a selector file every cell
count takes the library default launch."""
import ctypes
import math
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1112_0402_amd import capi, meshgen, selector, tune
from paper_1112_0402_amd.forms import Form
from tests.gpu_util import rel_fro, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu

SHAPES = [("laplace", 2, 1), ("laplace", 3, 1), ("mass", 3, 1), ("mass", 2, 1), ("laplace", 3, 2), ("mass", 3, 3),
          ("laplace", 3, 4), ("ns", 3, 2), ("elasticity", 3, 2), ("wlaplace", 3, 3), ("laplace", 2, 4)]


def _select(form, cells):
    cand, from_sel = ctypes.c_int32(), ctypes.c_int32()
    capi.check(capi.lib().ffc_form_select(form.handle, cells, ctypes.byref(cand), ctypes.byref(from_sel)))
    return cand.value, from_sel.value


def _need_file():
    if not os.path.exists(selector.DEFAULT_FILE):
        pytest.skip("no trained selector file beside the library")


def test_auto_picks_what_the_python_selector_picks():
    require_gpu()
    _need_file()
    sel = selector.Selector.load(selector.DEFAULT_FILE)
    compared = ties = 0
    for kind, dim, q in SHAPES:
        f = Form(kind, dim, q, kernel="auto")
        assert f.info["auto_launches"] >= 1
        picks = []
        for b in range(8, 22):
            cells = 1 << b
            cand, from_sel = _select(f, cells)
            assert from_sel == 1
            rec = {"kind": kind, "dim": dim, "degree": q, "cells": cells, "n_I": f.info["n_entries"],
                   "n_alpha": f.info["n_alpha"], "ms": [1.0] * len(tune.CANDIDATES_FP64)}
            pred = sel.predict_rel([rec])[0]
            order = np.argsort(pred)
            picks.append(cand)
            # near ties (FP32 on the GPU vs FP64 on the host): two best candidates, or the best
            # one at the decision margin
            at_margin = abs(pred[order[0]] - (pred[0] - math.log1p(sel.margin))) < 1e-4
            if pred[order[1]] - pred[order[0]] < 1e-4 or at_margin:
                ties += 1
                continue
            compared += 1
            assert cand == sel.decide(pred), (kind, dim, q, cells, cand, sel.decide(pred), pred)
        say(f"[auto] {kind} d={dim} q={q}: picks for 2^8..2^21 cells {picks} ({f.info['auto_launches']} launches)")
    say(f"[auto] {compared} picks compared with the Python selector, {ties} near ties skipped")
    assert compared > 0.9 * (compared + ties)


def test_auto_tabulation_matches_oracle():
    require_gpu()
    _need_file()
    quad_seen = False
    for kind, dim, q in SHAPES:
        f = Form(kind, dim, q, kernel="auto")
        # the cell counts of two buckets the selector treats differently, if any
        table = [_select(f, 1 << b)[0] for b in range(8, 20)]
        sizes = sorted({8 + table.index(c) for c in set(table)})[:3]
        for b in sizes:
            cells = 1 << b
            n = int(np.ceil(np.sqrt(cells / 2))) if dim == 2 else int(np.ceil((cells / 6) ** (1 / 3)))
            wl = meshgen.make_workload(kind, dim, q, n, 60 + b, max_cells=cells)
            cand, _ = _select(f, wl.cells)
            quad_seen |= tune.CANDIDATES_FP64[cand]["kernel"] == "quadrature"
            got = f.tabulate(to_dev(wl.coords), to_dev(wl.coeffs))
            torch.cuda.synchronize()
            ref = oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs)
            e = rel_fro(got.cpu().numpy(), ref)[0]
            say(f"[auto] {kind} d={dim} q={q} {wl.cells} cells: candidate {cand}, max {e:.2e}")
            assert e <= 1e-12
    say(f"[auto] quadrature kernel taken somewhere: {quad_seen}")


def test_auto_without_a_selector_file():
    require_gpu()
    old = os.environ.get("FFC_SELECTOR")
    try:
        os.environ["FFC_SELECTOR"] = "none"
        f = Form("laplace", 3, 1, kernel="auto")
        assert f.info["auto_launches"] == 1
        for b in (4, 12, 20):
            assert _select(f, 1 << b) == (0, 0)
        wl = meshgen.make_workload("laplace", 3, 1, 9, 3)
        X = to_dev(wl.coords)
        a = f.tabulate(X)
        b = Form("laplace", 3, 1).tabulate(X)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        os.environ["FFC_SELECTOR"] = "/nonexistent/selector.txt"
        with pytest.raises(capi.FFCError) as ei:
            Form("laplace", 3, 1, kernel="auto")
        assert ei.value.code == capi.FFC_E_INVALID
        # a non-AUTO form has no selection
        t = Form("laplace", 3, 1)
        cand = ctypes.c_int32()
        assert capi.lib().ffc_form_select(t.handle, 100, ctypes.byref(cand), None) == capi.FFC_E_INVALID
    finally:
        if old is None:
            os.environ.pop("FFC_SELECTOR", None)
        else:
            os.environ["FFC_SELECTOR"] = old
