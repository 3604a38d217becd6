"""Randomized mixed batches: seeded draws of forms, launch options, precisions and item sizes
(empty items, single cells, tile boundaries, ragged tails), with some outputs deliberately not
16-byte aligned (those items take the direct-store tile launch).  Every item of the batch must
equal, bit for bit, a single-mesh tabulation of the same form into an output of the same
alignment, and sampled cells must match the oracle (FP64 1e-12; split modes their bounds)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1112_0402_amd import capi, meshgen
from paper_1112_0402_amd.forms import Batch, Form
from tests.gpu_util import rel_fro, require_gpu, say, to_dev
from tests.test_gpu_parity import FP64_TOL, split_tol

pytestmark = pytest.mark.gpu

FORMS = [("mass", d, q) for d in (2, 3) for q in (1, 2, 3)] + [("laplace", d, q) for d in (2, 3) for q in (1, 2, 3, 4)] \
    + [("wlaplace", 2, q) for q in (1, 2, 3)] + [("wlaplace", 3, q) for q in (1, 2, 3)] \
    + [("elasticity", d, q) for d in (2, 3) for q in (1, 2)] + [("ns", d, q) for d in (2, 3) for q in (1, 2)]
# cell counts around the 16-, 32- and 64-cell tile edges, and ragged sizes
EDGE_CELLS = [0, 1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65, 127, 129]
# explicit launch options (FP64) besides the default; a form that cannot take one keeps the default
FP64_OPTIONS = [{}, {"persistent": -1}, {"persistent": -1, "geometry": "fused"}, {"persistent": -1, "geometry": "pass"},
                {"persistent": 1, "waves": 12}, {"persistent": 1, "waves": 12, "tile_cells": 32},
                {"persistent": 1, "waves": 16, "geometry": "pass"}]
SPLIT_OPTIONS = [{}, {"persistent": -1}, {"persistent": 1, "tile_cells": 32}, {"persistent": 1, "tile_cells": 64}]


def _workload(kind, dim, q, cells, seed):
    c = max(cells, 1)
    n = max(1, math.ceil(math.sqrt(c / 2.0))) if dim == 2 else max(1, math.ceil((c / 6.0) ** (1 / 3)))
    wl = meshgen.make_workload(kind, dim, q, n, seed, max_cells=c)
    if cells == 0:
        wl.coords = wl.coords[:, :0].copy()
        wl.coeffs = None if wl.coeffs is None else wl.coeffs[:, :0].copy()
    return wl


def _out(form, cells, aligned):
    """An output [cells, n, n]; unaligned: a view starting one element into a larger buffer."""
    n_el = cells * form.n_I
    buf = torch.full((n_el + 1,), float("nan"), dtype=form.out_dtype, device="cuda")
    o = (buf[:n_el] if aligned else buf[1:]).view(cells, form.n, form.n)
    assert (o.data_ptr() % 16 == 0) == aligned or cells == 0
    return o


def _form(kind, dim, q, precision, opts):
    try:
        return Form(kind, dim, q, precision=precision, **opts)
    except capi.FFCError:
        return Form(kind, dim, q, precision=precision)


@pytest.mark.parametrize("seed", range(12))
def test_random_mixed_batch(seed):
    require_gpu()
    rng = np.random.default_rng(4200 + seed)
    precision = ["fp64", "bf16x6", "fp64", "bf16x3"][seed % 4]
    options = FP64_OPTIONS if precision == "fp64" else SPLIT_OPTIONS
    n_items = int(rng.integers(6, 15))
    forms, items = {}, []
    for k in range(n_items):
        kind, dim, q = FORMS[int(rng.integers(len(FORMS)))]
        oi = int(rng.integers(len(options)))
        key = (kind, dim, q, oi)
        if key not in forms:
            forms[key] = _form(kind, dim, q, precision, options[oi])
        r = rng.random()
        cells = int(rng.choice(EDGE_CELLS)) if r < 0.45 else int(rng.integers(100, 12000 if dim == 3 else 20000))
        aligned = bool(rng.random() < 0.8)
        items.append((forms[key], _workload(kind, dim, q, cells, 5000 + 100 * seed + k), aligned))
    fl = [f for f, _, _ in items]
    X = [to_dev(wl.coords) for _, wl, _ in items]
    C = [to_dev(wl.coeffs) for _, wl, _ in items]
    outs = [_out(f, wl.cells, a) for f, wl, a in items]
    b = Batch(fl, X, C, outs)
    say(f"[random batch {seed}] {precision}: {n_items} items, {b.total_cells} cells, {b.work_units} units, "
        f"{b.launches} launches; " + ", ".join(f"{wl.kind}{wl.dim}{wl.degree}:{wl.cells}{'' if a else 'u'}"
                                                for _, wl, a in items))
    b.run()
    torch.cuda.synchronize()
    first = [o.clone() for o in outs]
    b.run()
    torch.cuda.synchronize()
    for (f, wl, aligned), x, c, o, o1 in zip(items, X, C, outs, first):
        if wl.cells == 0:
            continue
        assert torch.equal(o, o1), (wl.name, "second run differs")
        single = f.tabulate(x, c, out=_out(f, wl.cells, aligned))
        torch.cuda.synchronize()
        assert torch.equal(o, single), (wl.kind, wl.dim, wl.degree, wl.cells, aligned, f.info)
        idx = np.arange(wl.cells) if wl.cells <= 8 else np.unique(
            np.concatenate([[0, wl.cells - 1], rng.choice(wl.cells, 6, replace=False)]))
        ref = oracle.tabulate(wl.kind, wl.dim, wl.degree, np.ascontiguousarray(wl.coords[:, idx]),
                              None if wl.coeffs is None else np.ascontiguousarray(wl.coeffs[:, idx]))
        tol = FP64_TOL if precision == "fp64" else split_tol(precision, wl.kind, wl.dim, wl.degree)
        e = rel_fro(o.cpu().numpy()[idx], ref)[0]
        assert e <= tol, (wl.kind, wl.dim, wl.degree, wl.cells, aligned, e, tol)
