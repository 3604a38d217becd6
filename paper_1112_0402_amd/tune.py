"""Autotuner for the tabulation launches.

For one (form, dim, degree, precision, mesh) it times every candidate launch -- the tensor
kernel in its launch shapes and, in FP64, the quadrature kernel -- with HIP events on the
launch stream, and keeps the fastest.  Results go to a JSON tuning database keyed by form
and log2(cells); sweeps over many shapes are appended to a JSON-lines file and resume
where an interrupted sweep stopped.  The exhaustive search is also the judge of the learned
selector's choices (its regret is measured against it).
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

# Candidate launches.  Index order is part of the sweep-file format (the selector's outputs).
CANDIDATES_FP64 = (
    {"kernel": "tensor", "tile_cells": 0, "waves": 0, "persistent": 0, "tile_window": 0},      # library default
    # geometry pass, then the contraction
    {"kernel": "tensor", "tile_cells": 16, "waves": 16, "persistent": -1, "tile_window": -1, "geometry": "pass"},
    {"kernel": "tensor", "tile_cells": 64, "waves": 8, "persistent": -1, "tile_window": -1, "geometry": "pass"},
    {"kernel": "tensor", "tile_cells": 64, "waves": 4, "persistent": -1, "tile_window": 16, "geometry": "pass"},
    {"kernel": "tensor", "tile_cells": 32, "waves": 8, "persistent": -1, "tile_window": 16, "geometry": "pass"},
    # one launch: affine map computed per cell tile
    {"kernel": "tensor", "tile_cells": 64, "waves": 4, "persistent": -1, "tile_window": 16, "geometry": "fused"},
    {"kernel": "tensor", "tile_cells": 32, "waves": 8, "persistent": -1, "tile_window": 16, "geometry": "fused"},
    # persistent, 12 waves (A^0 fragments in registers, affine map computed one tile ahead),
    # cell tiles of 16, 32 and 64 cells (where they fit; else the library's fallback launch)
    {"kernel": "tensor", "tile_cells": 16, "waves": 12, "persistent": 1, "tile_window": 0},
    {"kernel": "tensor", "tile_cells": 32, "waves": 12, "persistent": 1, "tile_window": 0},
    {"kernel": "tensor", "tile_cells": 64, "waves": 12, "persistent": 1, "tile_window": 0},
    {"kernel": "quadrature"},  # last: the analytic rule's alternative
)
CANDIDATES_SPLIT = (
    {"kernel": "tensor", "tile_cells": 0, "waves": 0},
    {"kernel": "tensor", "tile_cells": 0, "waves": 0, "persistent": 1},
    {"kernel": "tensor", "tile_cells": 64, "waves": 4, "geometry": "pass"},
    {"kernel": "tensor", "tile_cells": 32, "waves": 8, "geometry": "pass"},
    {"kernel": "tensor", "tile_cells": 16, "waves": 8, "geometry": "pass"},
    {"kernel": "tensor", "tile_cells": 64, "waves": 4, "geometry": "fused"},
    {"kernel": "tensor", "tile_cells": 32, "waves": 8, "geometry": "fused"},
)


def candidates(precision: str):
    return CANDIDATES_FP64 if precision == "fp64" else CANDIDATES_SPLIT


def make_form(kind, dim, degree, precision, cand):
    from .forms import Form

    return Form(kind, dim, degree, precision=precision if cand["kernel"] == "tensor" else "fp64",
                kernel=cand["kernel"], tile_cells=cand.get("tile_cells", 0), waves=cand.get("waves", 0),
                persistent=cand.get("persistent", 0), tile_window=cand.get("tile_window", 0),
                geometry=cand.get("geometry", 0))


def measure(form, X, C, reps: int = 5, warmup: int = 2) -> float:
    """Median milliseconds of one tabulation (geometry + contraction, or quadrature)."""
    return measure_all([form], X, C, reps, warmup)[0]


def measure_all(forms, X, C, reps: int = 7, warmup: int = 2):
    """Median milliseconds of one tabulation for each form on the same mesh, measured in
    interleaved rounds (every form once per round), so clock and power drift during the
    measurement falls on all candidates alike; each round takes the forms in a fresh random
    order (seeded), so no form always follows the same launch (a long quadrature launch slows
    the launch after it).  Forms sharing an output dtype share one output buffer."""
    import torch

    outs = {}
    for f in forms:
        if f.out_dtype not in outs:
            outs[f.out_dtype] = f.empty_out(X.shape[1])
    for _ in range(warmup):
        for f in forms:
            f.tabulate(X, C, out=outs[f.out_dtype])
    torch.cuda.synchronize()
    times = [[] for _ in forms]
    rng = np.random.default_rng(12345)
    for _ in range(reps):
        for j in rng.permutation(len(forms)):
            f = forms[j]
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(f.stream)
            f.tabulate(X, C, out=outs[f.out_dtype])
            b.record(f.stream)
            b.synchronize()
            times[j].append(a.elapsed_time(b))
    return [float(np.median(t)) for t in times]


def shape_key(kind, dim, degree, precision, cells) -> str:
    return f"{kind}/{dim}/{degree}/{precision}/{int(round(math.log2(max(cells, 1))))}"


class TuneDB:
    """JSON map shape key -> {"candidate": index, "config": ..., "ms": ...}."""

    def __init__(self, path: str | None = None):
        self.path = path or os.environ.get("FFC_TUNE_DB", "")
        self.db = {}
        if self.path and os.path.exists(self.path):
            with open(self.path) as f:
                self.db = json.load(f)

    def put(self, key, entry):
        self.db[key] = entry
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.db, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)

    def lookup(self, kind, dim, degree, precision, cells):
        """Entry of the nearest cell-count bucket for this form, or None."""
        best, dist = None, None
        lc = math.log2(max(cells, 1))
        prefix = f"{kind}/{dim}/{degree}/{precision}/"
        for k, v in self.db.items():
            if k.startswith(prefix):
                d = abs(int(k.rsplit("/", 1)[1]) - lc)
                if dist is None or d < dist:
                    best, dist = v, d
        return best


def autotune(kind, dim, degree, precision, X, C, db: TuneDB | None = None, reps: int = 5):
    """Time every candidate on this mesh; return (index, config, ms list)."""
    forms = [make_form(kind, dim, degree, precision, cand) for cand in candidates(precision)]
    times = measure_all(forms, X, C, reps)
    for f in forms:
        f.close()
    best = int(np.argmin(times))
    if db is not None:
        db.put(shape_key(kind, dim, degree, precision, X.shape[1]),
               {"candidate": best, "config": candidates(precision)[best], "ms": times[best], "all_ms": times})
    return best, candidates(precision)[best], times


# A batch pick replaces the default launch only if it measured faster by more than this.
BATCH_TUNE_MARGIN = 0.02


def batch_forms(workloads, precision="fp64", choice="default", db: TuneDB | None = None, selector=None, reps=11):
    """One form per batch item (a Batch groups items by launch shape): the library default
    launch (`choice="default"`), the exhaustive autotuner's winner (`"autotune"`), or the
    trained selector's pick (`"selector"`, FP64).  A batch runs all items of one form and
    launch shape in one launch, so both decide once per form: the autotuner times every
    tensor candidate as a batch of that form's meshes (the way the batch will run it) and
    keeps the fastest if it beats the default by more than BATCH_TUNE_MARGIN, the selector
    judges the form's cells summed over the batch; per-mesh
    picks that differ would split a form's items over several launches.  Batches run the
    tensor kernel, so the quadrature candidate is excluded; items with the same form and
    launch share one Form.  `db` is accepted for the callers' sake and not used: a batch
    pick depends on the whole batch, not on one mesh's shape."""
    import torch

    from .forms import Batch

    cands = candidates(precision)
    tensor_idx = [i for i, c in enumerate(cands) if c["kernel"] == "tensor"]
    forms, out, picks = {}, [], []
    members = {}
    for w in workloads:
        members.setdefault((w.kind, w.dim, w.degree), []).append(w)
    pick = {}

    def form_of(w, j):  # one Form per (form variant, candidate), shared by the meshes
        key = (w.kind, w.dim, w.degree, j)
        if key not in forms:
            forms[key] = make_form(w.kind, w.dim, w.degree, precision, cands[j])
        return forms[key]

    def tune_form(ws):
        """The pick among the tensor candidates running these meshes as one batch: medians
        over interleaved rounds (every candidate once per round, in a fresh seeded random
        order, as in measure_all)."""
        X = [torch.from_numpy(w.coords).cuda() for w in ws]
        C = [None if w.coeffs is None else torch.from_numpy(w.coeffs).cuda() for w in ws]
        outs, batches = {}, []
        for j in tensor_idx:
            f = form_of(ws[0], j)
            if f.out_dtype not in outs:
                outs[f.out_dtype] = [f.empty_out(w.cells) for w in ws]
            batches.append(Batch([f] * len(ws), X, C, outs[f.out_dtype]))
        s = torch.cuda.current_stream()
        for _ in range(2):
            for b in batches:
                b.run()
        torch.cuda.synchronize()
        ts = [[] for _ in batches]
        rng = np.random.default_rng(777)
        for _ in range(reps):
            for k in rng.permutation(len(batches)):
                a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(s)
                batches[k].run()
                e.record(s)
                e.synchronize()
                ts[k].append(a.elapsed_time(e))
        for b in batches:
            b.close()
        times = [float(np.median(t)) for t in ts]
        # the default unless a candidate is faster by more than the margin: with ten
        # candidates timed on small batches, a plain argmin often keeps the luckiest timing
        best = int(np.argmin(times))
        return tensor_idx[best] if times[best] < times[0] * (1.0 - BATCH_TUNE_MARGIN) else 0

    for w in workloads:
        fk = (w.kind, w.dim, w.degree)
        if choice == "default":
            j = 0
        elif choice == "autotune":
            if fk not in pick:
                pick[fk] = tune_form(members[fk])
            j = pick[fk]
        elif choice == "selector":
            if fk not in pick:
                info = form_of(w, 0).info
                rec = {"kind": w.kind, "dim": w.dim, "degree": w.degree, "cells": sum(m.cells for m in members[fk]),
                       "n_I": info["n_entries"], "n_alpha": info["n_alpha"], "ms": [1.0] * len(cands)}
                pick[fk] = selector.decide(selector.predict_rel([rec])[0], tensor_idx)
            j = pick[fk]
        else:
            raise ValueError(f"unknown choice {choice!r}")
        out.append(form_of(w, j))
        picks.append(j)
    return out, picks


def sweep_shapes(variants, cells_list):
    return [(k, d, q, c) for (k, d, q) in variants for c in cells_list]


def sweep(shapes, path: str, precision: str = "fp64", reps: int = 7, seed: int = 5, log=print):
    """Time every candidate on every shape; one JSON line per shape, appended to `path`;
    shapes already in the file are skipped (resume)."""
    import torch

    from . import meshgen
    from .forms import Form

    done = set()
    if os.path.exists(path):
        for line in open(path):
            r = json.loads(line)
            done.add((r["kind"], r["dim"], r["degree"], r["precision"], r["cells"]))
    forms = {}
    for i, (kind, dim, degree, cells) in enumerate(shapes):
        if (kind, dim, degree, precision, cells) in done:
            continue
        n = math.ceil(math.sqrt(cells / 2.0)) if dim == 2 else math.ceil((cells / 6.0) ** (1.0 / 3.0))
        wl = meshgen.make_workload(kind, dim, degree, max(n, 1), seed + i, max_cells=cells)
        X = torch.from_numpy(wl.coords).cuda()
        C = None if wl.coeffs is None else torch.from_numpy(wl.coeffs).cuda()
        for j, cand in enumerate(candidates(precision)):
            key = (kind, dim, degree, j)
            if key not in forms:
                forms[key] = make_form(kind, dim, degree, precision, cand)
        times = measure_all([forms[(kind, dim, degree, j)] for j in range(len(candidates(precision)))], X, C, reps)
        info = Form(kind, dim, degree, precision=precision).info
        rec = {"kind": kind, "dim": dim, "degree": degree, "precision": precision, "cells": cells,
               "n_I": info["n_entries"], "n_alpha": info["n_alpha"], "ms": times, "time": time.time()}
        with open(path, "a") as f:
            f.write(json.dumps(rec) + "\n")
        log(f"sweep {kind} d={dim} q={degree} cells={cells}: best {int(np.argmin(times))} "
            f"({min(times):.4f} ms) of {[round(t, 4) for t in times]}")
    return path


def load_sweep(path: str):
    with open(path) as f:
        return [json.loads(line) for line in f if line.strip()]


def default_sweep_shapes():
    """The mixed-batch form variants plus the two large single-form workloads, each at
    cell counts 2^10 .. 2^19."""
    from .meshgen import BATCH_VARIANTS

    variants = list(BATCH_VARIANTS) + [("elasticity", 3, 2), ("wlaplace", 3, 3)]
    return sweep_shapes(variants, [2 ** k for k in (10, 12, 14, 16, 18, 19)])


if __name__ == "__main__":
    import argparse

    ap = argparse.ArgumentParser(description="time every candidate launch on a sweep of shapes (resumable)")
    ap.add_argument("--out", required=True, help="JSON-lines file to append to")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--reps", type=int, default=7)
    args = ap.parse_args()
    sweep(default_sweep_shapes(), args.out, precision=args.precision, reps=args.reps,
          log=lambda s: print(s, flush=True))
