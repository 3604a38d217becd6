#!/usr/bin/env python3
"""Element tensors/s of the tensor-representation path on one MI355X.

Workload (default): 3D linear elasticity int sigma(u):eps(v) with lambda = mu = 1, vector
P2 tetrahedra (30 dofs), 6 * 50^3 = 750,000 cells of a jittered unit cube (seed 2), FP64.
A step is one pass of the hot path over the mesh, inputs resident in HBM:
  geometry kernel (coords -> det J, J^{-1}, one lane per cell)
  + contraction kernel (G_K tile in LDS, A^0 tiles on FP64 MFMA, 900 x 81 per cell).
The plain GPU quadrature kernel is timed beside it on the same mesh, and the FP64 oracle
is timed on the host cores on a bounded sample of the same mesh.

Prints one JSON line.  Options: --gpus (1 only), --steps, --warmup.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
FP64_MFMA_PEAK_TF = 78.6   # MI355X dense FP64 matrix
BF16_MFMA_PEAK_TF = 2500.0  # MI355X dense BF16 matrix
METRIC = "element tensors/s + %HBM/MFMA peak, tensor-rep vs quadrature kernel, rel err≤1e-12"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "contract_f64_elasticity3d_p2_750k_traffic.txt")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h"):
        with open(os.path.join(ROOT, "paper_1112_0402_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(cells: int):
    """HBM bytes per launch of the contraction kernel from the committed rocprofv3 PMC
    summary, if it was taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_source_hash() or int(kv.get("cells", -1)) != cells:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target wall time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-quadrature", action="store_true")
    ap.add_argument("--tile-cells", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--persistent", type=int, default=0, help="0 auto, 1 on, -1 off")
    ap.add_argument("--tile-window", type=int, default=0,
                    help="grouping of output entries into MFMA tiles (0 = library default)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (HBM counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the element-tensor path has no "
                                   "cross-GPU step (cells shard with no exchange); run with --gpus 1"}))
        return 2

    import numpy as np
    import torch

    from paper_1112_0402_amd import meshgen
    from paper_1112_0402_amd.forms import Form, compute_geometry

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        return 1
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": src.numel() * 8, "bytes_written": dst.numel() * 8}))
        return 0
    wl = meshgen.config2()
    cells = wl.cells
    X = torch.from_numpy(wl.coords).cuda()
    form = Form("elasticity", 3, 2, tile_cells=args.tile_cells, waves=args.waves, tile_window=args.tile_window,
                persistent=args.persistent)
    info = form.info
    amap = torch.empty((10, cells), dtype=torch.float64, device="cuda")
    out = form.empty_out(cells)
    stream = torch.cuda.current_stream()

    def step():
        compute_geometry(X, 3, out=amap)
        form.tabulate_affine(amap, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: K steps, each bracketed by HIP events on the launch stream
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        compute_geometry(X, 3, out=amap)
        ev[k][1].record(stream)
        form.tabulate_affine(amap, out=out)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    geo_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    con_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    value = cells / (ms_step * 1e-3)

    # algorithmic bytes / flops per cell
    n_I, n_alpha, nnz = info["n_entries"], info["n_alpha"], info["nnz_a0"]
    con_bytes = cells * ((1 + 9) * 8 + n_I * 8)            # affine map in + element tensor out
    geo_bytes = cells * (12 * 8 + (1 + 9) * 8)              # coords in + affine map out
    path_bytes = cells * (12 * 8 + n_I * 8)                 # coords in + element tensor out
    alg_flops = cells * 2 * nnz                              # zeros of A^0 skipped
    mfma_flops = cells * info["mfma_k_per_tile"] * 32        # executed on the matrix cores
    con_gbs = con_bytes / (con_ms * 1e-3) / 1e9
    traffic = load_traffic(cells)

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "element tensors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "elasticity3d_p2_750k",
            "form": "int sigma(u):eps(v), lambda=mu=1, vector P2 tetrahedra",
            "cells": cells,
            "n_entries": n_I,
            "n_alpha": n_alpha,
            "mesh": "6*50^3 Kuhn tetrahedra of the unit cube, interior vertices jittered U(+-0.2h), seed 2",
            "tile_cells": info["tile_cells"],
            "waves": info["persistent_waves"] or info["waves"],
            "persistent": bool(info["persistent_waves"]),
            "tile_window": args.tile_window,
            "mfma_tiles": info["n_tiles"],
        },
        "roofline": {
            "kernel": "contract_f64_kernel",
            "bound": "hbm",
            "achieved": con_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": con_gbs / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": con_bytes,
            "ms_per_launch": con_ms,
        },
        "mfma": {
            "kernel": "contract_f64_kernel",
            "executed_tflops": mfma_flops / (con_ms * 1e-3) / 1e12,
            "peak_tflops": FP64_MFMA_PEAK_TF,
            "frac": mfma_flops / (con_ms * 1e-3) / 1e12 / FP64_MFMA_PEAK_TF,
            "algorithmic_tflops": alg_flops / (con_ms * 1e-3) / 1e12,
            "executed_flops_per_cell": info["mfma_k_per_tile"] * 32,
            "algorithmic_flops_per_cell": 2 * nnz,
        },
        "geometry_kernel": {
            "ms_per_launch": geo_ms,
            "achieved_gbs": geo_bytes / (geo_ms * 1e-3) / 1e9,
            "frac": geo_bytes / (geo_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes_per_launch": geo_bytes,
        },
        "path": {
            "algorithmic_bytes_per_step": path_bytes,
            "achieved_gbs": path_bytes / (ms_step * 1e-3) / 1e9,
            "hbm_lower_bound_ms": path_bytes / (HBM_PEAK_GBS * 1e9) * 1e3,
        },
    }

    if not args.no_quadrature:
        qform = Form("elasticity", 3, 2, kernel="quadrature")
        qout = qform.empty_out(cells)
        for _ in range(max(1, args.warmup)):
            qform.tabulate(X, out=qout)
        torch.cuda.synchronize()
        qe = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for a, b in qe:
            a.record(stream)
            qform.tabulate(X, out=qout)
            b.record(stream)
        torch.cuda.synchronize()
        q_ms = float(np.mean([a.elapsed_time(b) for a, b in qe]))
        npts = qform.info["quad_points"]
        q_flops = cells * n_I * npts * (2 + 2 * 3 + 1)  # n^2 N (n_f + n_D d + 1)-style count
        result["quadrature_kernel"] = {
            "value": cells / (q_ms * 1e-3),
            "unit": "element tensors/s",
            "ms_per_launch": q_ms,
            "quad_points": npts,
            "speedup_tensor_over_quadrature": (cells / (ms_step * 1e-3)) / (cells / (q_ms * 1e-3)),
            "achieved_gbs": path_bytes / (q_ms * 1e-3) / 1e9,
            "approx_fp64_tflops": q_flops / (q_ms * 1e-3) / 1e12,
        }
        del qout, qform

    if not args.no_cpu_baseline:
        import oracle

        threads = oracle.max_threads()
        calib = 500
        t = time.perf_counter()
        oracle.tabulate("elasticity", 3, 2, wl.coords[:, :calib])
        dt = time.perf_counter() - t
        sample = int(min(65536, max(calib, calib * args.cpu_seconds / max(dt, 1e-6))))
        sub = np.ascontiguousarray(wl.coords[:, :sample])
        t = time.perf_counter()
        ref = oracle.tabulate("elasticity", 3, 2, sub)
        dt = time.perf_counter() - t
        got = out[:sample].cpu().numpy().reshape(sample, -1)
        r = ref.reshape(sample, -1)
        err = np.linalg.norm(got - r, axis=1) / np.linalg.norm(r, axis=1)
        result["cpu_baseline"] = {
            "value": sample / dt,
            "unit": "element tensors/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"first {sample} cells of the same 750,000-cell mesh, FP64 quadrature on the "
                      f"physical cell, OpenMP over cells ({threads} threads), {dt:.1f} s wall",
        }
        result["rel_err_vs_oracle"] = {"max": float(err.max()), "median": float(np.median(err)),
                                       "cells": sample, "tol": 1e-12}

    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
