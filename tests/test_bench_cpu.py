"""Host-side checks of bench.py: the one-GPU contract, the traffic summary reader and the
quadrature operation count."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_summary_reader():
    # a summary is used only for its own workload size and the kernel source it was taken on
    assert bench.load_traffic("elasticity3d_p2_750k", 1) is None
    assert bench.load_traffic("no_such_workload", 750000) is None
    t = bench.load_traffic("elasticity3d_p2_750k", 750000)
    if t is not None:  # taken on the current kernel source: HBM bytes near the algorithmic 7,280 B/cell
        assert 1.0 <= t / (750000 * 7280) < 1.1


def test_quadrature_operation_count():
    # Sec. 4.3's count for the three benchmarked forms: elasticity P2 3D (30 dofs, 8 points),
    # weighted Laplace P3 3D (20 dofs, 27 points), P1 Laplacian on triangles (1 point)
    assert bench.quadrature_model_flops("elasticity", 900, 8, 3) == 50_400
    assert bench.quadrature_model_flops("wlaplace", 400, 27, 3) == 86_400
    assert bench.quadrature_model_flops("laplace", 9, 1, 2) == 45
    assert bench.quadrature_model_flops("mass", 16, 4, 3) == 64


def test_oracle_pass_covers_every_cell_in_chunks():
    import numpy as np

    import oracle
    from paper_1112_0402_amd import meshgen

    wl = meshgen.make_workload("wlaplace", 2, 2, 5, 1)  # 50 cells, chunks of 7 leave a ragged tail
    ref = oracle.tabulate("wlaplace", 2, 2, wl.coords, wl.coeffs)
    base, errs = bench.oracle_pass(wl, {"same": lambda c0, c1: ref[c0:c1],
                                        "scaled": lambda c0, c1: ref[c0:c1] * (1 + 1e-9)}, np, chunk=7)
    assert errs["same"]["max"] == 0.0 and errs["same"]["cells"] == wl.cells
    assert abs(errs["scaled"]["max"] - 1e-9) < 1e-12
    assert base["kind"] == "oracle" and base["value"] > 0 and base["sample"].startswith("every cell")
    base, errs = bench.oracle_pass(wl, {"same": lambda c0, c1: ref[c0:c1]}, np, cells=12, chunk=5)
    assert errs["same"]["cells"] == 12 and base["sample"].startswith("first 12 cells")
