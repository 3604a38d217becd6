"""Build libffc_hip.so (HIP kernels for gfx950 + the C-ABI + the host compile step)
in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libffc_hip.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # never emit packed-FP32 instructions (wrong results seen with some of their forms)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wall",
]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = True) -> str:
    """Compile every source (in parallel: the objects are independent), then link."""
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    # host-only compile step
    o = os.path.join(objdir, "reference_tensor.o")
    jobs.append((["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-c", os.path.join(CSRC, "reference_tensor.cpp"),
                  "-o", o], o))
    kernel_units = sorted(f for f in os.listdir(CSRC) if f.startswith("kernels_") and f.endswith(".hip"))
    for src in (*kernel_units, "mlp.hip", "assembly.hip", "capi.cpp"):
        o = os.path.join(objdir, src.split(".")[0] + ".o")
        extra = ["-x", "hip"] if src.endswith(".cpp") else []
        jobs.append(([HIPCC, *HIP_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", o], o))
    procs = []
    for cmd, _ in jobs:
        print("+", " ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    failed = [cmd for (cmd, _), p in zip(jobs, procs) if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *[o for _, o in jobs]])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
