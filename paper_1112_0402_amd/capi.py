"""ctypes binding of libffc_hip.so: argument marshalling only.

Every step of the tabulation runs in the library's HIP kernels; this module only turns
torch CUDA tensors into device pointers and streams.  There is no fallback: if the
library is missing, or no gfx950 device is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libffc_hip.so")

KINDS = {"mass": 0, "laplace": 1, "wlaplace": 2, "elasticity": 3, "ns": 4, "piola": 5, "curved": 6, "nedelec": 7}
PRECISIONS = {"fp64": 0, "bf16x3": 1, "bf16x6": 2}
KERNELS = {"auto": 0, "tensor": 1, "quadrature": 2}
GEOMETRY = {"default": 0, "pass": 1, "fused": 2}

FFC_OK = 0
FFC_E_INVALID = -1
FFC_E_UNSUPPORTED = -2
FFC_E_DEVICE = -3
FFC_E_DEGENERATE = -4
FFC_E_NOMEM = -5


class FormDesc(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("dim", ctypes.c_int32),
        ("degree", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("kernel", ctypes.c_int32),
        ("tile_cells", ctypes.c_int32),
        ("waves", ctypes.c_int32),
        ("tile_window", ctypes.c_int32),
        ("persistent", ctypes.c_int32),
        ("geometry", ctypes.c_int32),
        ("symmetry", ctypes.c_int32),
        ("lambda_", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("stream", ctypes.c_void_p),
    ]


class FormInfo(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "n_dofs", "n_entries", "n_alpha", "nnz_a0", "n_coords", "n_coeffs", "out_bytes",
        "mfma_k_per_tile", "n_tiles", "quad_points", "persistent_waves", "persistent_kmax", "tile_cells",
        "waves", "fused_geometry", "g_entries", "symmetric", "auto_launches")]


class FFCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ffc error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libffc_hip.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc for gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int32
    L.ffc_last_error.restype = ctypes.c_char_p
    L.ffc_version.restype = ctypes.c_char_p
    L.ffc_compile_reference_tensor.argtypes = [ctypes.POINTER(FormDesc), ctypes.POINTER(i64), ctypes.POINTER(i64), vp]
    L.ffc_form_create.argtypes = [ctypes.POINTER(FormDesc), ctypes.POINTER(vp)]
    L.ffc_form_get_info.argtypes = [vp, ctypes.POINTER(FormInfo)]
    L.ffc_form_select.argtypes = [vp, i64, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.ffc_form_destroy.argtypes = [vp]
    L.ffc_form_destroy.restype = None
    L.ffc_tabulate_tensor.argtypes = [vp, i64, vp, vp, vp]
    L.ffc_tabulate_tensor_affine.argtypes = [vp, i64, vp, vp, vp]
    L.ffc_apply_tensor.argtypes = [vp, i64, vp, vp, vp, vp]
    L.ffc_compute_geometry.argtypes = [i32, i64, vp, vp, vp]
    L.ffc_check_cells.argtypes = [i32, i64, vp, ctypes.c_double, ctypes.POINTER(i64), ctypes.POINTER(i64), vp]
    L.ffc_batch_create.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(vp),
                                   ctypes.POINTER(vp), ctypes.POINTER(vp), vp, ctypes.POINTER(vp)]
    L.ffc_batch_run.argtypes = [vp]
    L.ffc_batch_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.ffc_batch_destroy.argtypes = [vp]
    L.ffc_batch_destroy.restype = None
    L.ffc_assembly_create.argtypes = [i64, i32, vp, i64, vp, ctypes.POINTER(vp)]
    L.ffc_assembly_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.ffc_assembly_pattern.argtypes = [vp, vp, vp]
    L.ffc_assemble.argtypes = [vp, vp, i32, vp, i32]
    L.ffc_operator_apply.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.ffc_operator_apply_noalloc.argtypes = [vp, vp, vp, vp, vp, vp]
    L.ffc_assembly_destroy.argtypes = [vp]
    L.ffc_assembly_destroy.restype = None
    for name in ("ffc_assembly_create", "ffc_assembly_info", "ffc_assembly_pattern", "ffc_assemble",
                 "ffc_operator_apply", "ffc_operator_apply_noalloc"):
        getattr(L, name).restype = ctypes.c_int
    fp = ctypes.c_float
    L.ffc_mlp_param_count.argtypes = [i32, i32, i32]
    L.ffc_mlp_param_count.restype = i64
    L.ffc_mlp_forward.argtypes = [i32, i32, i32, i64, vp, vp, vp, vp, vp]
    L.ffc_mlp_backward.argtypes = [i32, i32, i32, i64, vp, vp, vp, vp, vp, vp, vp]
    L.ffc_mlp_mse.argtypes = [i64, vp, vp, vp, vp, vp, vp]
    L.ffc_adam_step.argtypes = [i64, vp, vp, vp, vp, fp, fp, fp, fp, fp, i32, vp]
    for name in ("ffc_mlp_forward", "ffc_mlp_backward", "ffc_mlp_mse", "ffc_adam_step"):
        getattr(L, name).restype = ctypes.c_int
    for name in ("ffc_compile_reference_tensor", "ffc_form_create", "ffc_form_get_info", "ffc_form_select",
                 "ffc_tabulate_tensor",
                 "ffc_tabulate_tensor_affine", "ffc_apply_tensor",
                 "ffc_compute_geometry", "ffc_check_cells", "ffc_batch_create", "ffc_batch_run", "ffc_batch_info"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != FFC_OK:
        raise FFCError(rc, lib().ffc_last_error().decode())


def make_desc(kind, dim, degree, precision="fp64", kernel="tensor", tile_cells=0, waves=0,
              lam=1.0, mu=1.0, stream=None, tile_window=0, persistent=0, geometry=0, symmetry=0) -> FormDesc:
    d = FormDesc()
    d.kind = KINDS[kind] if isinstance(kind, str) else int(kind)
    d.dim = dim
    d.degree = degree
    d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    d.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    d.tile_cells = tile_cells
    d.waves = waves
    d.tile_window = tile_window
    d.persistent = persistent
    d.geometry = GEOMETRY[geometry] if isinstance(geometry, str) else int(geometry)
    d.symmetry = int(symmetry)
    d.lambda_ = lam
    d.mu = mu
    d.stream = stream
    return d


def reference_tensor(kind, dim, degree, lam=1.0, mu=1.0) -> np.ndarray:
    """A^0 [n_I, n_alpha] from the compile step (host only, no device needed)."""
    L = lib()
    d = make_desc(kind, dim, degree, lam=lam, mu=mu)
    nI = ctypes.c_int64()
    na = ctypes.c_int64()
    check(L.ffc_compile_reference_tensor(ctypes.byref(d), ctypes.byref(nI), ctypes.byref(na), None))
    A0 = np.zeros((nI.value, na.value), dtype=np.float64)
    check(L.ffc_compile_reference_tensor(ctypes.byref(d), ctypes.byref(nI), ctypes.byref(na),
                                         A0.ctypes.data_as(ctypes.c_void_p)))
    return A0


def exported_symbols() -> list[str]:
    """Names of the functions declared in include/ffc_hip.h that the library exports."""
    L = lib()
    out = []
    import re
    hdr = os.path.join(os.path.dirname(_HERE), "include", "ffc_hip.h")
    names = re.findall(r"\b(ffc_[a-z_]+)\s*\(", open(hdr).read())
    for n in sorted(set(names)):
        if hasattr(L, n):
            out.append(n)
    return out


def declared_symbols() -> list[str]:
    import re
    hdr = os.path.join(os.path.dirname(_HERE), "include", "ffc_hip.h")
    return sorted(set(re.findall(r"\b(ffc_[a-z_]+)\s*\(", open(hdr).read())))
