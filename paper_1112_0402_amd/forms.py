"""Form handles, tabulation and batches over torch CUDA tensors (ctypes marshalling only;
every step runs in libffc_hip's HIP kernels)."""
from __future__ import annotations

import ctypes

import numpy as np

import torch

from . import capi


def _stream_handle(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _check_tensor(name, t, dtype, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Form:
    """A compiled form on the current device (compile step + upload happen here)."""

    def __init__(self, kind, dim, degree, precision="fp64", kernel="tensor", tile_cells=0, waves=0,
                 lam=1.0, mu=1.0, stream=None, tile_window=0, persistent=0, geometry=0, symmetry=0):
        self.kind, self.dim, self.degree = kind, dim, degree
        self.precision, self.kernel = precision, kernel
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._desc = capi.make_desc(kind, dim, degree, precision, kernel, tile_cells, waves, lam, mu,
                                    _stream_handle(self.stream), tile_window, persistent, geometry, symmetry)
        h = ctypes.c_void_p()
        capi.check(capi.lib().ffc_form_create(ctypes.byref(self._desc), ctypes.byref(h)))
        self._h = h
        info = capi.FormInfo()
        capi.check(capi.lib().ffc_form_get_info(h, ctypes.byref(info)))
        self.info = {name: getattr(info, name) for name, _ in capi.FormInfo._fields_}
        self.n = self.info["n_dofs"]
        self.n_I = self.info["n_entries"]
        self.out_dtype = torch.float32 if self.info["out_bytes"] == 4 else torch.float64

    @property
    def handle(self):
        return self._h

    def empty_out(self, cells: int) -> torch.Tensor:
        return torch.empty((cells, self.n, self.n), dtype=self.out_dtype, device="cuda")

    def tabulate(self, coords: torch.Tensor, coeffs: torch.Tensor | None = None,
                 out: torch.Tensor | None = None) -> torch.Tensor:
        """Element tensors [cells, n, n] (row = test function), enqueued on the form's stream."""
        d = self.dim
        _check_tensor("coords", coords, torch.float64)
        nc = self.info["n_coords"]
        if coords.dim() != 2 or coords.shape[0] != nc:
            raise ValueError(f"coords must be [{nc}, cells]")
        cells = coords.shape[1]
        if self.info["n_coeffs"]:
            if coeffs is None:
                raise ValueError(f"form {self.kind} needs coefficients [{self.info['n_coeffs']}, cells]")
            _check_tensor("coeffs", coeffs, torch.float64, (self.info["n_coeffs"], cells))
        if out is None:
            out = self.empty_out(cells)
        _check_tensor("out", out, self.out_dtype)
        if out.numel() != cells * self.n_I:
            raise ValueError("out has the wrong number of entries")
        capi.check(capi.lib().ffc_tabulate_tensor(self._h, cells, _ptr(coords), _ptr(coeffs), _ptr(out)))
        return out

    def tabulate_affine(self, affine_map: torch.Tensor, coeffs: torch.Tensor | None = None,
                        out: torch.Tensor | None = None) -> torch.Tensor:
        """Contraction only, from an affine map [1 + d*d, cells] of compute_geometry()."""
        d = self.dim
        _check_tensor("affine_map", affine_map, torch.float64)
        if affine_map.dim() != 2 or affine_map.shape[0] != 1 + d * d:
            raise ValueError(f"affine_map must be [{1 + d * d}, cells]")
        cells = affine_map.shape[1]
        if self.info["n_coeffs"]:
            if coeffs is None:
                raise ValueError(f"form {self.kind} needs coefficients")
            _check_tensor("coeffs", coeffs, torch.float64, (self.info["n_coeffs"], cells))
        if out is None:
            out = self.empty_out(cells)
        _check_tensor("out", out, self.out_dtype)
        if out.numel() != cells * self.n_I:
            raise ValueError("out has the wrong number of entries")
        capi.check(capi.lib().ffc_tabulate_tensor_affine(self._h, cells, _ptr(affine_map), _ptr(coeffs), _ptr(out)))
        return out

    def apply(self, coords: torch.Tensor, x: torch.Tensor, coeffs: torch.Tensor | None = None,
              y: torch.Tensor | None = None) -> torch.Tensor:
        """Operator action y_K = A^K x_K per cell (x, y: [cells, n] FP64), without writing
        the element tensors; FP64 tensor-kernel forms."""
        d = self.dim
        _check_tensor("coords", coords, torch.float64)
        nc = self.info["n_coords"]
        if coords.dim() != 2 or coords.shape[0] != nc:
            raise ValueError(f"coords must be [{nc}, cells]")
        cells, n = coords.shape[1], self.info["n_dofs"]
        if self.info["n_coeffs"]:
            if coeffs is None:
                raise ValueError(f"form {self.kind} needs coefficients [{self.info['n_coeffs']}, cells]")
            _check_tensor("coeffs", coeffs, torch.float64, (self.info["n_coeffs"], cells))
        _check_tensor("x", x, torch.float64)
        if x.numel() != cells * n:
            raise ValueError(f"x must hold [cells, n] = [{cells}, {n}] values")
        if y is None:
            y = torch.empty((cells, n), dtype=torch.float64, device=coords.device)
        _check_tensor("y", y, torch.float64)
        if y.numel() != cells * n:
            raise ValueError("y has the wrong number of entries")
        capi.check(capi.lib().ffc_apply_tensor(self._h, cells, _ptr(coords), _ptr(coeffs), _ptr(x), _ptr(y)))
        return y

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            capi.lib().ffc_form_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def check_cells(coords: torch.Tensor, dim: int, tol: float = 0.0, stream=None):
    """Validation mode: (number of degenerate cells, smallest such index or -1); a cell is
    degenerate when |det J| <= tol * h^d (h its longest edge) or det J is not finite.  Does
    not raise for degenerate cells (the C call returns FFC_E_DEGENERATE for them)."""
    _check_tensor("coords", coords, torch.float64)
    count, first = ctypes.c_int64(), ctypes.c_int64()
    rc = capi.lib().ffc_check_cells(dim, coords.shape[1], _ptr(coords), float(tol), ctypes.byref(count),
                                    ctypes.byref(first), _stream_handle(stream))
    if rc not in (capi.FFC_OK, capi.FFC_E_DEGENERATE):
        capi.check(rc)
    return count.value, first.value


def compute_geometry(coords: torch.Tensor, dim: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Affine map per cell: [1 + d*d, cells] (det J, then g_ab = (J^{-1})_ab)."""
    _check_tensor("coords", coords, torch.float64)
    cells = coords.shape[1]
    if out is None:
        out = torch.empty((1 + dim * dim, cells), dtype=torch.float64, device=coords.device)
    _check_tensor("affine_map", out, torch.float64, (1 + dim * dim, cells))
    capi.check(capi.lib().ffc_compute_geometry(dim, cells, _ptr(coords), _ptr(out), _stream_handle(stream)))
    return out


class Batch:
    """Many (form, mesh) items evaluated by a short fixed sequence of launches: one
    persistent launch per form whose element tensors use a persistent kernel (after the
    items' geometry passes) and one tile launch per group of the other items."""

    def __init__(self, forms, coords, coeffs, outs, stream=None):
        n = len(forms)
        self.forms, self.coords, self.coeffs, self.outs = list(forms), list(coords), list(coeffs), list(outs)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        vp = ctypes.c_void_p
        F = (vp * n)(*[f.handle.value for f in forms])
        C = (ctypes.c_int64 * n)(*[int(c.shape[1]) for c in coords])
        X = (vp * n)(*[c.data_ptr() for c in coords])
        K = (vp * n)(*[(k.data_ptr() if k is not None else None) for k in coeffs])
        O = (vp * n)(*[o.data_ptr() for o in outs])
        for f, c, k, o in zip(forms, coords, coeffs, outs):
            _check_tensor("coords", c, torch.float64)
            if k is not None:
                _check_tensor("coeffs", k, torch.float64)
            _check_tensor("out", o, f.out_dtype)
            if o.numel() != c.shape[1] * f.n_I:
                raise ValueError("batch output of the wrong size")
        h = vp()
        capi.check(capi.lib().ffc_batch_create(n, F, C, X, K, O, _stream_handle(self.stream), ctypes.byref(h)))
        self._h = h
        tc, wu, gr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        capi.check(capi.lib().ffc_batch_info(h, ctypes.byref(tc), ctypes.byref(wu), ctypes.byref(gr)))
        self.total_cells, self.work_units, self.launches = tc.value, wu.value, gr.value

    def run(self):
        capi.check(capi.lib().ffc_batch_run(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            capi.lib().ffc_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SourceForm:
    """The linear form L(v) = int f v dx with f in the same Lagrange P_q space as v (the
    right-hand side of the Poisson form file, Sec. 5.5).  Its tensor representation is
    b_K,i = A^0_{ia} G_K,a with A^0_{ia} = int_K0 Phi_i Phi_a and G_K,a = |det J| f_a: the mass
    form's reference tensor contracted with the cell's f dofs, so b_K is the mass form's
    operator action on f_K (ffc_apply_tensor), and the assembled load vector is
    Assembly.apply(form.mass, coords, f)."""

    def __init__(self, dim, degree, stream=None):
        self.dim, self.degree = dim, degree
        self.mass = Form("mass", dim, degree, stream=stream)

    def tabulate(self, coords: torch.Tensor, f_local: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Element vectors [cells, n] from the nodal values of f on each cell [cells, n]."""
        return self.mass.apply(coords, f_local, y=out)


class Assembly:
    """Global assembly into CSR (the insertion step of Algorithm 2): the pattern and the
    CSR index of every element-tensor entry are built once from a local-to-global map."""

    def __init__(self, dofmap: np.ndarray, n_global: int, stream=None):
        dm = np.ascontiguousarray(dofmap, dtype=np.int32)
        if dm.ndim != 2:
            raise ValueError("dofmap must be [cells, n_local]")
        self.cells, self.n_local = dm.shape
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        capi.check(capi.lib().ffc_assembly_create(self.cells, self.n_local, dm.ctypes.data, int(n_global),
                                                  _stream_handle(self.stream), ctypes.byref(h)))
        self._h = h
        nr, nz = ctypes.c_int64(), ctypes.c_int64()
        capi.check(capi.lib().ffc_assembly_info(h, ctypes.byref(nr), ctypes.byref(nz)))
        self.n_rows, self.nnz = nr.value, nz.value

    def pattern(self):
        """(row_ptr int64 [n_rows + 1], col_idx int32 [nnz]) on the host."""
        rp = np.empty(self.n_rows + 1, dtype=np.int64)
        ci = np.empty(max(self.nnz, 1), dtype=np.int32)
        capi.check(capi.lib().ffc_assembly_pattern(self._h, rp.ctypes.data, ci.ctypes.data))
        return rp, ci[: self.nnz]

    def assemble(self, tensors: torch.Tensor, values: torch.Tensor | None = None, accumulate: bool = False):
        """CSR values [nnz] (FP64) of the sum of the element tensors [cells, n, n]."""
        if tensors.dtype not in (torch.float64, torch.float32):
            raise TypeError("element tensors must be float64 or float32")
        _check_tensor("element_tensors", tensors, tensors.dtype)
        if tensors.numel() != self.cells * self.n_local * self.n_local:
            raise ValueError("element tensors of the wrong size")
        if values is None:
            values = torch.empty(self.nnz, dtype=torch.float64, device="cuda")
        _check_tensor("values", values, torch.float64, (self.nnz,))
        capi.check(capi.lib().ffc_assemble(self._h, _ptr(tensors), 8 if tensors.dtype == torch.float64 else 4,
                                           _ptr(values), 1 if accumulate else 0))
        return values

    def apply(self, form: "Form", coords: torch.Tensor, x: torch.Tensor, coeffs: torch.Tensor | None = None,
              y: torch.Tensor | None = None, work: torch.Tensor | None = None) -> torch.Tensor:
        """Matrix-free y = A x (x, y: [n_rows] FP64) for the matrix `form` would assemble on
        this mesh; work: optional scratch of 2 * cells * n_local doubles."""
        _check_tensor("coords", coords, torch.float64)
        if coords.dim() != 2 or coords.shape[1] != self.cells:
            raise ValueError(f"coords must be [(d+1)*d, {self.cells}]")
        if form.info["n_coeffs"]:
            if coeffs is None:
                raise ValueError(f"form {form.kind} needs coefficients")
            _check_tensor("coeffs", coeffs, torch.float64, (form.info["n_coeffs"], self.cells))
        _check_tensor("x", x, torch.float64, (self.n_rows,))
        if y is None:
            y = torch.empty(self.n_rows, dtype=torch.float64, device="cuda")
        _check_tensor("y", y, torch.float64, (self.n_rows,))
        if work is None:
            work = torch.empty(2 * self.cells * self.n_local, dtype=torch.float64, device="cuda")
        _check_tensor("work", work, torch.float64)
        if work.numel() < 2 * self.cells * self.n_local:
            raise ValueError("work holds fewer than 2 * cells * n_local doubles")
        capi.check(capi.lib().ffc_operator_apply(self._h, form._h, _ptr(coords), _ptr(coeffs), _ptr(x), _ptr(y),
                                                 _ptr(work)))
        return y

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            capi.lib().ffc_assembly_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
