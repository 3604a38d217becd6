"""Oracle for global assembly -- TEST INFRASTRUCTURE ONLY (tests, smoke() and the bench's
CPU baseline use it; the library never does).

The plain definition of the element-by-element algorithm (Sec. 2.2, Algorithms 1 and 2):
A = sum over cells K of P_K^T A^K P_K, i.e. every element-tensor entry A^K_{ij} added to
the global entry (iota(K, i), iota(K, j)).  Written as a coordinate list summed by
scipy.sparse (a library primitive: duplicates are added on conversion to CSR)."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def assemble(tensors: np.ndarray, dofmap: np.ndarray, n_global: int) -> sp.csr_matrix:
    """tensors [cells, n, n] (row = test function), dofmap [cells, n] -> CSR [n_global]^2
    with sorted column indices (explicit zeros kept: the pattern is every dof pair that
    shares a cell)."""
    nc, n = dofmap.shape
    t = np.asarray(tensors, dtype=np.float64).reshape(nc, n, n)
    rows = np.broadcast_to(dofmap[:, :, None], (nc, n, n)).reshape(-1)
    cols = np.broadcast_to(dofmap[:, None, :], (nc, n, n)).reshape(-1)
    A = sp.coo_matrix((t.reshape(-1), (rows, cols)), shape=(n_global, n_global)).tocsr()
    A.sort_indices()
    return A
