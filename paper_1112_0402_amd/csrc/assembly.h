// Global assembly: the insertion step of the element-by-element assembly algorithm
// (Sec. 2.2, Algorithm 2), A = sum over cells K of P_K^T A^K P_K, into a CSR matrix.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace ffc {

// CSR sparsity pattern of the assembled matrix on the host: row r holds every dof that
// shares a cell with dof r, columns ascending.  dofmap [cells][n] (test = trial map).
// Also the element-tensor rows that land in each matrix row: slots[slot_ptr[r] ..
// slot_ptr[r+1]) = c * n + i for every (cell c, local row i) with dofmap[c][i] = r,
// ascending.  Returns false if the pattern would have 2^31 or more entries.
bool csr_pattern(int64_t cells, int n, const int32_t* dofmap, int64_t n_dofs, std::vector<int64_t>* row_ptr,
                 std::vector<int32_t>* col, std::vector<int64_t>* slot_ptr, std::vector<int32_t>* slots);

// pos[c][i][j] = index of entry (dofmap[c][i], dofmap[c][j]) within its CSR row, i.e. its
// CSR index minus the row start (binary search in the row; rows of at most 1024 entries)
hipError_t scatter_positions(int64_t cells, int n, const int32_t* dofmap, const int64_t* row_ptr, const int32_t* col,
                             uint16_t* pos, hipStream_t s);
// Row gather: one wave per matrix row r sums, in slot order, the element-tensor rows that
// land in r (each read as one contiguous run) into an LDS copy of the CSR row at the
// entries' in-row indices pos, then writes the row once (plus its previous values if
// accumulate).  No atomics, a fixed summation order.  tensors FP64 (tensor_bytes 8) or
// FP32 (4, split-BF16 output); max_row = the longest CSR row.
hipError_t gather_rows(int64_t n_rows, int n, const int64_t* slot_ptr, const int32_t* slots, const void* tensors,
                       int tensor_bytes, const uint16_t* pos, const int64_t* row_ptr, double* values, int accumulate,
                       int max_row, hipStream_t s);

// Matrix-free operator steps.  Gather: xl[k] = x[dofmap[k]] for k < m (m = cells * n).
// Sum: y[r] = sum of yl[slots[k]] over the slots of dof r, in slot order (one lane per dof;
// every dof is written, 0 where no cell touches it).
hipError_t gather_local(int64_t m, const int32_t* dofmap, const double* x, double* xl, hipStream_t s);
hipError_t sum_slots(int64_t n_rows, const int64_t* slot_ptr, const int32_t* slots, const double* yl, double* y,
                     hipStream_t s);

}  // namespace ffc
