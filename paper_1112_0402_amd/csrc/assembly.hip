// Global assembly of element tensors into a CSR matrix (Sec. 2.2, Algorithm 2's insertion
// step).  Symbolic phase once per mesh: the pattern and, per matrix row, the element-tensor
// rows landing in it, on the host; every element entry's CSR index on the GPU.  Numeric
// phase: a row gather (one wave per matrix row, no atomics, fixed summation order).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <thread>

#include "assembly.h"

namespace ffc {

bool csr_pattern(int64_t cells, int n, const int32_t* dofmap, int64_t n_dofs, std::vector<int64_t>* row_ptr,
                 std::vector<int32_t>* col, std::vector<int64_t>* slot_ptr, std::vector<int32_t>* slots) {
    // dof -> incident cells
    std::vector<int64_t> inc_ptr(n_dofs + 1, 0);
    for (int64_t k = 0; k < cells * n; ++k) ++inc_ptr[dofmap[k] + 1];
    for (int64_t r = 0; r < n_dofs; ++r) inc_ptr[r + 1] += inc_ptr[r];
    std::vector<int64_t> inc(inc_ptr[n_dofs]);
    slots->assign(inc_ptr[n_dofs], 0);
    {
        std::vector<int64_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
        for (int64_t c = 0; c < cells; ++c)
            for (int i = 0; i < n; ++i) {
                const int64_t k = fill[dofmap[c * n + i]]++;
                inc[k] = c;
                (*slots)[k] = static_cast<int32_t>(c * n + i);
            }
    }
    *slot_ptr = inc_ptr;
    // rows in parallel: the union of the incident cells' dofs, sorted
    const int nt = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
    std::vector<std::vector<int32_t>> cols(nt);
    std::vector<std::vector<int64_t>> lens(nt);
    auto work = [&](int t) {
        const int64_t r0 = n_dofs * t / nt, r1 = n_dofs * (t + 1) / nt;
        std::vector<int32_t> buf;
        for (int64_t r = r0; r < r1; ++r) {
            buf.clear();
            for (int64_t k = inc_ptr[r]; k < inc_ptr[r + 1]; ++k) {
                const int32_t* dm = dofmap + inc[k] * n;
                buf.insert(buf.end(), dm, dm + n);
            }
            std::sort(buf.begin(), buf.end());
            buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
            cols[t].insert(cols[t].end(), buf.begin(), buf.end());
            lens[t].push_back(static_cast<int64_t>(buf.size()));
        }
    };
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(work, t);
    for (auto& x : th) x.join();
    row_ptr->assign(n_dofs + 1, 0);
    int64_t r = 0, nnz = 0;
    for (int t = 0; t < nt; ++t)
        for (int64_t len : lens[t]) {
            nnz += len;
            (*row_ptr)[++r] = nnz;
        }
    if (nnz >= (int64_t(1) << 31)) return false;
    col->clear();
    col->reserve(nnz);
    for (int t = 0; t < nt; ++t) col->insert(col->end(), cols[t].begin(), cols[t].end());
    return true;
}

namespace {

__global__ void positions_kernel(int64_t cells, int n, const int32_t* __restrict__ dofmap,
                                 const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                 uint16_t* __restrict__ pos) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nn = static_cast<int64_t>(n) * n;
    if (e >= cells * nn) return;
    const int64_t c = e / nn;
    const int k = static_cast<int>(e - c * nn);
    const int i = k / n, j = k - (k / n) * n;
    const int32_t r = dofmap[c * n + i], t = dofmap[c * n + j];
    int64_t lo = row_ptr[r], hi = row_ptr[r + 1] - 1;
    while (lo < hi) {  // first index with col >= t; t is in the row by construction
        const int64_t mid = (lo + hi) >> 1;
        if (col[mid] < t)
            lo = mid + 1;
        else
            hi = mid;
    }
    pos[e] = static_cast<uint16_t>(lo - row_ptr[r]);  // rows hold at most 1024 entries
}


constexpr int kRowWaves = 4;  // waves per workgroup of the gather

// RPW matrix rows per wave: 2 when an element-tensor row fits half a wave (n <= 32), the
// two halves then work on their own rows (own LDS buffers), doubling the loads in flight.
template <typename T, int RPW>
__global__ __launch_bounds__(64 * kRowWaves) void gather_rows_kernel(
    int64_t n_rows, int n, const int64_t* __restrict__ slot_ptr, const int32_t* __restrict__ slots,
    const T* __restrict__ tensors, const uint16_t* __restrict__ pos, const int64_t* __restrict__ row_ptr,
    double* __restrict__ values, int accumulate, int max_row) {
    extern __shared__ double rowbuf[];
    constexpr int L = 64 / RPW;  // lanes per row
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int h = lane / L, j = lane - h * L;
    const int64_t r = (static_cast<int64_t>(blockIdx.x) * kRowWaves + w) * RPW + h;
    const bool live = r < n_rows;
    double* b = rowbuf + static_cast<int64_t>(w * RPW + h) * max_row;
    const int64_t base = live ? row_ptr[r] : 0;
    const int len = live ? static_cast<int>(row_ptr[r + 1] - base) : 0;
    for (int k = j; k < len; k += L) b[k] = accumulate ? values[base + k] : 0.0;
    const int64_t s0 = live ? slot_ptr[r] : 0, s1 = live ? slot_ptr[r + 1] : 0;
    // LDS operations of one wave complete in issue order, so the slots' read-add-writes of a
    // shared entry follow one another; within a slot every lane has its own entry
    constexpr int U = 8;  // slots whose loads are in flight together
    for (int64_t s = s0; s < s1; s += U) {
        T v[U];
        int32_t p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            v[u] = T(0);
            p[u] = -1;
            if (s + u < s1 && j < n) {
                const int64_t e = static_cast<int64_t>(slots[s + u]) * n + j;
                v[u] = tensors[e];
                p[u] = pos[e];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (p[u] >= 0) b[p[u]] += static_cast<double>(v[u]);
    }
    for (int k = j; k < len; k += L) values[base + k] = b[k];
}

}  // namespace

hipError_t scatter_positions(int64_t cells, int n, const int32_t* dofmap, const int64_t* row_ptr, const int32_t* col,
                             uint16_t* pos, hipStream_t s) {
    const int64_t total = cells * n * n;
    if (total <= 0) return hipSuccess;
    positions_kernel<<<static_cast<unsigned>((total + 255) / 256), 256, 0, s>>>(cells, n, dofmap, row_ptr, col, pos);
    return hipGetLastError();
}


hipError_t gather_rows(int64_t n_rows, int n, const int64_t* slot_ptr, const int32_t* slots, const void* tensors,
                       int tensor_bytes, const uint16_t* pos, const int64_t* row_ptr, double* values, int accumulate,
                       int max_row, hipStream_t s) {
    if (n_rows <= 0) return hipSuccess;
    if (n > 64) return hipErrorInvalidValue;  // one lane per element-tensor column
    const int rpw = n <= 32 ? 2 : 1;
    const int64_t rows_per_block = static_cast<int64_t>(kRowWaves) * rpw;
    const unsigned g = static_cast<unsigned>((n_rows + rows_per_block - 1) / rows_per_block);
    const size_t lds = static_cast<size_t>(rows_per_block) * (max_row > 0 ? max_row : 1) * sizeof(double);
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    const unsigned block = 64 * kRowWaves;
    if (tensor_bytes == 4) {
        const float* t = static_cast<const float*>(tensors);
        if (rpw == 2)
            gather_rows_kernel<float, 2><<<g, block, lds, s>>>(n_rows, n, slot_ptr, slots, t, pos, row_ptr, values,
                                                               accumulate, max_row);
        else
            gather_rows_kernel<float, 1><<<g, block, lds, s>>>(n_rows, n, slot_ptr, slots, t, pos, row_ptr, values,
                                                               accumulate, max_row);
    } else {
        const double* t = static_cast<const double*>(tensors);
        if (rpw == 2)
            gather_rows_kernel<double, 2><<<g, block, lds, s>>>(n_rows, n, slot_ptr, slots, t, pos, row_ptr, values,
                                                                accumulate, max_row);
        else
            gather_rows_kernel<double, 1><<<g, block, lds, s>>>(n_rows, n, slot_ptr, slots, t, pos, row_ptr, values,
                                                                accumulate, max_row);
    }
    return hipGetLastError();
}

namespace {
__global__ void gather_local_kernel(int64_t m, const int32_t* __restrict__ dofmap, const double* __restrict__ x,
                                    double* __restrict__ xl) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < m) xl[k] = x[dofmap[k]];
}

__global__ void sum_slots_kernel(int64_t n_rows, const int64_t* __restrict__ slot_ptr,
                                 const int32_t* __restrict__ slots, const double* __restrict__ yl,
                                 double* __restrict__ y) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    double s = 0.0;
    const int64_t k0 = slot_ptr[r], k1 = slot_ptr[r + 1];
    // loads of eight (then four) slots in flight together, added in slot order (the same sum
    // as one slot at a time; each dof's slots are random reads of yl, so a lane otherwise
    // waits out one load latency per slot)
    int64_t k = k0;
    for (; k + 8 <= k1; k += 8) {
        int32_t a[8];
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = slots[k + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = yl[a[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; k + 4 <= k1; k += 4) {
        const int32_t a0 = slots[k], a1 = slots[k + 1], a2 = slots[k + 2], a3 = slots[k + 3];
        const double v0 = yl[a0], v1 = yl[a1], v2 = yl[a2], v3 = yl[a3];
        s += v0;
        s += v1;
        s += v2;
        s += v3;
    }
    for (; k < k1; ++k) s += yl[slots[k]];
    y[r] = s;
}
}  // namespace

hipError_t gather_local(int64_t m, const int32_t* dofmap, const double* x, double* xl, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    gather_local_kernel<<<static_cast<unsigned>((m + 255) / 256), 256, 0, s>>>(m, dofmap, x, xl);
    return hipGetLastError();
}

hipError_t sum_slots(int64_t n_rows, const int64_t* slot_ptr, const int32_t* slots, const double* yl, double* y,
                     hipStream_t s) {
    if (n_rows <= 0) return hipSuccess;
    sum_slots_kernel<<<static_cast<unsigned>((n_rows + 255) / 256), 256, 0, s>>>(n_rows, slot_ptr, slots, yl, y);
    return hipGetLastError();
}

}  // namespace ffc
