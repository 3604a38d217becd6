// Device kernels of the tabulation path and their host-side launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ffc {

struct ContractArgs {
    int64_t cells;          // cells handled by this launch
    const double* amap;     // affine map SoA [1 + d*d][astride]: det J, then g_ab
    int64_t astride;
    const double* coeffs;   // SoA [n_coeff][cstride] or nullptr
    int64_t cstride;
    void* out;              // [cells][n_I] double or float
    int n_I, n_alpha, n_tiles;
    double lambda, mu;      // unused by the contraction (inside A^0), kept for symmetry
    // FP64 tiles
    const int32_t* koff;    // [n_tiles + 1]
    const uint32_t* apack;  // [koff[n_tiles] / 4] alpha indices, 4 per word
    const int32_t* entry;   // [n_tiles][16] output entry per tile column, -1 = padding
    const double* b;        // [koff[n_tiles]][16]
    // BF16 tiles
    const uint16_t* bb;     // [n_tiles][kpad/8][16][8]
    const uint8_t* nonzero; // [n_tiles]
    int kpad, n_seg;
    int gpiece[6];
    // LDS plan, filled by launch_contract
    int staged;
    size_t stage_bytes, head_bytes;
};

// LDS budget of one workgroup (gfx950: 160 KiB per CU; a little kept for static LDS).
constexpr size_t kLdsBudget = 160 * 1024 - 256;

struct LdsPlan {
    bool staged;
    size_t stage_bytes, head_bytes, g_bytes, total;
};
LdsPlan plan_lds(int dim, int kind, int tile_cells, int n_I, int n_alpha, int kpad, bool bf16, size_t budget);

struct QuadArgs {
    int64_t cells;
    const double* coords;  // SoA [(d+1)*d][cstride]
    int64_t cstride;
    const double* coeffs;  // SoA [n_coeff][kstride] or nullptr
    int64_t kstride;
    double* out;           // [cells][n_I]
    int ns, n, n_I, npts;
    const double* pts;     // [npts][d]
    const double* wts;     // [npts]
    const double* phi;     // [npts][ns]
    const double* dphi;    // [npts][ns][d]
    double lambda, mu;
    int cells_per_block;
};

hipError_t launch_geometry(int dim, int64_t cells, const double* coords, int64_t cstride, double* amap,
                           int64_t astride, hipStream_t stream);
hipError_t launch_contract(int dim, int kind, bool bf16, int tile_cells, int waves, ContractArgs a,
                           hipStream_t stream);

// Persistent FP64 contraction: 16-cell tiles, output rows staged in LDS, each wave's share
// of the A^0 tiles (B fragments and alpha offsets, at most kmax k steps) held in registers.
struct PersistArgs {
    const int32_t* woff;          // [waves + 1]
    const int32_t* step_kstep;    // [steps]
    const int32_t* step_end;      // [steps]
    const int32_t* zero_entries;  // [n_zero]
    int n_zero;
};
// Waves of a persistent workgroup that only write the staged output out (the others run
// the MFMA steps); a schedule for W waves is built over W - kIoWaves compute waves.
constexpr int kIoWaves = 6;
// 16-byte register slots per I/O lane holding a staged tile (16 rows of up to 912 doubles)
constexpr int kIoSlots = 20;
// Returns hipErrorInvalidValue when the form does not fit this kernel (caller falls back).
hipError_t launch_contract_persistent(int dim, int kind, int kmax, int waves, int grid, ContractArgs a,
                                      const PersistArgs& p, hipStream_t stream);
hipError_t launch_quadrature(int dim, int kind, const QuadArgs& a, hipStream_t stream);
size_t contract_lds_bytes(int dim, int kind, int tile_cells, int n_I, int n_alpha, int kpad, bool bf16);
int quad_cells_per_block(int dim, int kind, int ns, int npts);

// Persistent mixed-batch kernel: one descriptor per item (a mesh with its form).
struct BatchItem {
    int64_t cells;
    int64_t unit_begin;     // first work unit of this item (prefix sum)
    const double* coords;   // SoA [(d+1)*d][cells]
    const double* coeffs;   // SoA or nullptr
    void* out;
    int32_t dim, kind, n_I, n_alpha, n_tiles, kpad, n_seg, n_coeff;
    const int32_t* koff;
    const uint32_t* apack;
    const int32_t* entry;
    const double* b;
    const uint16_t* bb;
    const uint8_t* nonzero;
    int32_t gpiece[6];
};

// persistent batch: 16-cell work units claimed kBatchChunk at a time, kBatchWaves waves
constexpr int kBatchCT = 16;
constexpr int kBatchChunk = 4;
constexpr int kBatchWaves = 16;
constexpr int kBatchMaxCoeff = 12;
hipError_t launch_batch(const BatchItem* items_dev, int n_items, int64_t total_units, int* counter_dev,
                        int grid, bool bf16, size_t lds_bytes, size_t stage_cap, hipStream_t stream);
size_t batch_lds_bytes(int max_alpha, int max_kpad, int max_stage_nI, bool bf16);

}  // namespace ffc
