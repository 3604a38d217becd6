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
    const double* coords;   // non-null: SoA [(d+1)*d][cells] coordinates, affine map computed
                            // per tile in LDS (amap unused; tile kernels only)
    void* out;              // [cells][n_I] double or float
    int n_I, n_alpha, n_tiles;
    int sym_n;              // FP64 tiles of a symmetric form: element dofs (tiles hold the
                            // entries i1 <= i2; each result also goes to i2 * n + i1); else 0
    double lambda, mu;      // unused by the contraction (inside A^0)
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
    // operator action (y_K = A^K x_K): local vectors x [cells][n_dof]; out = y [cells][n_dof]
    const double* xloc;
    int n_dof;
    // curvilinear cells with coords (G built in the tile): geometry basis gradients at the
    // quadrature points [n_pts][n_geo][dim]
    const double* geo_grad;
    int n_pts;
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

// out[0] = number of cells with |det J| <= tol * h^D (h = longest edge) or det J not finite,
// out[1] = the smallest such index (~0 if none); out: 2 device words
hipError_t launch_degenerate_cells(int dim, int64_t cells, const double* coords, double tol, unsigned long long* out,
                                   hipStream_t stream);
hipError_t launch_geometry(int dim, int64_t cells, const double* coords, int64_t cstride, double* amap,
                           int64_t astride, hipStream_t stream);
// Cells with P2 geometry: coords SoA [n_geo * dim][cstride] (P2 nodes in the dof order), grad
// [n_pts][n_geo][dim] reference gradients of the P2 basis at the quadrature points; writes
// G SoA [n_pts * dim(dim+1)/2][gstride] (|det J| (g g^T)_ab at each point, pairs a <= b).
hipError_t launch_curved_geometry(int dim, int64_t cells, const double* coords, int64_t cstride, int n_pts,
                                  const double* grad, double* G, int64_t gstride, hipStream_t stream);
hipError_t launch_contract(int dim, int kind, bool bf16, int tile_cells, int waves, ContractArgs a,
                           hipStream_t stream);

// Persistent FP64 contraction: 16-cell tiles, output rows staged in LDS, each wave's share
// of the A^0 tiles (B fragments and alpha offsets, at most kmax k steps) held in registers.
struct PersistArgs {
    const int32_t* woff;          // [compute waves + 1] step range of each wave
    // per compute wave w, step s (s < kmax, zero past the wave's steps) and lane l:
    const double* wave_b;         // [w][s][l] B fragment value
    const uint32_t* wave_word;    // [w][s][l] LDS column of the alpha | (output entry + 1) << 8
                                  // | (transposed entry + 1) << 20 (symmetric forms, else 0)
    const uint32_t* wave_mask;    // [w] bit s: step s ends a tile
    const int32_t* zero_entries;  // [n_zero]
    int n_zero;
};
// Waves of a persistent workgroup that only write the staged output out (the others run
// the MFMA steps); a schedule for W waves is built over W - kIoWaves compute waves.
constexpr int kIoWaves = 6;
// 16-byte register slots per I/O lane holding a staged tile (16 rows of up to 912 doubles)
constexpr int kIoSlots = 20;
// the same for tiles of 16 * mt cells: 32-cell tiles of up to 408 entries per cell, 64-cell
// tiles of up to 144 (fewer slots leave the registers that the extra MFMA row blocks need)
constexpr int persistent_io_slots(int mt) { return mt == 1 ? kIoSlots : mt == 2 ? 18 : 13; }
// Cell tiles of 16 * mt cells (mt = 1, 2 or 4; 2 and 4 with 16 waves and at most 16 steps).
// With a.coords set the kernel computes each tile's affine map from the coordinates
// (a.amap unused; 12 waves, mt = 1); else it reads the affine map from a.amap.
// Returns hipErrorInvalidValue when the form does not fit this kernel (caller falls back).
hipError_t launch_contract_persistent(int dim, int kind, int kmax, int waves, int mt, int grid, ContractArgs a,
                                      const PersistArgs& p, hipStream_t stream);
// Whether a form's tiles of 16 * mt cells fit the persistent FP64 kernel (output rows staged in
// LDS and in the I/O waves' registers), and its LDS plan.
bool persistent_fits(int dim, int kind, int n_I, int n_alpha, int mt, bool geo, size_t* stage_bytes,
                     size_t* head_bytes, size_t* total_bytes);
// Persistent split-BF16 contraction (same pipeline) on cell tiles of 16 or 32 cells:
// wave w of the 16 - kIoWaves compute waves owns A^0 tiles w, w + 10, ...; their B
// fragments (kpad / 32 chunks each) stay in registers.
// register steps per compute wave; LDS plan (staged = false when the form does not fit)
int bf16_persistent_steps(int n_tiles, int kpad);
int bf16_persistent_max_steps(int tile_cells, int n_seg);
LdsPlan plan_bf16_persistent(int dim, int kind, int tile_cells, int n_I, int n_tiles, int kpad, int n_seg);
// Returns hipErrorInvalidValue when the form or the output does not fit this kernel.
hipError_t launch_contract_bf16_persistent(int dim, int kind, int tile_cells, int grid, ContractArgs a,
                                           hipStream_t stream);
// Operator action of FP64 forms, y_K = A^K x_K per cell: the element tensors of a cell tile are
// built in LDS exactly as for tabulation and multiplied there by the cells' local vectors;
// only x and y (n_dof doubles per cell) cross HBM.  Tile kernel: returns hipErrorInvalidValue
// when the tile's rows cannot be staged; persistent kernel: same conditions as the persistent
// contraction, plus at most 16 register steps per wave and 16 * n_dof <= 2 * 64 * kIoWaves.
size_t apply_lds_bytes(int dim, int kind, int tile_cells, int n_I, int n_alpha, int n_dof);
hipError_t launch_apply(int dim, int kind, int tile_cells, int waves, ContractArgs a, hipStream_t stream);
// LDS of the persistent FP64 kernel's map / coefficient / coordinate rows (geo: the kernel
// computes the affine map), and the rows its compute waves fetch per tile
size_t persistent_head_bytes(int dim, int kind, bool geo, int tile_cells);
int persistent_fetch_rows(int dim, int kind, bool geo);
hipError_t launch_apply_persistent(int dim, int kind, int kmax, int waves, int grid, ContractArgs a,
                                   const PersistArgs& p, hipStream_t stream);
hipError_t launch_quadrature(int dim, int kind, const QuadArgs& a, hipStream_t stream);
size_t contract_lds_bytes(int dim, int kind, int tile_cells, int n_I, int n_alpha, int kpad, bool bf16);
int quad_cells_per_block(int dim, int kind, int ns, int npts);

// Mixed batches.  One descriptor per item (a mesh with its form); an item runs either in a
// tile launch (one workgroup per cell tile of 16*mt cells, geometry computed in place) or in
// the persistent launch of its form (FP64 forms with a persistent schedule; the 16-cell
// tiles of all its items form one sequence; affine map from a geometry pass into `amap`).
struct BatchItem {
    int64_t cells;
    int64_t unit_begin;     // first tile of this item in its launch's tile sequence
    const double* coords;   // SoA [(d+1)*d][cells]
    const double* coeffs;   // SoA [n_coeff][cells] or nullptr
    void* out;              // [cells][n_I]
    const double* amap;     // persistent items: SoA [1 + d*d][cells]
    int32_t dim, kind, n_I, n_alpha, n_tiles, kpad, n_seg, n_coeff;
    int32_t mt, staged;     // tile items: cell tile 16*mt, output rows staged in LDS
    int32_t sym_n, reserved2;  // FP64 symmetric forms: element dofs, else 0
    int32_t kmax, waves;    // persistent items: register steps per wave; FP64: waves per workgroup
                            // (12: the launch computes the affine maps, 16: read from amap)
    size_t stage_bytes, head_bytes;  // LDS plan: staged rows (0 = direct stores), map + coefficients
    const int32_t* koff;
    const uint32_t* apack;
    const int32_t* entry;
    const double* b;
    const uint16_t* bb;
    const uint8_t* nonzero;
    int32_t gpiece[6];
    PersistArgs p;
};

// Tile launch over items of one tile size (16*mt cells): grid = total tiles, unit_item[u] =
// item of tile u; nseg 0 = FP64, 3 / 6 = split BF16 with that many products; each item's LDS
// plan (stage_bytes, head_bytes, G) fits in `lds`.
hipError_t launch_batch_tiles(const BatchItem* items, const int32_t* unit_item, int64_t units, int waves, int mt,
                              int nseg, size_t lds, hipStream_t stream);
// Persistent launch over the items of one form (items in unit_begin order, `tiles` cell
// tiles in all): `grid` workgroups, workgroup w runs tiles w, w + grid, ...
// nseg 0: FP64 kernel (16-cell tiles, kmax register steps; 12 waves computing the affine
// maps from the coordinates, or 16 waves reading them from the items' amap); nseg 3 / 6:
// split-BF16 kernel (16 waves, 16*mt-cell tiles, kmax = its register steps, amap read).
hipError_t launch_batch_persistent(int dim, int kind, int kmax, int nseg, int mt, int waves, const BatchItem* items,
                                   int n_items, int64_t tiles, int grid, size_t lds, hipStream_t stream);

}  // namespace ffc
