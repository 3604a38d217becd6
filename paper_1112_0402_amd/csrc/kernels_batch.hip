// Mixed batches: tile launches over many items, persistent launches per form.
#include "kernels_device.h"

namespace ffc {

template <int NSEG, int MT>
__global__ __launch_bounds__(1024) void batch_tiles_kernel(const BatchItem* __restrict__ items,
                                                           const int32_t* __restrict__ unit_item) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int64_t u = blockIdx.x;
    const BatchItem& it = items[__builtin_amdgcn_readfirstlane(unit_item[u])];
    const int64_t c0 = (u - it.unit_begin) * 16 * MT;
    switch (it.dim * 8 + it.kind) {
    case 16 + K_MASS: batch_tile<2, K_MASS, MT, NSEG>(it, c0, smem_raw); break;
    case 16 + K_LAPLACE: batch_tile<2, K_LAPLACE, MT, NSEG>(it, c0, smem_raw); break;
    case 16 + K_WLAPLACE: batch_tile<2, K_WLAPLACE, MT, NSEG>(it, c0, smem_raw); break;
    case 16 + K_ELASTICITY: batch_tile<2, K_ELASTICITY, MT, NSEG>(it, c0, smem_raw); break;
    case 16 + K_NS: batch_tile<2, K_NS, MT, NSEG>(it, c0, smem_raw); break;
    case 24 + K_MASS: batch_tile<3, K_MASS, MT, NSEG>(it, c0, smem_raw); break;
    case 24 + K_LAPLACE: batch_tile<3, K_LAPLACE, MT, NSEG>(it, c0, smem_raw); break;
    case 24 + K_WLAPLACE: batch_tile<3, K_WLAPLACE, MT, NSEG>(it, c0, smem_raw); break;
    case 24 + K_ELASTICITY: batch_tile<3, K_ELASTICITY, MT, NSEG>(it, c0, smem_raw); break;
    default: batch_tile<3, K_NS, MT, NSEG>(it, c0, smem_raw); break;
    }
}

template <int NSEG>
static hipError_t launch_batch_tiles_n(int mt, unsigned grid, unsigned block, size_t lds, hipStream_t s,
                                       const BatchItem* items, const int32_t* unit_item) {
    switch (mt) {
    case 1: return launch_lds(batch_tiles_kernel<NSEG, 1>, grid, block, lds, s, items, unit_item);
    case 2: return launch_lds(batch_tiles_kernel<NSEG, 2>, grid, block, lds, s, items, unit_item);
    default: return launch_lds(batch_tiles_kernel<NSEG, 4>, grid, block, lds, s, items, unit_item);
    }
}

hipError_t launch_batch_tiles(const BatchItem* items, const int32_t* unit_item, int64_t units, int waves, int mt,
                              int nseg, size_t lds, hipStream_t stream) {
    if (units <= 0) return hipSuccess;
    const unsigned grid = static_cast<unsigned>(units);
    const unsigned block = 64u * waves;
    if (nseg == 3) return launch_batch_tiles_n<3>(mt, grid, block, lds, stream, items, unit_item);
    if (nseg == 6) return launch_batch_tiles_n<6>(mt, grid, block, lds, stream, items, unit_item);
    return launch_batch_tiles_n<0>(mt, grid, block, lds, stream, items, unit_item);
}

// Persistent launch over the items of one form: the 16-cell tiles of all items form one
// sequence, and workgroup w runs tiles w, w + grid, ... of it with the persistent tile loop
// above (A^0 fragments loaded once, the pipeline never drained between items; every tile
// costs the same, so the static split is balanced to one tile).

template <int D, int KIND, int KMAX, int MAXT, bool GEO, int MT>
__global__ __launch_bounds__(MAXT) void batch_persistent_kernel(const BatchItem* __restrict__ items, int n_items,
                                                                int64_t total_tiles) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    // every item of the launch has the same form: tables and LDS plan from the first
    const BatchItem& f = items[0];
    ContractArgs A{};
    A.n_I = f.n_I;
    A.b = as_global(f.b);
    A.apack = as_global(f.apack);
    A.entry = as_global(f.entry);
    A.stage_bytes = f.stage_bytes;
    A.head_bytes = f.head_bytes;
    const PersistArgs P{as_global(f.p.woff), as_global(f.p.wave_b), as_global(f.p.wave_word),
                        as_global(f.p.wave_mask), as_global(f.p.zero_entries), f.p.n_zero};
    ItemCursor<16 * MT> src{items, n_items, -1, 0, 0, MeshTile{}};
    // GEO: the affine map of each tile is computed in the kernel from the items' coordinates
    persistent_tiles<D, KIND, KMAX, persistent_io_slots(MT), false, GEO, MT>(A, P, src, blockIdx.x, total_tiles,
                                                                            gridDim.x, smem_raw);
}

template <int D, int KIND, int NSEG, int KS, int MT>
__global__ __launch_bounds__(1024) void batch_persistent_bf16_kernel(const BatchItem* __restrict__ items, int n_items,
                                                                     int64_t total_tiles) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const BatchItem& f = items[0];  // every item of the launch has the same form
    ContractArgs A{};
    A.n_I = f.n_I;
    A.n_tiles = f.n_tiles;
    A.kpad = f.kpad;
    A.n_seg = f.n_seg;
    for (int i = 0; i < 6; ++i) A.gpiece[i] = f.gpiece[i];
    A.bb = as_global(f.bb);
    A.stage_bytes = f.stage_bytes;
    A.head_bytes = f.head_bytes;
    ItemCursor<16 * MT> src{items, n_items, -1, 0, 0, MeshTile{}};
    persistent_tiles_bf16<D, KIND, NSEG, KS, MT>(A, src, blockIdx.x, total_tiles, gridDim.x, smem_raw);
}

template <int D, int KIND, int NSEG, int MT>
static hipError_t launch_batch_bf16_m(int ks, const BatchItem* items, int n_items, int64_t tiles, int grid, size_t lds,
                                      hipStream_t s) {
    if (ks <= 8)
        return launch_lds(batch_persistent_bf16_kernel<D, KIND, NSEG, 8, MT>, grid, 1024u, lds, s, items, n_items,
                          tiles);
    return launch_lds(batch_persistent_bf16_kernel<D, KIND, NSEG, 16, MT>, grid, 1024u, lds, s, items, n_items,
                      tiles);
}

template <int D, int NSEG>
static hipError_t launch_batch_bf16_d(int kind, int mt, int ks, const BatchItem* items, int n_items, int64_t tiles,
                                      int grid, size_t lds, hipStream_t s) {
#define FFC_BATCH_BF16_KIND(K)                                                                \
    return mt == 1   ? launch_batch_bf16_m<D, K, NSEG, 1>(ks, items, n_items, tiles, grid, lds, s) \
           : mt == 2 ? launch_batch_bf16_m<D, K, NSEG, 2>(ks, items, n_items, tiles, grid, lds, s) \
                     : launch_batch_bf16_m<D, K, NSEG, 4>(ks, items, n_items, tiles, grid, lds, s)
    switch (kind) {
    case K_MASS: FFC_BATCH_BF16_KIND(K_MASS);
    case K_LAPLACE: FFC_BATCH_BF16_KIND(K_LAPLACE);
    case K_WLAPLACE: FFC_BATCH_BF16_KIND(K_WLAPLACE);
    case K_ELASTICITY: FFC_BATCH_BF16_KIND(K_ELASTICITY);
    default: FFC_BATCH_BF16_KIND(K_NS);
    }
#undef FFC_BATCH_BF16_KIND
}

template <int D, int KIND, int MAXT, bool GEO>
static hipError_t launch_batch_persistent_kt(int kmax, int mt, const BatchItem* items, int n_items, int64_t tiles,
                                             int grid, size_t lds, hipStream_t s) {
    if (mt == 2 || mt == 4) {  // 12 waves, 32- or 64-cell tiles
        if constexpr (MAXT != 768) {
            return hipErrorInvalidValue;
        } else if (mt == 2) {
            if (kmax <= 8)
                return launch_lds(batch_persistent_kernel<D, KIND, 8, MAXT, GEO, 2>, grid, MAXT, lds, s, items, n_items,
                                  tiles);
            if (kmax <= 16)
                return launch_lds(batch_persistent_kernel<D, KIND, 16, MAXT, GEO, 2>, grid, MAXT, lds, s, items, n_items,
                                  tiles);
            return hipErrorInvalidValue;
        } else {
            if (kmax <= 8)
                return launch_lds(batch_persistent_kernel<D, KIND, 8, MAXT, GEO, 4>, grid, MAXT, lds, s, items, n_items,
                                  tiles);
            if (kmax <= 16)
                return launch_lds(batch_persistent_kernel<D, KIND, 16, MAXT, GEO, 4>, grid, MAXT, lds, s, items, n_items,
                                  tiles);
            return hipErrorInvalidValue;
        }
    }
    if (kmax <= 8)
        return launch_lds(batch_persistent_kernel<D, KIND, 8, MAXT, GEO, 1>, grid, MAXT, lds, s, items, n_items, tiles);
    if (kmax <= 16)
        return launch_lds(batch_persistent_kernel<D, KIND, 16, MAXT, GEO, 1>, grid, MAXT, lds, s, items, n_items, tiles);
    return launch_lds(batch_persistent_kernel<D, KIND, 24, MAXT, GEO, 1>, grid, MAXT, lds, s, items, n_items, tiles);
}

template <int D, int KIND>
static hipError_t launch_batch_persistent_k(int kmax, int waves, int mt, const BatchItem* items, int n_items,
                                            int64_t tiles, int grid, size_t lds, hipStream_t s) {
    // 12 waves: the launch computes its affine maps (the register budget of the geometry);
    // 16 waves: it reads the maps of the batch's geometry passes
    return waves == 12
               ? launch_batch_persistent_kt<D, KIND, 768, true>(kmax, mt, items, n_items, tiles, grid, lds, s)
               : launch_batch_persistent_kt<D, KIND, 1024, false>(kmax, mt, items, n_items, tiles, grid, lds, s);
}

template <int D>
static hipError_t launch_batch_persistent_d(int kind, int kmax, int waves, int mt, const BatchItem* items, int n_items,
                                            int64_t tiles, int grid, size_t lds, hipStream_t s) {
#define FFC_BATCH_P(K) return launch_batch_persistent_k<D, K>(kmax, waves, mt, items, n_items, tiles, grid, lds, s)
    switch (kind) {
    case K_MASS: FFC_BATCH_P(K_MASS);
    case K_LAPLACE: FFC_BATCH_P(K_LAPLACE);
    case K_WLAPLACE: FFC_BATCH_P(K_WLAPLACE);
    case K_ELASTICITY: FFC_BATCH_P(K_ELASTICITY);
    default: FFC_BATCH_P(K_NS);
    }
#undef FFC_BATCH_P
}

hipError_t launch_batch_persistent(int dim, int kind, int kmax, int nseg, int mt, int waves, const BatchItem* items,
                                   int n_items, int64_t tiles, int grid, size_t lds, hipStream_t stream) {
    if (tiles <= 0 || n_items <= 0) return hipSuccess;
    if (grid > tiles) grid = static_cast<int>(tiles);
    if (nseg == 3)
        return dim == 2 ? launch_batch_bf16_d<2, 3>(kind, mt, kmax, items, n_items, tiles, grid, lds, stream)
                        : launch_batch_bf16_d<3, 3>(kind, mt, kmax, items, n_items, tiles, grid, lds, stream);
    if (nseg == 6)
        return dim == 2 ? launch_batch_bf16_d<2, 6>(kind, mt, kmax, items, n_items, tiles, grid, lds, stream)
                        : launch_batch_bf16_d<3, 6>(kind, mt, kmax, items, n_items, tiles, grid, lds, stream);
    if (waves != 12 && waves != 16) return hipErrorInvalidValue;
    return dim == 2 ? launch_batch_persistent_d<2>(kind, kmax, waves, mt, items, n_items, tiles, grid, lds, stream)
                    : launch_batch_persistent_d<3>(kind, kmax, waves, mt, items, n_items, tiles, grid, lds, stream);
}

}  // namespace ffc
