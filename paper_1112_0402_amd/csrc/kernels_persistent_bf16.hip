// Persistent split-BF16 contraction: kernels and launchers.
#include "kernels_device.h"

namespace ffc {

template <int D, int KIND, int NSEG, int KS, int MT>
__global__ __launch_bounds__(1024) void contract_bf16_persistent(ContractArgs A) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    OneMesh src{A};
    persistent_tiles_bf16<D, KIND, NSEG, KS, MT>(A, src, blockIdx.x, (A.cells + 16 * MT - 1) / (16 * MT), gridDim.x,
                                                smem_raw);
}

// Register budget (128 per lane at 1024 threads): at most 16 register-resident steps.
int bf16_persistent_max_steps(int tile_cells, int n_seg) {
    (void)tile_cells;
    (void)n_seg;
    return 16;
}

template <int D, int KIND, int NSEG, int MT>
static hipError_t launch_bf16_persistent_m(int ks, int grid, size_t lds, const ContractArgs& a, hipStream_t s) {
    if (ks <= 8) return launch_lds(contract_bf16_persistent<D, KIND, NSEG, 8, MT>, grid, 1024u, lds, s, a);
    return launch_lds(contract_bf16_persistent<D, KIND, NSEG, 16, MT>, grid, 1024u, lds, s, a);
}

template <int D, int KIND, int NSEG>
static hipError_t launch_bf16_persistent_k(int mt, int ks, int grid, size_t lds, const ContractArgs& a,
                                           hipStream_t s) {
    return mt == 1   ? launch_bf16_persistent_m<D, KIND, NSEG, 1>(ks, grid, lds, a, s)
           : mt == 2 ? launch_bf16_persistent_m<D, KIND, NSEG, 2>(ks, grid, lds, a, s)
                     : launch_bf16_persistent_m<D, KIND, NSEG, 4>(ks, grid, lds, a, s);
}

template <int D, int NSEG>
static hipError_t launch_bf16_persistent_d(int kind, int mt, int ks, int grid, size_t lds, const ContractArgs& a,
                                           hipStream_t s) {
    switch (kind) {
    case K_MASS: return launch_bf16_persistent_k<D, K_MASS, NSEG>(mt, ks, grid, lds, a, s);
    case K_LAPLACE: return launch_bf16_persistent_k<D, K_LAPLACE, NSEG>(mt, ks, grid, lds, a, s);
    case K_WLAPLACE: return launch_bf16_persistent_k<D, K_WLAPLACE, NSEG>(mt, ks, grid, lds, a, s);
    case K_ELASTICITY: return launch_bf16_persistent_k<D, K_ELASTICITY, NSEG>(mt, ks, grid, lds, a, s);
    case K_PIOLA:
    case K_CURVED:
    case K_NEDELEC: return hipErrorInvalidValue;
    default: return launch_bf16_persistent_k<D, K_NS, NSEG>(mt, ks, grid, lds, a, s);
    }
}

int bf16_persistent_steps(int n_tiles, int kpad) {
    const int n_compute = 16 - kIoWaves;
    return (n_tiles + n_compute - 1) / n_compute * (kpad / 32);
}

LdsPlan plan_bf16_persistent(int dim, int kind, int tile_cells, int n_I, int n_tiles, int kpad, int n_seg) {
    LdsPlan p = plan_lds(dim, kind, tile_cells, n_I, 0, kpad, true, kLdsBudget);
    const int ios = tile_cells == 16   ? Bf16PersistTraits<1>::ios
                    : tile_cells == 32 ? Bf16PersistTraits<2>::ios
                                       : Bf16PersistTraits<4>::ios;
    const int64_t units = (tile_cells * static_cast<int64_t>(n_I) + 3) / 4;
    const bool fits = (tile_cells == 16 || tile_cells == 32 || tile_cells == 64) && p.staged &&
                      bf16_persistent_steps(n_tiles, kpad) <= bf16_persistent_max_steps(tile_cells, n_seg) &&
                      units <= static_cast<int64_t>(ios) * 64 * kIoWaves &&
                      (1 + dim * dim + n_coeff_of(dim, kind)) * tile_cells <= 1024;
    if (!fits) p.staged = false;
    return p;
}

hipError_t launch_contract_bf16_persistent(int dim, int kind, int tile_cells, int grid, ContractArgs a,
                                           hipStream_t stream) {
    if (a.cells <= 0) return hipSuccess;
    if ((reinterpret_cast<uintptr_t>(a.out) & 15u) != 0) return hipErrorInvalidValue;
    const LdsPlan pl = plan_bf16_persistent(dim, kind, tile_cells, a.n_I, a.n_tiles, a.kpad, a.n_seg);
    if (!pl.staged) return hipErrorInvalidValue;
    a.staged = 1;
    a.stage_bytes = pl.stage_bytes;
    a.head_bytes = pl.head_bytes;
    const int ks = bf16_persistent_steps(a.n_tiles, a.kpad);
    const int mt = tile_cells / 16;
    const int64_t ntiles = (a.cells + tile_cells - 1) / tile_cells;
    if (grid > ntiles) grid = static_cast<int>(ntiles);
    if (a.n_seg == 3)
        return dim == 2 ? launch_bf16_persistent_d<2, 3>(kind, mt, ks, grid, pl.total, a, stream)
                        : launch_bf16_persistent_d<3, 3>(kind, mt, ks, grid, pl.total, a, stream);
    return dim == 2 ? launch_bf16_persistent_d<2, 6>(kind, mt, ks, grid, pl.total, a, stream)
                    : launch_bf16_persistent_d<3, 6>(kind, mt, ks, grid, pl.total, a, stream);
}

}  // namespace ffc
