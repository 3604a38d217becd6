// Persistent FP64 contraction (and operator action): kernels and launchers.
#include "kernels_device.h"

namespace ffc {

template <int D, int KIND, int KMAX, int MAXT, int IOS, bool ACT = false, bool GEO = false>
__global__ __launch_bounds__(MAXT) void contract_f64_persistent(ContractArgs A, PersistArgs P) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    OneMesh src{A};
    persistent_tiles<D, KIND, KMAX, IOS, ACT, GEO>(A, P, src, blockIdx.x, (A.cells + 15) / 16, gridDim.x, smem_raw);
}

// Workgroups of 12 waves (768 threads: 6 compute + 6 I/O waves) get ~168 registers per lane,
// 16 waves (1024 threads: 10 + 6) 128; the kernel computing its own affine maps needs the
// former (at 128 registers its geometry would spill).
template <int D, int KIND, bool ACT, bool GEO, int MAXT>
static hipError_t launch_persistent_kt(int kmax, int grid, size_t lds, const ContractArgs& a, const PersistArgs& p,
                                       hipStream_t s) {
    constexpr unsigned block = MAXT;
    if (kmax <= 8)
        return launch_lds(contract_f64_persistent<D, KIND, 8, MAXT, kIoSlots, ACT, GEO>, grid, block, lds, s, a, p);
    if (kmax <= 16)
        return launch_lds(contract_f64_persistent<D, KIND, 16, MAXT, kIoSlots, ACT, GEO>, grid, block, lds, s, a, p);
    // the operator action stops at 16 register steps (past them its registers spill)
    if constexpr (ACT) return hipErrorInvalidValue;
    else return launch_lds(contract_f64_persistent<D, KIND, 24, MAXT, kIoSlots, ACT, GEO>, grid, block, lds, s, a, p);
}

template <int D, int KIND, bool ACT, bool GEO>
static hipError_t launch_persistent_k(int kmax, int waves, int grid, size_t lds, const ContractArgs& a,
                                      const PersistArgs& p, hipStream_t s) {
    if (waves == 12) return launch_persistent_kt<D, KIND, ACT, GEO, 768>(kmax, grid, lds, a, p, s);
    if constexpr (GEO) return hipErrorInvalidValue;
    else return launch_persistent_kt<D, KIND, ACT, GEO, 1024>(kmax, grid, lds, a, p, s);
}

template <int D, bool ACT = false, bool GEO = false>
static hipError_t launch_persistent_d(int kind, int kmax, int waves, int grid, size_t lds, const ContractArgs& a,
                                      const PersistArgs& p, hipStream_t s) {
    switch (kind) {
    case K_MASS: return launch_persistent_k<D, K_MASS, ACT, GEO>(kmax, waves, grid, lds, a, p, s);
    case K_LAPLACE: return launch_persistent_k<D, K_LAPLACE, ACT, GEO>(kmax, waves, grid, lds, a, p, s);
    case K_WLAPLACE: return launch_persistent_k<D, K_WLAPLACE, ACT, GEO>(kmax, waves, grid, lds, a, p, s);
    case K_ELASTICITY: return launch_persistent_k<D, K_ELASTICITY, ACT, GEO>(kmax, waves, grid, lds, a, p, s);
    case K_PIOLA:
    case K_CURVED:
    case K_NEDELEC: return hipErrorInvalidValue;  // tile kernels only
    default: return launch_persistent_k<D, K_NS, ACT, GEO>(kmax, waves, grid, lds, a, p, s);
    }
}

size_t persistent_head_bytes(int dim, int kind, bool geo) {
    // map rows (two blocks when the kernel computes them), coefficients, coordinates; row
    // stride 17 doubles
    const int rows = geo ? 2 * (1 + dim * dim) + n_coeff_of(dim, kind) + (dim + 1) * dim
                         : 1 + dim * dim + n_coeff_of(dim, kind);
    return align16(static_cast<size_t>(rows) * 17 * sizeof(double));
}

int persistent_fetch_rows(int dim, int kind, bool geo) {
    return geo ? n_coeff_of(dim, kind) + (dim + 1) * dim : 1 + dim * dim + n_coeff_of(dim, kind);
}

hipError_t launch_contract_persistent(int dim, int kind, int kmax, int waves, int grid, ContractArgs a,
                                      const PersistArgs& p, hipStream_t stream) {
    if (a.cells <= 0) return hipSuccess;
    if (kmax > 24 || (waves != 16 && waves != 12) || (reinterpret_cast<uintptr_t>(a.out) & 15u) != 0)
        return hipErrorInvalidValue;
    // the staged rows of one tile must fit the I/O lanes' register slots, with lane 0's
    // last slot free for an odd tail
    const int64_t pairs = (16 * static_cast<int64_t>(a.n_I)) / 2;
    if (pairs > static_cast<int64_t>(kIoSlots) * 64 * kIoWaves - 64 * kIoWaves) return hipErrorInvalidValue;
    // coordinates given: the kernel computes the affine map itself (no geometry pass; 12 waves)
    const bool geo = a.coords != nullptr;
    if (geo && waves != 12) return hipErrorInvalidValue;
    const LdsPlan pl = plan_lds(dim, kind, 16, a.n_I, a.n_alpha, 0, false, kLdsBudget);
    const size_t head = persistent_head_bytes(dim, kind, geo);
    const size_t total = pl.stage_bytes + head + pl.g_bytes;
    if (!pl.staged || total > kLdsBudget || persistent_fetch_rows(dim, kind, geo) * 16 > 64 * (waves - kIoWaves))
        return hipErrorInvalidValue;
    a.staged = 1;
    a.stage_bytes = pl.stage_bytes;
    a.head_bytes = head;
    const int64_t ntiles = (a.cells + 15) / 16;
    if (grid > ntiles) grid = static_cast<int>(ntiles);
    if (geo)
        return dim == 2 ? launch_persistent_d<2, false, true>(kind, kmax, waves, grid, total, a, p, stream)
                        : launch_persistent_d<3, false, true>(kind, kmax, waves, grid, total, a, p, stream);
    return dim == 2 ? launch_persistent_d<2>(kind, kmax, waves, grid, total, a, p, stream)
                    : launch_persistent_d<3>(kind, kmax, waves, grid, total, a, p, stream);
}

hipError_t launch_apply_persistent(int dim, int kind, int kmax, int waves, int grid, ContractArgs a,
                                   const PersistArgs& p, hipStream_t stream) {
    if (a.cells <= 0) return hipSuccess;
    if (kmax > 16 || (waves != 16 && waves != 12) || !a.xloc || a.n_dof <= 0 || a.n_I != a.n_dof * a.n_dof ||
        16 * a.n_dof > 2 * 64 * kIoWaves)
        return hipErrorInvalidValue;
    const LdsPlan pl = plan_lds(dim, kind, 16, a.n_I, a.n_alpha, 0, false, kLdsBudget);
    const size_t lds = pl.total + 2 * 16 * static_cast<size_t>(a.n_dof) * sizeof(double);  // + two x buffers
    if (!pl.staged || lds > kLdsBudget || (1 + dim * dim + n_coeff_of(dim, kind)) * 16 > 64 * (waves - kIoWaves))
        return hipErrorInvalidValue;
    a.staged = 1;
    a.stage_bytes = pl.stage_bytes;
    a.head_bytes = pl.head_bytes;
    const int64_t ntiles = (a.cells + 15) / 16;
    if (grid > ntiles) grid = static_cast<int>(ntiles);
    return dim == 2 ? launch_persistent_d<2, true>(kind, kmax, waves, grid, lds, a, p, stream)
                    : launch_persistent_d<3, true>(kind, kmax, waves, grid, lds, a, p, stream);
}

}  // namespace ffc
