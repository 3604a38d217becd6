// Persistent FP64 contraction (and operator action): kernels and launchers.
#include "kernels_device.h"

namespace ffc {

template <int D, int KIND, int KMAX, int MAXT, int IOS, bool ACT = false, bool GEO = false, int MT = 1>
__global__ __launch_bounds__(MAXT) void contract_f64_persistent(ContractArgs A, PersistArgs P) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    OneMesh src{A};
    persistent_tiles<D, KIND, KMAX, IOS, ACT, GEO, MT>(A, P, src, blockIdx.x, (A.cells + 16 * MT - 1) / (16 * MT),
                                                       gridDim.x, smem_raw);
}

// Workgroups of 12 waves (768 threads: 6 compute + 6 I/O waves) get ~168 registers per lane,
// 16 waves (1024 threads: 10 + 6) 128; the kernel computing its own affine maps needs the
// former (at 128 registers its geometry would spill), and so do tiles of 32 and 64 cells
// (MT = 2, 4: more accumulators and row-block operands), instantiated for 12 waves with up to
// 16 register steps.
template <int D, int KIND, bool ACT, bool GEO, int MAXT>
static hipError_t launch_persistent_kt(int kmax, int mt, int grid, size_t lds, const ContractArgs& a,
                                       const PersistArgs& p, hipStream_t s) {
    constexpr unsigned block = MAXT;
    if (mt == 2 || mt == 4) {
        if constexpr (ACT || MAXT != 768) {
            return hipErrorInvalidValue;
        } else if (mt == 2) {
            if (kmax <= 8)
                return launch_lds(contract_f64_persistent<D, KIND, 8, MAXT, persistent_io_slots(2), false, GEO, 2>,
                                  grid, block, lds, s, a, p);
            if (kmax <= 16)
                return launch_lds(contract_f64_persistent<D, KIND, 16, MAXT, persistent_io_slots(2), false, GEO, 2>,
                                  grid, block, lds, s, a, p);
            return hipErrorInvalidValue;
        } else {
            if (kmax <= 8)
                return launch_lds(contract_f64_persistent<D, KIND, 8, MAXT, persistent_io_slots(4), false, GEO, 4>,
                                  grid, block, lds, s, a, p);
            if (kmax <= 16)
                return launch_lds(contract_f64_persistent<D, KIND, 16, MAXT, persistent_io_slots(4), false, GEO, 4>,
                                  grid, block, lds, s, a, p);
            return hipErrorInvalidValue;
        }
    }
    if (mt != 1) return hipErrorInvalidValue;
    if (kmax <= 8)
        return launch_lds(contract_f64_persistent<D, KIND, 8, MAXT, kIoSlots, ACT, GEO>, grid, block, lds, s, a, p);
    if (kmax <= 16)
        return launch_lds(contract_f64_persistent<D, KIND, 16, MAXT, kIoSlots, ACT, GEO>, grid, block, lds, s, a, p);
    // the operator action stops at 16 register steps (past them its registers spill)
    if constexpr (ACT) return hipErrorInvalidValue;
    else return launch_lds(contract_f64_persistent<D, KIND, 24, MAXT, kIoSlots, ACT, GEO>, grid, block, lds, s, a, p);
}

template <int D, int KIND, bool ACT, bool GEO>
static hipError_t launch_persistent_k(int kmax, int waves, int mt, int grid, size_t lds, const ContractArgs& a,
                                      const PersistArgs& p, hipStream_t s) {
    if (waves == 12) return launch_persistent_kt<D, KIND, ACT, GEO, 768>(kmax, mt, grid, lds, a, p, s);
    if constexpr (GEO) return hipErrorInvalidValue;
    else return launch_persistent_kt<D, KIND, ACT, GEO, 1024>(kmax, mt, grid, lds, a, p, s);
}

template <int D, bool ACT = false, bool GEO = false>
static hipError_t launch_persistent_d(int kind, int kmax, int waves, int mt, int grid, size_t lds,
                                      const ContractArgs& a, const PersistArgs& p, hipStream_t s) {
    switch (kind) {
    case K_MASS: return launch_persistent_k<D, K_MASS, ACT, GEO>(kmax, waves, mt, grid, lds, a, p, s);
    case K_LAPLACE: return launch_persistent_k<D, K_LAPLACE, ACT, GEO>(kmax, waves, mt, grid, lds, a, p, s);
    case K_WLAPLACE: return launch_persistent_k<D, K_WLAPLACE, ACT, GEO>(kmax, waves, mt, grid, lds, a, p, s);
    case K_ELASTICITY: return launch_persistent_k<D, K_ELASTICITY, ACT, GEO>(kmax, waves, mt, grid, lds, a, p, s);
    case K_PIOLA:
    case K_CURVED:
    case K_NEDELEC: return hipErrorInvalidValue;  // tile kernels only
    default: return launch_persistent_k<D, K_NS, ACT, GEO>(kmax, waves, mt, grid, lds, a, p, s);
    }
}

size_t persistent_head_bytes(int dim, int kind, bool geo, int tile_cells) {
    // map rows (two blocks when the kernel computes them), coefficients, coordinates; row
    // stride tile_cells + 1 doubles
    const int rows = geo ? 2 * (1 + dim * dim) + n_coeff_of(dim, kind) + (dim + 1) * dim
                         : 1 + dim * dim + n_coeff_of(dim, kind);
    return align16(static_cast<size_t>(rows) * (tile_cells + 1) * sizeof(double));
}

bool persistent_fits(int dim, int kind, int n_I, int n_alpha, int mt, bool geo, size_t* stage, size_t* head,
                     size_t* total) {
    if (mt != 1 && mt != 2 && mt != 4) return false;
    const int ct = 16 * mt;
    // the staged rows of one tile must fit the I/O lanes' register slots, with lane 0's last
    // slot free for an odd tail
    const int64_t pairs = (ct * static_cast<int64_t>(n_I)) / 2;
    if (pairs > static_cast<int64_t>(persistent_io_slots(mt)) * 64 * kIoWaves - 64 * kIoWaves) return false;
    const LdsPlan pl = plan_lds(dim, kind, ct, n_I, n_alpha, 0, false, kLdsBudget);
    const size_t h = persistent_head_bytes(dim, kind, geo, ct);
    const size_t t = pl.stage_bytes + h + pl.g_bytes;
    if (!pl.staged || t > kLdsBudget) return false;
    if (stage) *stage = pl.stage_bytes;
    if (head) *head = h;
    if (total) *total = t;
    return true;
}

int persistent_fetch_rows(int dim, int kind, bool geo) {
    return geo ? n_coeff_of(dim, kind) + (dim + 1) * dim : 1 + dim * dim + n_coeff_of(dim, kind);
}

hipError_t launch_contract_persistent(int dim, int kind, int kmax, int waves, int mt, int grid, ContractArgs a,
                                      const PersistArgs& p, hipStream_t stream) {
    if (a.cells <= 0) return hipSuccess;
    if (kmax > 24 || (waves != 16 && waves != 12) || (reinterpret_cast<uintptr_t>(a.out) & 15u) != 0)
        return hipErrorInvalidValue;
    // coordinates given: the kernel computes the affine map itself (no geometry pass); that
    // and tiles of 32 or 64 cells take 12 waves
    const bool geo = a.coords != nullptr;
    if ((geo || mt != 1) && waves != 12) return hipErrorInvalidValue;
    size_t stage = 0, head = 0, total = 0;
    if (!persistent_fits(dim, kind, a.n_I, a.n_alpha, mt, geo, &stage, &head, &total)) return hipErrorInvalidValue;
    a.staged = 1;
    a.stage_bytes = stage;
    a.head_bytes = head;
    const int64_t ntiles = (a.cells + 16 * mt - 1) / (16 * mt);
    if (grid > ntiles) grid = static_cast<int>(ntiles);
    if (geo)
        return dim == 2 ? launch_persistent_d<2, false, true>(kind, kmax, waves, mt, grid, total, a, p, stream)
                        : launch_persistent_d<3, false, true>(kind, kmax, waves, mt, grid, total, a, p, stream);
    return dim == 2 ? launch_persistent_d<2>(kind, kmax, waves, mt, grid, total, a, p, stream)
                    : launch_persistent_d<3>(kind, kmax, waves, mt, grid, total, a, p, stream);
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
    return dim == 2 ? launch_persistent_d<2, true>(kind, kmax, waves, 1, grid, lds, a, p, stream)
                    : launch_persistent_d<3, true>(kind, kmax, waves, 1, grid, lds, a, p, stream);
}

}  // namespace ffc
