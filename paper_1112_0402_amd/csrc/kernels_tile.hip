// One workgroup per cell tile: the LDS plan, the FP64 and split-BF16 tile contractions, the
// operator action of a tile.
#include "kernels_device.h"

namespace ffc {

LdsPlan plan_lds(int dim, int kind, int tile_cells, int n_I, int n_alpha, int kpad, bool bf16, size_t budget) {
    LdsPlan p{};
    const size_t ob = bf16 ? sizeof(float) : sizeof(double);
    p.stage_bytes = align16(static_cast<size_t>(tile_cells) * n_I * ob);
    // head rows: affine map and coefficients, or (curvilinear cells) the P2 node coordinates
    const int rows = kind == K_CURVED ? (dim == 2 ? 12 : 30) : 1 + dim * dim + n_coeff_of(dim, kind);
    // (tile_cells + 1 per row: the persistent kernels pad the row stride)
    const size_t head = align16(static_cast<size_t>(rows) * (tile_cells + 1) * sizeof(double));
    const size_t g = bf16 ? static_cast<size_t>(tile_cells) * (kpad + 8) * sizeof(uint16_t)
                          : static_cast<size_t>(tile_cells) * (n_alpha | 1) * sizeof(double);
    p.head_bytes = head;
    p.g_bytes = align16(g);
    p.staged = p.stage_bytes + head + p.g_bytes <= budget;
    if (!p.staged) p.stage_bytes = 0;
    p.total = p.stage_bytes + head + p.g_bytes;
    return p;
}

size_t contract_lds_bytes(int dim, int kind, int tile_cells, int n_I, int n_alpha, int kpad, bool bf16) {
    return plan_lds(dim, kind, tile_cells, n_I, n_alpha, kpad, bf16, kLdsBudget).total;
}

// Flat copy of n staged values to global memory (out 16-byte aligned) with 16-byte stores.
template <int D, int KIND, int MT>
__global__ __launch_bounds__(1024) void contract_f64_kernel(ContractArgs A) {
    using FT = FormTraits<KIND, D>;
    constexpr int CT = 16 * MT;
    constexpr int NC = FT::n_coeff;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    double* st = A.staged ? reinterpret_cast<double*>(smem_raw) : nullptr;
    double* am = reinterpret_cast<double*>(smem_raw + A.stage_bytes);
    double* cf = am + (1 + D * D) * CT;
    double* Gs = reinterpret_cast<double*>(smem_raw + A.stage_bytes + A.head_bytes);
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * CT;
    if constexpr (KIND != K_CURVED) {
        if (A.coords)
            stage_tile_from_coords<D, NC>(A.coords, A.coeffs, A.cells, c0, CT, am, cf);
        else
            stage_tile<D, NC>(A, c0, CT, am, cf);
        __syncthreads();
    } else if (A.coords) {
        // curvilinear cells, G built in the tile: the P2 nodes to LDS ([k*D + j][CT]), then
        // one lane per (point, cell): J(X_p) = sum_k x_k (grad Psi_k(X_p))^T, det J, g = J^{-1},
        // G[(p, a <= b)] = |det J| (g g^T)_ab
        constexpr int NG = D == 2 ? 6 : 10;
        constexpr int NP = D * (D + 1) / 2;
        for (int i = threadIdx.x; i < NG * D * CT; i += blockDim.x) {
            const int r = i / CT, c = i - (i / CT) * CT;
            const int64_t cell = c0 + c;
            am[i] = cell < A.cells ? A.coords[r * A.cells + cell] : 0.0;
        }
        __syncthreads();
        const int GS = A.n_alpha | 1;
        for (int i = threadIdx.x; i < CT * A.n_pts; i += blockDim.x) {
            const int p = i / CT, c = i - (i / CT) * CT;
            double* gr = Gs + c * GS + p * NP;
            if (c0 + c >= A.cells) {
#pragma unroll
                for (int q = 0; q < NP; ++q) gr[q] = 0.0;
                continue;
            }
            double J[D][D];
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int b = 0; b < D; ++b) J[j][b] = 0.0;
#pragma unroll
            for (int k = 0; k < NG; ++k)
#pragma unroll
                for (int b = 0; b < D; ++b) {
                    const double gk = A.geo_grad[(p * NG + k) * D + b];
#pragma unroll
                    for (int j = 0; j < D; ++j) J[j][b] = fma(am[(k * D + j) * CT + c], gk, J[j][b]);
                }
            double det, g[D][D];
            invert_jacobian<D>(J, det, g);
            const double adet = fabs(det);
            int pr = 0;
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = a; b < D; ++b, ++pr) {
                    double s = 0.0;
#pragma unroll
                    for (int k = 0; k < D; ++k) s += g[a][k] * g[b][k];
                    gr[pr] = adet * s;
                }
        }
    }
    contract_tile_f64<D, KIND, MT>(am, cf, Gs, st, c0, A.cells, A.n_I, A.n_tiles, A.koff, A.apack, A.entry, A.b,
                                   static_cast<double*>(A.out), A.sym_n, A.n_alpha,
                                   KIND == K_CURVED && A.coords ? nullptr : A.amap, A.astride);
}

// Operator action, one cell tile per workgroup: the tile's local vectors go to LDS beside
// the G tile, the element tensors to the staged rows, then thread (c, i1) forms
// y[c][i1] = sum_i2 A^K[c][i1][i2] x[c][i2] and the tile's y rows leave as one contiguous run.
template <int D, int KIND, int MT>
__global__ __launch_bounds__(1024) void apply_f64_kernel(ContractArgs A) {
    using FT = FormTraits<KIND, D>;
    constexpr int CT = 16 * MT;
    constexpr int NC = FT::n_coeff;
    constexpr int GS = FT::n_alpha | 1;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    double* st = reinterpret_cast<double*>(smem_raw);
    double* am = reinterpret_cast<double*>(smem_raw + A.stage_bytes);
    double* cf = am + (1 + D * D) * CT;
    double* Gs = reinterpret_cast<double*>(smem_raw + A.stage_bytes + A.head_bytes);
    double* xs = Gs + CT * GS;
    const int n = A.n_dof, nI = A.n_I;
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * CT;
    const int64_t nc = A.cells - c0 < CT ? A.cells - c0 : CT;
    const double* xg = A.xloc + c0 * n;
    for (int i = threadIdx.x; i < CT * n; i += blockDim.x) xs[i] = i < nc * n ? xg[i] : 0.0;
    if (A.coords)
        stage_tile_from_coords<D, NC>(A.coords, A.coeffs, A.cells, c0, CT, am, cf);
    else
        stage_tile<D, NC>(A, c0, CT, am, cf);
    __syncthreads();
    contract_tile_f64<D, KIND, MT>(am, cf, Gs, st, c0, A.cells, nI, A.n_tiles, A.koff, A.apack, A.entry, A.b,
                                   nullptr, A.sym_n);
    __syncthreads();
    double* y = static_cast<double*>(A.out) + c0 * n;
    for (int t = threadIdx.x; t < nc * n; t += blockDim.x) {
        const int c = t / n, i1 = t - c * n;
        const double* row = st + c * nI + i1 * n;
        const double* xc = xs + c * n;
        double s = 0.0;
        for (int i2 = 0; i2 < n; ++i2) s = fma(row[i2], xc[i2], s);
        y[t] = s;
    }
}

template <int D, int KIND>
static hipError_t launch_f64_mt(int tile_cells, int waves, size_t lds, const ContractArgs& a, hipStream_t s) {
    const unsigned grid = static_cast<unsigned>((a.cells + tile_cells - 1) / tile_cells);
    const unsigned block = 64u * waves;
    switch (tile_cells) {
    case 16: return launch_lds(contract_f64_kernel<D, KIND, 1>, grid, block, lds, s, a);
    case 32: return launch_lds(contract_f64_kernel<D, KIND, 2>, grid, block, lds, s, a);
    default: return launch_lds(contract_f64_kernel<D, KIND, 4>, grid, block, lds, s, a);
    }
}

template <int D>
static hipError_t launch_f64_d(int kind, int tile_cells, int waves, size_t lds, const ContractArgs& a, hipStream_t s) {
    switch (kind) {
    case K_MASS: return launch_f64_mt<D, K_MASS>(tile_cells, waves, lds, a, s);
    case K_LAPLACE: return launch_f64_mt<D, K_LAPLACE>(tile_cells, waves, lds, a, s);
    case K_WLAPLACE: return launch_f64_mt<D, K_WLAPLACE>(tile_cells, waves, lds, a, s);
    case K_ELASTICITY: return launch_f64_mt<D, K_ELASTICITY>(tile_cells, waves, lds, a, s);
    case K_PIOLA: return launch_f64_mt<D, K_PIOLA>(tile_cells, waves, lds, a, s);
    case K_CURVED: return launch_f64_mt<D, K_CURVED>(tile_cells, waves, lds, a, s);
    case K_NEDELEC: return launch_f64_mt<D, K_NEDELEC>(tile_cells, waves, lds, a, s);
    default: return launch_f64_mt<D, K_NS>(tile_cells, waves, lds, a, s);
    }
}

template <int D, int KIND, int MT, int NSEG>
__global__ __launch_bounds__(1024) void contract_bf16_kernel(ContractArgs A) {
    using FT = FormTraits<KIND, D>;
    constexpr int CT = 16 * MT;
    constexpr int NC = FT::n_coeff;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    float* st = A.staged ? reinterpret_cast<float*>(smem_raw) : nullptr;
    double* am = reinterpret_cast<double*>(smem_raw + A.stage_bytes);
    double* cf = am + (1 + D * D) * CT;
    unsigned short* Gp = reinterpret_cast<unsigned short*>(smem_raw + A.stage_bytes + A.head_bytes);
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * CT;
    if (A.coords)
        stage_tile_from_coords<D, NC>(A.coords, A.coeffs, A.cells, c0, CT, am, cf);
    else
        stage_tile<D, NC>(A, c0, CT, am, cf);
    __syncthreads();
    contract_tile_bf16<D, KIND, MT, NSEG>(am, cf, Gp, st, c0, A.cells, A.n_I, A.n_tiles, A.kpad, A.gpiece, A.bb,
                                          A.nonzero, static_cast<float*>(A.out));
}

template <int D, int KIND, int NSEG>
static hipError_t launch_bf16_mt(int tile_cells, int waves, size_t lds, const ContractArgs& a, hipStream_t s) {
    const unsigned grid = static_cast<unsigned>((a.cells + tile_cells - 1) / tile_cells);
    const unsigned block = 64u * waves;
    switch (tile_cells) {
    case 16: return launch_lds(contract_bf16_kernel<D, KIND, 1, NSEG>, grid, block, lds, s, a);
    case 32: return launch_lds(contract_bf16_kernel<D, KIND, 2, NSEG>, grid, block, lds, s, a);
    default: return launch_lds(contract_bf16_kernel<D, KIND, 4, NSEG>, grid, block, lds, s, a);
    }
}

template <int D, int NSEG>
static hipError_t launch_bf16_d(int kind, int tile_cells, int waves, size_t lds, const ContractArgs& a, hipStream_t s) {
    switch (kind) {
    case K_MASS: return launch_bf16_mt<D, K_MASS, NSEG>(tile_cells, waves, lds, a, s);
    case K_LAPLACE: return launch_bf16_mt<D, K_LAPLACE, NSEG>(tile_cells, waves, lds, a, s);
    case K_WLAPLACE: return launch_bf16_mt<D, K_WLAPLACE, NSEG>(tile_cells, waves, lds, a, s);
    case K_ELASTICITY: return launch_bf16_mt<D, K_ELASTICITY, NSEG>(tile_cells, waves, lds, a, s);
    case K_PIOLA: return launch_bf16_mt<D, K_PIOLA, NSEG>(tile_cells, waves, lds, a, s);
    case K_CURVED: return hipErrorInvalidValue;  // FP64 only
    case K_NEDELEC: return launch_bf16_mt<D, K_NEDELEC, NSEG>(tile_cells, waves, lds, a, s);
    default: return launch_bf16_mt<D, K_NS, NSEG>(tile_cells, waves, lds, a, s);
    }
}

// Plans the LDS of the launch (staging the output when it fits and `out` is 16-byte
// aligned) and launches the FP64 or split-BF16 contraction.
hipError_t launch_contract(int dim, int kind, bool bf16, int tile_cells, int waves, ContractArgs a,
                           hipStream_t stream) {
    if (a.cells <= 0) return hipSuccess;
    LdsPlan p = plan_lds(dim, kind, tile_cells, a.n_I, a.n_alpha, a.kpad, bf16, kLdsBudget);
    if (p.staged && (reinterpret_cast<uintptr_t>(a.out) & 15u) != 0) {
        p = plan_lds(dim, kind, tile_cells, a.n_I, a.n_alpha, a.kpad, bf16, 0);  // unaligned output: direct stores
        p.total = p.head_bytes + p.g_bytes;
    }
    a.staged = p.staged ? 1 : 0;
    a.stage_bytes = p.stage_bytes;
    a.head_bytes = p.head_bytes;
    if (!bf16) return dim == 2 ? launch_f64_d<2>(kind, tile_cells, waves, p.total, a, stream)
                               : launch_f64_d<3>(kind, tile_cells, waves, p.total, a, stream);
    if (a.n_seg == 3)
        return dim == 2 ? launch_bf16_d<2, 3>(kind, tile_cells, waves, p.total, a, stream)
                        : launch_bf16_d<3, 3>(kind, tile_cells, waves, p.total, a, stream);
    return dim == 2 ? launch_bf16_d<2, 6>(kind, tile_cells, waves, p.total, a, stream)
                    : launch_bf16_d<3, 6>(kind, tile_cells, waves, p.total, a, stream);
}

size_t apply_lds_bytes(int dim, int kind, int tile_cells, int n_I, int n_alpha, int n_dof) {
    const LdsPlan p = plan_lds(dim, kind, tile_cells, n_I, n_alpha, 0, false, ~size_t(0));
    return p.total + align16(static_cast<size_t>(tile_cells) * n_dof * sizeof(double));
}

template <int D, int KIND>
static hipError_t launch_apply_k(int tile_cells, unsigned grid, unsigned block, size_t lds, const ContractArgs& a,
                                 hipStream_t s) {
    switch (tile_cells) {
    case 16: return launch_lds(apply_f64_kernel<D, KIND, 1>, grid, block, lds, s, a);
    case 32: return launch_lds(apply_f64_kernel<D, KIND, 2>, grid, block, lds, s, a);
    default: return launch_lds(apply_f64_kernel<D, KIND, 4>, grid, block, lds, s, a);
    }
}

template <int D>
static hipError_t launch_apply_d(int kind, int tile_cells, unsigned grid, unsigned block, size_t lds,
                                 const ContractArgs& a, hipStream_t s) {
    switch (kind) {
    case K_MASS: return launch_apply_k<D, K_MASS>(tile_cells, grid, block, lds, a, s);
    case K_LAPLACE: return launch_apply_k<D, K_LAPLACE>(tile_cells, grid, block, lds, a, s);
    case K_WLAPLACE: return launch_apply_k<D, K_WLAPLACE>(tile_cells, grid, block, lds, a, s);
    case K_ELASTICITY: return launch_apply_k<D, K_ELASTICITY>(tile_cells, grid, block, lds, a, s);
    case K_PIOLA: return launch_apply_k<D, K_PIOLA>(tile_cells, grid, block, lds, a, s);
    case K_CURVED: return hipErrorInvalidValue;
    case K_NEDELEC: return launch_apply_k<D, K_NEDELEC>(tile_cells, grid, block, lds, a, s);
    default: return launch_apply_k<D, K_NS>(tile_cells, grid, block, lds, a, s);
    }
}

hipError_t launch_apply(int dim, int kind, int tile_cells, int waves, ContractArgs a, hipStream_t stream) {
    if (a.cells <= 0) return hipSuccess;
    if (!a.xloc || a.n_dof <= 0 || a.n_I != a.n_dof * a.n_dof || waves < 1 || waves > 16 ||
        (tile_cells != 16 && tile_cells != 32 && tile_cells != 64))
        return hipErrorInvalidValue;
    const LdsPlan p = plan_lds(dim, kind, tile_cells, a.n_I, a.n_alpha, 0, false, kLdsBudget);
    const size_t lds = apply_lds_bytes(dim, kind, tile_cells, a.n_I, a.n_alpha, a.n_dof);
    if (!p.staged || lds > kLdsBudget) return hipErrorInvalidValue;
    a.staged = 1;
    a.stage_bytes = p.stage_bytes;
    a.head_bytes = p.head_bytes;
    const unsigned grid = static_cast<unsigned>((a.cells + tile_cells - 1) / tile_cells);
    const unsigned block = 64u * waves;
    return dim == 2 ? launch_apply_d<2>(kind, tile_cells, grid, block, lds, a, stream)
                    : launch_apply_d<3>(kind, tile_cells, grid, block, lds, a, stream);
}

}  // namespace ffc
