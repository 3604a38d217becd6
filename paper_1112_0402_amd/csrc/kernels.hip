// Tabulation kernels for gfx950 (CDNA4, 64-wide waves, 160 KiB LDS per CU).
//
//  geometry_kernel     one lane per cell, FP64: J = [x^1 - x^0, ...], det J, g = J^{-1}
//                      (the affine map of Sec. 3.2; det and g_ab = dX_a/dx_b are what
//                      the generated code of Sec. 5.4 reads from its AffineMap)
//  contract_f64        G_K tile built in LDS from the affine map (+ coefficients), then
//                      out[c, i] = sum_alpha G[c, alpha] A^0[i, alpha] on
//                      v_mfma_f64_16x16x4f64: M = 16 cells, N = 16 output entries,
//                      K = the alpha columns of A^0 that are nonzero in those 16 rows
//                      (zero entries of A^0 are skipped, Sec. 6; batching cells turns the
//                      per-cell matrix-vector product into a matrix-matrix product, Sec. 4.5)
//  contract_bf16       the same with G and A^0 split into BF16 pieces, concatenated along
//                      K, on v_mfma_f32_16x16x32_bf16 with FP32 accumulation
//  quadrature_kernel   plain quadrature (Sec. 4.3 / Sec. 6): per cell, physical basis
//                      gradients at the points of a collapsed Gauss-Jacobi rule, then every
//                      entry summed over the points
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace ffc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

enum { K_MASS = 0, K_LAPLACE = 1, K_WLAPLACE = 2, K_ELASTICITY = 3, K_NS = 4 };

// Launch with `lds` bytes of dynamic LDS; above 64 KiB the per-kernel limit is raised
// first (gfx950 has 160 KiB per CU).
template <typename Kernel, typename... Args>
static hipError_t launch_lds(Kernel kernel, unsigned grid, unsigned block, size_t lds, hipStream_t s,
                             const Args&... a) {
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    kernel<<<grid, block, lds, s>>>(a...);
    return hipGetLastError();
}

template <int KIND, int D>
struct FormTraits {
    static constexpr int n_alpha = KIND == K_MASS ? 1
                                 : KIND == K_LAPLACE ? D * D
                                 : KIND == K_WLAPLACE ? (D + 1) * D * D
                                 : KIND == K_ELASTICITY ? D * D * D * D
                                                        : D * (D + 1) * D;
    static constexpr int n_coeff = KIND == K_WLAPLACE ? D + 1 : KIND == K_NS ? D * (D + 1) : 0;
};

// ------------------------------------------------------------------ geometry ----

template <int D>
__device__ __forceinline__ void affine_map(const double (&x)[D + 1][D], double& det, double (&g)[D][D]) {
    double J[D][D];
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
        for (int b = 0; b < D; ++b) J[k][b] = x[b + 1][k] - x[0][k];
    if constexpr (D == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double r = 1.0 / det;
        g[0][0] = J[1][1] * r;
        g[0][1] = -J[0][1] * r;
        g[1][0] = -J[1][0] * r;
        g[1][1] = J[0][0] * r;
    } else {
        const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        const double r = 1.0 / det;
        g[0][0] = c00 * r;
        g[1][0] = c01 * r;
        g[2][0] = c02 * r;
        g[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
        g[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
        g[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
        g[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
        g[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
        g[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
    }
}

template <int D>
__global__ __launch_bounds__(256) void geometry_kernel(int64_t cells, const double* __restrict__ coords,
                                                       int64_t cstride, double* __restrict__ amap, int64_t astride) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (c >= cells) return;
    double x[D + 1][D];
#pragma unroll
    for (int v = 0; v <= D; ++v)
#pragma unroll
        for (int k = 0; k < D; ++k) x[v][k] = __builtin_nontemporal_load(&coords[(v * D + k) * cstride + c]);
    double det, g[D][D];
    affine_map<D>(x, det, g);
    amap[c] = det;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) amap[(1 + a * D + b) * astride + c] = g[a][b];
}

hipError_t launch_geometry(int dim, int64_t cells, const double* coords, int64_t cstride, double* amap,
                           int64_t astride, hipStream_t stream) {
    if (cells <= 0) return hipSuccess;
    const unsigned grid = static_cast<unsigned>((cells + 255) / 256);
    if (dim == 2)
        geometry_kernel<2><<<grid, 256, 0, stream>>>(cells, coords, cstride, amap, astride);
    else
        geometry_kernel<3><<<grid, 256, 0, stream>>>(cells, coords, cstride, amap, astride);
    return hipGetLastError();
}

// ------------------------------------------------------------------ G_K build ---
// am: affine map of the tile in LDS, [1 + D*D][CT] (row 0 = det J, row 1 + a*D + b = g_ab)
// cf: coefficients of the tile in LDS, [n_coeff][CT]

template <int KIND, int D>
__device__ __forceinline__ double g_entry(const double* am, const double* cf, int CT, int c, int alpha) {
    const double adet = fabs(am[c]);
    auto g = [&](int a, int b) { return am[(1 + a * D + b) * CT + c]; };
    if constexpr (KIND == K_MASS) {
        return adet;
    } else if constexpr (KIND == K_LAPLACE) {
        const int a = alpha / D, b = alpha % D;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s += g(a, k) * g(b, k);
        return adet * s;
    } else if constexpr (KIND == K_WLAPLACE) {
        const int t = alpha / (D * D), a = (alpha / D) % D, b = alpha % D;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s += g(a, k) * g(b, k);
        return cf[t * CT + c] * adet * s;
    } else if constexpr (KIND == K_ELASTICITY) {
        const int a = alpha / (D * D * D), j = (alpha / (D * D)) % D, b = (alpha / D) % D, l = alpha % D;
        return adet * g(a, j) * g(b, l);
    } else {  // K_NS: alpha = (k*(D+1) + t)*D + a, G = |det| g_ak w_{k,t}
        const int kt = alpha / D, a = alpha % D;
        const int k = kt / (D + 1);
        return adet * g(a, k) * cf[kt * CT + c];
    }
}

template <int D, int NC>
__device__ __forceinline__ void stage_tile(const ContractArgs& A, int64_t c0, int CT, double* am, double* cf) {
    const int nthr = blockDim.x;
    for (int i = threadIdx.x; i < (1 + D * D) * CT; i += nthr) {
        const int r = i / CT, c = i - r * CT;
        const int64_t cell = c0 + c;
        am[i] = cell < A.cells ? A.amap[r * A.astride + cell] : (r == 0 ? 1.0 : 0.0);
    }
    if constexpr (NC > 0) {
        for (int i = threadIdx.x; i < NC * CT; i += nthr) {
            const int r = i / CT, c = i - r * CT;
            const int64_t cell = c0 + c;
            cf[i] = cell < A.cells ? A.coeffs[r * A.cstride + cell] : 0.0;
        }
    }
}

// Geometry computed in place for a tile (persistent batch path): one lane per cell.
template <int D, int NC>
__device__ __forceinline__ void stage_tile_from_coords(const double* __restrict__ coords, const double* __restrict__ coeffs,
                                                       int64_t cells, int64_t c0, int CT, double* am, double* cf) {
    const int c = threadIdx.x;
    if (c < CT) {
        const int64_t cell = c0 + c;
        if (cell < cells) {
            double x[D + 1][D];
#pragma unroll
            for (int v = 0; v <= D; ++v)
#pragma unroll
                for (int k = 0; k < D; ++k) x[v][k] = __builtin_nontemporal_load(&coords[(v * D + k) * cells + cell]);
            double det, g[D][D];
            affine_map<D>(x, det, g);
            am[c] = det;
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = 0; b < D; ++b) am[(1 + a * D + b) * CT + c] = g[a][b];
        } else {
            am[c] = 1.0;
#pragma unroll
            for (int a = 0; a < D * D; ++a) am[(1 + a) * CT + c] = 0.0;
        }
    }
    if constexpr (NC > 0) {
        for (int i = threadIdx.x; i < NC * CT; i += blockDim.x) {
            const int r = i / CT, cc = i - r * CT;
            const int64_t cell = c0 + cc;
            cf[i] = cell < cells ? coeffs[r * cells + cell] : 0.0;
        }
    }
}

// ----------------------------------------------------------- FP64 contraction ---
// One cell tile of CT = 16*MT cells: G tile into LDS (row stride GS = n_alpha | 1, odd,
// so the 16 lanes reading one alpha column hit distinct banks), then every 16-entry output
// tile on the wave that owns it (tile t on wave t mod waves).
// MFMA operands: lane = 16*kq + r holds A[r][kq] = G[cell r][alpha of k row kq] and
// B[kq][r] = A^0[entry r][that alpha]; the 4 results of lane 16*kq + r are rows
// kq, kq + 4, kq + 8, kq + 12 of column r (the FP64 16x16x4 result layout on gfx950,
// which interleaves rows unlike the BF16 instruction below).

template <int D, int KIND, int MT>
__device__ __forceinline__ void contract_tile_f64(const double* am, const double* cf, double* Gs, int64_t c0,
                                                  int64_t cells, int nI, int n_tiles, const int32_t* __restrict__ koff,
                                                  const int32_t* __restrict__ alpha, const double* __restrict__ bvals,
                                                  double* __restrict__ out) {
    using FT = FormTraits<KIND, D>;
    constexpr int CT = 16 * MT;
    constexpr int NA = FT::n_alpha;
    constexpr int GS = NA | 1;
    for (int i = threadIdx.x; i < CT * NA; i += blockDim.x) {
        const int c = i / NA, al = i - c * NA;
        Gs[c * GS + al] = g_entry<KIND, D>(am, cf, CT, c, al);
    }
    __syncthreads();
    const int waves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    for (int t = wave; t < n_tiles; t += waves) {
        d4 acc[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = d4{0.0, 0.0, 0.0, 0.0};
        const int k0 = koff[t], k1 = koff[t + 1];
        for (int k = k0; k < k1; k += 4) {
            const int al = alpha[k + lk];
            const double bv = bvals[static_cast<int64_t>(k + lk) * 16 + lr];
#pragma unroll
            for (int m = 0; m < MT; ++m)
                acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(Gs[(m * 16 + lr) * GS + al], bv, acc[m], 0, 0, 0);
        }
        const int e = t * 16 + lr;
        if (e < nI) {
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t cell = c0 + m * 16 + i * 4 + lk;
                    if (cell < cells) __builtin_nontemporal_store(acc[m][i], &out[cell * nI + e]);
                }
        }
    }
}

template <int D, int KIND, int MT>
__global__ __launch_bounds__(512) void contract_f64_kernel(ContractArgs A) {
    using FT = FormTraits<KIND, D>;
    constexpr int CT = 16 * MT;
    constexpr int NC = FT::n_coeff;
    extern __shared__ double smem[];
    double* am = smem;
    double* cf = am + (1 + D * D) * CT;
    double* Gs = cf + NC * CT;
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * CT;
    stage_tile<D, NC>(A, c0, CT, am, cf);
    __syncthreads();
    contract_tile_f64<D, KIND, MT>(am, cf, Gs, c0, A.cells, A.n_I, A.n_tiles, A.koff, A.alpha, A.b,
                                   static_cast<double*>(A.out));
}

size_t contract_lds_bytes(int dim, int kind, int tile_cells, int n_alpha, int kpad, bool bf16) {
    const int nc = kind == K_WLAPLACE ? dim + 1 : kind == K_NS ? dim * (dim + 1) : 0;
    size_t head = static_cast<size_t>((1 + dim * dim) + nc) * tile_cells * sizeof(double);
    if (!bf16) return head + static_cast<size_t>(tile_cells) * (n_alpha | 1) * sizeof(double);
    return head + static_cast<size_t>(tile_cells) * (kpad + 8) * sizeof(uint16_t);
}

template <int D, int KIND>
static hipError_t launch_f64_mt(int tile_cells, int waves, const ContractArgs& a, hipStream_t s) {
    const int nA = FormTraits<KIND, D>::n_alpha;
    const size_t lds = contract_lds_bytes(D, KIND, tile_cells, nA, 0, false);
    const unsigned grid = static_cast<unsigned>((a.cells + tile_cells - 1) / tile_cells);
    const unsigned block = 64u * waves;
    switch (tile_cells) {
    case 16: return launch_lds(contract_f64_kernel<D, KIND, 1>, grid, block, lds, s, a);
    case 32: return launch_lds(contract_f64_kernel<D, KIND, 2>, grid, block, lds, s, a);
    default: return launch_lds(contract_f64_kernel<D, KIND, 4>, grid, block, lds, s, a);
    }
}

template <int D>
static hipError_t launch_f64_d(int kind, int tile_cells, int waves, const ContractArgs& a, hipStream_t s) {
    switch (kind) {
    case K_MASS: return launch_f64_mt<D, K_MASS>(tile_cells, waves, a, s);
    case K_LAPLACE: return launch_f64_mt<D, K_LAPLACE>(tile_cells, waves, a, s);
    case K_WLAPLACE: return launch_f64_mt<D, K_WLAPLACE>(tile_cells, waves, a, s);
    case K_ELASTICITY: return launch_f64_mt<D, K_ELASTICITY>(tile_cells, waves, a, s);
    default: return launch_f64_mt<D, K_NS>(tile_cells, waves, a, s);
    }
}

hipError_t launch_contract_f64(int dim, int kind, int tile_cells, int waves, const ContractArgs& a,
                               hipStream_t stream) {
    if (a.cells <= 0) return hipSuccess;
    return dim == 2 ? launch_f64_d<2>(kind, tile_cells, waves, a, stream)
                    : launch_f64_d<3>(kind, tile_cells, waves, a, stream);
}

// ----------------------------------------------------------- BF16 contraction ---

// round to nearest even BF16, returned as the double it represents (|x| in normal range)
__device__ __forceinline__ double rn_bf16(double x) {
    unsigned long long u = __double_as_longlong(x);
    const unsigned long long lsb = (u >> 45) & 1ull;
    u += ((1ull << 44) - 1ull) + lsb;
    u &= ~((1ull << 45) - 1ull);
    return __longlong_as_double(u);
}

__device__ __forceinline__ unsigned short bf16_of(double representable) {
    const float f = static_cast<float>(representable);  // exact
    return static_cast<unsigned short>(__float_as_uint(f) >> 16);
}

// G tile split into BF16 pieces laid out as the concatenated K of the form's segments:
// Gp[c][s * n_alpha + alpha] = piece gpiece[s] of G[c][alpha]; row stride kpad + 8.
// MFMA operands: lane = 16*kq + r holds 8 consecutive K values kq*8 .. kq*8+7 of row r of
// the G tile (A) and of column r of the A^0 tile (B); the same K order on both sides.
// The 4 results of lane 16*kq + r are rows 4*kq .. 4*kq + 3 of column r.
template <int D, int KIND, int MT, int NSEG>
__device__ __forceinline__ void contract_tile_bf16(const double* am, const double* cf, unsigned short* Gp, int64_t c0,
                                                   int64_t cells, int nI, int n_tiles, int kpad, const int* gpiece,
                                                   const uint16_t* __restrict__ bb,
                                                   const uint8_t* __restrict__ nonzero, float* __restrict__ out) {
    using FT = FormTraits<KIND, D>;
    constexpr int CT = 16 * MT;
    constexpr int NA = FT::n_alpha;
    const int KS = kpad + 8;
    for (int i = threadIdx.x; i < CT * NA; i += blockDim.x) {
        const int c = i / NA, al = i - c * NA;
        const double gv = g_entry<KIND, D>(am, cf, CT, c, al);
        double piece[3];
        piece[0] = rn_bf16(gv);
        piece[1] = rn_bf16(gv - piece[0]);
        piece[2] = rn_bf16((gv - piece[0]) - piece[1]);
#pragma unroll
        for (int s = 0; s < NSEG; ++s) Gp[c * KS + s * NA + al] = bf16_of(piece[gpiece[s]]);
    }
    const int w = kpad - NSEG * NA;
    for (int i = threadIdx.x; i < CT * w; i += blockDim.x) {
        const int c = i / w, k = NSEG * NA + (i - c * w);
        Gp[c * KS + k] = 0;
    }
    __syncthreads();
    const int waves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int kchunks = kpad / 32;
    for (int t = wave; t < n_tiles; t += waves) {
        f4 acc[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = f4{0.f, 0.f, 0.f, 0.f};
        if (nonzero[t]) {
            const u16x8* bt = reinterpret_cast<const u16x8*>(bb) + static_cast<int64_t>(t) * (kpad / 8) * 16;
            for (int kc = 0; kc < kchunks; ++kc) {
                const bf8 bv = __builtin_bit_cast(bf8, bt[(kc * 4 + lk) * 16 + lr]);
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    const u16x8 av = *reinterpret_cast<const u16x8*>(&Gp[(m * 16 + lr) * KS + kc * 32 + lk * 8]);
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, av), bv, acc[m], 0, 0, 0);
                }
            }
        }
        const int e = t * 16 + lr;
        if (e < nI) {
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t cell = c0 + m * 16 + lk * 4 + i;
                    if (cell < cells) __builtin_nontemporal_store(acc[m][i], &out[cell * nI + e]);
                }
        }
    }
}

template <int D, int KIND, int MT, int NSEG>
__global__ __launch_bounds__(512) void contract_bf16_kernel(ContractArgs A) {
    using FT = FormTraits<KIND, D>;
    constexpr int CT = 16 * MT;
    constexpr int NC = FT::n_coeff;
    extern __shared__ double smem[];
    double* am = smem;
    double* cf = am + (1 + D * D) * CT;
    unsigned short* Gp = reinterpret_cast<unsigned short*>(cf + NC * CT);
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * CT;
    stage_tile<D, NC>(A, c0, CT, am, cf);
    __syncthreads();
    contract_tile_bf16<D, KIND, MT, NSEG>(am, cf, Gp, c0, A.cells, A.n_I, A.n_tiles, A.kpad, A.gpiece, A.bb, A.nonzero,
                                          static_cast<float*>(A.out));
}

template <int D, int KIND, int NSEG>
static hipError_t launch_bf16_mt(int tile_cells, int waves, const ContractArgs& a, hipStream_t s) {
    const int nA = FormTraits<KIND, D>::n_alpha;
    const size_t lds = contract_lds_bytes(D, KIND, tile_cells, nA, a.kpad, true);
    const unsigned grid = static_cast<unsigned>((a.cells + tile_cells - 1) / tile_cells);
    const unsigned block = 64u * waves;
    switch (tile_cells) {
    case 16: return launch_lds(contract_bf16_kernel<D, KIND, 1, NSEG>, grid, block, lds, s, a);
    case 32: return launch_lds(contract_bf16_kernel<D, KIND, 2, NSEG>, grid, block, lds, s, a);
    default: return launch_lds(contract_bf16_kernel<D, KIND, 4, NSEG>, grid, block, lds, s, a);
    }
}

template <int D, int NSEG>
static hipError_t launch_bf16_d(int kind, int tile_cells, int waves, const ContractArgs& a, hipStream_t s) {
    switch (kind) {
    case K_MASS: return launch_bf16_mt<D, K_MASS, NSEG>(tile_cells, waves, a, s);
    case K_LAPLACE: return launch_bf16_mt<D, K_LAPLACE, NSEG>(tile_cells, waves, a, s);
    case K_WLAPLACE: return launch_bf16_mt<D, K_WLAPLACE, NSEG>(tile_cells, waves, a, s);
    case K_ELASTICITY: return launch_bf16_mt<D, K_ELASTICITY, NSEG>(tile_cells, waves, a, s);
    default: return launch_bf16_mt<D, K_NS, NSEG>(tile_cells, waves, a, s);
    }
}

hipError_t launch_contract_bf16(int dim, int kind, int tile_cells, int waves, const ContractArgs& a,
                                hipStream_t stream) {
    if (a.cells <= 0) return hipSuccess;
    if (a.n_seg == 3)
        return dim == 2 ? launch_bf16_d<2, 3>(kind, tile_cells, waves, a, stream)
                        : launch_bf16_d<3, 3>(kind, tile_cells, waves, a, stream);
    return dim == 2 ? launch_bf16_d<2, 6>(kind, tile_cells, waves, a, stream)
                    : launch_bf16_d<3, 6>(kind, tile_cells, waves, a, stream);
}

// ------------------------------------------------------- persistent mixed batch ---
// Work unit = (item, 64-cell tile).  Each workgroup takes units from one atomic counter
// until the queue is empty; the last workgroup to leave resets the counters, so the
// launch can be replayed (for example from a captured graph) with no separate reset.
// Geometry is computed in place, one lane per cell.

constexpr int kBatchMT = 4;
constexpr int kBatchCT = 16 * kBatchMT;
constexpr int kBatchMaxCoeff = 12;

size_t batch_lds_bytes(int max_alpha, int max_kpad, bool bf16) {
    size_t head = static_cast<size_t>((1 + 9) + kBatchMaxCoeff) * kBatchCT * sizeof(double);
    if (!bf16) return head + static_cast<size_t>(kBatchCT) * (max_alpha | 1) * sizeof(double);
    return head + static_cast<size_t>(kBatchCT) * (max_kpad + 8) * sizeof(uint16_t);
}

template <int D, int KIND, bool BF16>
__device__ __forceinline__ void batch_unit(const BatchItem& it, int64_t c0, double* smem) {
    constexpr int NC = FormTraits<KIND, D>::n_coeff;
    double* am = smem;
    double* cf = am + (1 + D * D) * kBatchCT;
    double* G = cf + NC * kBatchCT;
    stage_tile_from_coords<D, NC>(it.coords, it.coeffs, it.cells, c0, kBatchCT, am, cf);
    __syncthreads();
    if constexpr (BF16) {
        if (it.n_seg == 3)
            contract_tile_bf16<D, KIND, kBatchMT, 3>(am, cf, reinterpret_cast<unsigned short*>(G), c0, it.cells, it.n_I,
                                                     it.n_tiles, it.kpad, it.gpiece, it.bb, it.nonzero,
                                                     static_cast<float*>(it.out));
        else
            contract_tile_bf16<D, KIND, kBatchMT, 6>(am, cf, reinterpret_cast<unsigned short*>(G), c0, it.cells, it.n_I,
                                                     it.n_tiles, it.kpad, it.gpiece, it.bb, it.nonzero,
                                                     static_cast<float*>(it.out));
    } else {
        contract_tile_f64<D, KIND, kBatchMT>(am, cf, G, c0, it.cells, it.n_I, it.n_tiles, it.koff, it.alpha, it.b,
                                             static_cast<double*>(it.out));
    }
}

template <bool BF16>
__global__ __launch_bounds__(256) void batch_kernel(const BatchItem* __restrict__ items, int n_items,
                                                    int64_t total_units, int* counters) {
    extern __shared__ double smem[];
    __shared__ int64_t s_unit;
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t u = atomicAdd(&counters[0], 1);
            int lo = 0;
            if (u < total_units) {
                int hi = n_items - 1;
                while (lo < hi) {  // last item with unit_begin <= u
                    const int mid = (lo + hi + 1) >> 1;
                    if (items[mid].unit_begin <= u)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
            }
            s_unit = u;
            s_item = lo;
        }
        __syncthreads();
        const int64_t u = s_unit;
        if (u >= total_units) break;
        const BatchItem& it = items[s_item];
        const int64_t c0 = (u - it.unit_begin) * kBatchCT;
        switch (it.dim * 8 + it.kind) {
        case 16 + K_MASS: batch_unit<2, K_MASS, BF16>(it, c0, smem); break;
        case 16 + K_LAPLACE: batch_unit<2, K_LAPLACE, BF16>(it, c0, smem); break;
        case 16 + K_WLAPLACE: batch_unit<2, K_WLAPLACE, BF16>(it, c0, smem); break;
        case 16 + K_ELASTICITY: batch_unit<2, K_ELASTICITY, BF16>(it, c0, smem); break;
        case 16 + K_NS: batch_unit<2, K_NS, BF16>(it, c0, smem); break;
        case 24 + K_MASS: batch_unit<3, K_MASS, BF16>(it, c0, smem); break;
        case 24 + K_LAPLACE: batch_unit<3, K_LAPLACE, BF16>(it, c0, smem); break;
        case 24 + K_WLAPLACE: batch_unit<3, K_WLAPLACE, BF16>(it, c0, smem); break;
        case 24 + K_ELASTICITY: batch_unit<3, K_ELASTICITY, BF16>(it, c0, smem); break;
        default: batch_unit<3, K_NS, BF16>(it, c0, smem); break;
        }
        __syncthreads();  // LDS and s_unit are reused by the next unit
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const int done = atomicAdd(&counters[1], 1);
        if (done == static_cast<int>(gridDim.x) - 1) {  // every other workgroup has left the loop
            atomicExch(&counters[0], 0);
            atomicExch(&counters[1], 0);
        }
    }
}

hipError_t launch_batch(const BatchItem* items_dev, int n_items, int64_t total_units, int* counter_dev, int grid,
                        bool bf16, size_t lds, hipStream_t stream) {
    if (total_units <= 0) return hipSuccess;
    if (bf16) return launch_lds(batch_kernel<true>, grid, 256, lds, stream, items_dev, n_items, total_units, counter_dev);
    return launch_lds(batch_kernel<false>, grid, 256, lds, stream, items_dev, n_items, total_units, counter_dev);
}

// ------------------------------------------------------------------ quadrature ---
// LDS per cell slot: geo [1 + D*D] (|det|, g), W [npts] (weight * |det| * coefficient),
// grad [npts][ns][D] physical gradients, conv [npts][ns] ((w . grad) phi, NS only).
// Shared: phi [npts][ns] reference values.

__host__ __device__ static int quad_slot_doubles(int dim, int kind, int ns, int npts) {
    int s = (1 + dim * dim) + npts;
    if (kind != K_MASS) s += npts * ns * dim;
    if (kind == K_NS) s += npts * ns;
    return s;
}

int quad_cells_per_block(int dim, int kind, int ns, int npts) {
    const size_t budget = 64 * 1024;
    const size_t shared = static_cast<size_t>(npts) * ns * sizeof(double);
    const size_t slot = static_cast<size_t>(quad_slot_doubles(dim, kind, ns, npts)) * sizeof(double);
    int qc = static_cast<int>((budget - std::min(budget / 2, shared)) / slot);
    if (qc > 8) qc = 8;
    if (qc < 1) qc = 1;
    return qc;
}

template <int D, int KIND>
__global__ __launch_bounds__(256) void quadrature_kernel(QuadArgs A) {
    extern __shared__ double smem[];
    const int ns = A.ns, n = A.n, nI = A.n_I, NQ = A.npts, QC = A.cells_per_block;
    const int slot = quad_slot_doubles(D, KIND, ns, NQ);
    double* phis = smem;                 // [NQ][ns]
    double* slots = smem + NQ * ns;      // [QC][slot]
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * QC;
    const int tid = threadIdx.x, nthr = blockDim.x;

    for (int i = tid; i < NQ * ns; i += nthr) phis[i] = A.phi[i];
    // geometry, one lane per cell
    if (tid < QC) {
        double* geo = slots + tid * slot;
        const int64_t cell = c0 + tid;
        if (cell < A.cells) {
            double x[D + 1][D];
#pragma unroll
            for (int v = 0; v <= D; ++v)
#pragma unroll
                for (int k = 0; k < D; ++k) x[v][k] = A.coords[(v * D + k) * A.cstride + cell];
            double det, g[D][D];
            affine_map<D>(x, det, g);
            geo[0] = fabs(det);
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = 0; b < D; ++b) geo[1 + a * D + b] = g[a][b];
        } else {
            geo[0] = 0.0;
#pragma unroll
            for (int a = 0; a < D * D; ++a) geo[1 + a] = (a % (D + 1) == 0) ? 1.0 : 0.0;
        }
    }
    __syncthreads();
    // per point: weights (with the P1 coefficient for wlaplace) and physical gradients
    for (int i = tid; i < QC * NQ; i += nthr) {
        const int c = i / NQ, q = i - c * NQ;
        double* geo = slots + c * slot;
        double W = A.wts[q] * geo[0];
        if constexpr (KIND == K_WLAPLACE) {
            const int64_t cell = c0 + c;
            double lam[D + 1];
            lam[0] = 1.0;
#pragma unroll
            for (int b = 0; b < D; ++b) {
                lam[b + 1] = A.pts[q * D + b];
                lam[0] -= lam[b + 1];
            }
            double w = 0.0;
            if (cell < A.cells)
#pragma unroll
                for (int t = 0; t <= D; ++t) w += A.coeffs[t * A.kstride + cell] * lam[t];
            W *= w;
        }
        geo[1 + D * D + q] = W;
    }
    if constexpr (KIND != K_MASS) {
        for (int i = tid; i < QC * NQ * ns; i += nthr) {
            const int c = i / (NQ * ns), r = i - c * (NQ * ns);  // r = q * ns + s
            double* geo = slots + c * slot;
            double* grad = geo + 1 + D * D + NQ;
            const double* dref = A.dphi + static_cast<int64_t>(r) * D;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                double s = 0.0;
#pragma unroll
                for (int b = 0; b < D; ++b) s += geo[1 + b * D + k] * dref[b];
                grad[r * D + k] = s;
            }
        }
    }
    if constexpr (KIND == K_NS) {
        __syncthreads();
        for (int i = tid; i < QC * NQ * ns; i += nthr) {
            const int c = i / (NQ * ns), r = i - c * (NQ * ns);
            const int q = r / ns;
            double* geo = slots + c * slot;
            const double* grad = geo + 1 + D * D + NQ;
            double* conv = geo + 1 + D * D + NQ + NQ * ns * D;
            const int64_t cell = c0 + c;
            double lam[D + 1];
            lam[0] = 1.0;
#pragma unroll
            for (int b = 0; b < D; ++b) {
                lam[b + 1] = A.pts[q * D + b];
                lam[0] -= lam[b + 1];
            }
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                double wk = 0.0;
                if (cell < A.cells)
#pragma unroll
                    for (int t = 0; t <= D; ++t) wk += A.coeffs[(k * (D + 1) + t) * A.kstride + cell] * lam[t];
                s += wk * grad[r * D + k];
            }
            conv[r] = s;
        }
    }
    __syncthreads();
    // entries
    for (int i = tid; i < QC * nI; i += nthr) {
        const int c = i / nI, e = i - c * nI;
        const int64_t cell = c0 + c;
        if (cell >= A.cells) continue;
        const double* geo = slots + c * slot;
        const double* W = geo + 1 + D * D;
        const double* grad = W + NQ;
        const int i1 = e / n, i2 = e - i1 * n;
        double acc = 0.0;
        if constexpr (KIND == K_MASS) {
            for (int q = 0; q < NQ; ++q) acc += W[q] * phis[q * ns + i1] * phis[q * ns + i2];
        } else if constexpr (KIND == K_LAPLACE || KIND == K_WLAPLACE) {
            for (int q = 0; q < NQ; ++q) {
                const double* gi = grad + (q * ns + i1) * D;
                const double* gj = grad + (q * ns + i2) * D;
                double dot = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k) dot += gi[k] * gj[k];
                acc += W[q] * dot;
            }
        } else if constexpr (KIND == K_ELASTICITY) {
            const int c1 = i1 / ns, s1 = i1 - c1 * ns, c2 = i2 / ns, s2 = i2 - c2 * ns;
            const double mu = A.mu, lam = A.lambda;
            for (int q = 0; q < NQ; ++q) {
                const double* gi = grad + (q * ns + s1) * D;
                const double* gj = grad + (q * ns + s2) * D;
                double v = mu * gi[c2] * gj[c1] + lam * gi[c1] * gj[c2];
                if (c1 == c2) {
                    double dot = 0.0;
#pragma unroll
                    for (int k = 0; k < D; ++k) dot += gi[k] * gj[k];
                    v += mu * dot;
                }
                acc += W[q] * v;
            }
        } else {  // NS
            const int c1 = i1 / ns, s1 = i1 - c1 * ns, c2 = i2 / ns, s2 = i2 - c2 * ns;
            if (c1 == c2) {
                const double* conv = grad + NQ * ns * D;
                for (int q = 0; q < NQ; ++q) acc += W[q] * phis[q * ns + s1] * conv[q * ns + s2];
            }
        }
        A.out[cell * nI + e] = acc;
    }
}

template <int D>
static hipError_t launch_quad_d(int kind, const QuadArgs& a, hipStream_t s) {
    const size_t lds = (static_cast<size_t>(a.npts) * a.ns +
                        static_cast<size_t>(a.cells_per_block) * quad_slot_doubles(D, kind, a.ns, a.npts)) *
                       sizeof(double);
    const unsigned grid = static_cast<unsigned>((a.cells + a.cells_per_block - 1) / a.cells_per_block);
    switch (kind) {
    case K_MASS: return launch_lds(quadrature_kernel<D, K_MASS>, grid, 256, lds, s, a);
    case K_LAPLACE: return launch_lds(quadrature_kernel<D, K_LAPLACE>, grid, 256, lds, s, a);
    case K_WLAPLACE: return launch_lds(quadrature_kernel<D, K_WLAPLACE>, grid, 256, lds, s, a);
    case K_ELASTICITY: return launch_lds(quadrature_kernel<D, K_ELASTICITY>, grid, 256, lds, s, a);
    default: return launch_lds(quadrature_kernel<D, K_NS>, grid, 256, lds, s, a);
    }
}

hipError_t launch_quadrature(int dim, int kind, const QuadArgs& a, hipStream_t stream) {
    if (a.cells <= 0) return hipSuccess;
    return dim == 2 ? launch_quad_d<2>(kind, a, stream) : launch_quad_d<3>(kind, a, stream);
}

}  // namespace ffc
