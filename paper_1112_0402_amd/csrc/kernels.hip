// Tabulation kernels for gfx950 (CDNA4, 64-wide waves, 160 KiB LDS per CU).
//
//  geometry_kernel     one lane per cell, FP64: J = [x^1 - x^0, ...], det J, g = J^{-1}
//                      (the affine map of Sec. 3.2; det and g_ab = dX_a/dx_b are what
//                      the generated code of Sec. 5.5 reads from its AffineMap)
//  contract_f64        G_K tile built in LDS from the affine map (+ coefficients), then
//                      out[c, i] = sum_alpha G[c, alpha] A^0[i, alpha] on
//                      v_mfma_f64_16x16x4f64: M = 16 cells, N = 16 output entries,
//                      K = the alpha columns of A^0 that are nonzero in those 16 rows
//                      (zero entries of A^0 are skipped, Sec. 6; batching cells turns the
//                      per-cell matrix-vector product into a matrix-matrix product, Sec. 3.5)
//  contract_bf16       the same with G and A^0 split into BF16 pieces, concatenated along
//                      K, on v_mfma_f32_16x16x32_bf16 with FP32 accumulation
//  contract_*_persistent  one 1024-thread workgroup per CU walking cell tiles: each compute
//                      wave keeps its share of the A^0 tiles in registers, dedicated I/O
//                      waves write the staged rows of one tile during the next tile's MFMA
//                      steps (also the operator action y_K = A^K x_K, and mixed batches)
//  curved_geometry_kernel  cells with P2 geometry: |det J| g g^T at every quadrature point
//                      (Sec. 3.4: the integral becomes a sum over points, still a contraction)
//  quadrature_kernel   the quadrature comparison (Sec. 4.3 / Sec. 6): per cell, physical
//                      basis gradients at the points of a collapsed Gauss-Jacobi rule, then
//                      every entry summed over the points, register-blocked over entries
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace ffc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

enum { K_MASS = 0, K_LAPLACE = 1, K_WLAPLACE = 2, K_ELASTICITY = 3, K_NS = 4, K_PIOLA = 5, K_CURVED = 6, K_NEDELEC = 7 };

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

// Pointers read from a descriptor in memory are generic to the compiler, which then emits
// flat loads and stores (slower, and counted by lgkmcnt as well, so LDS waits would also
// wait for them).  Every buffer of this library lives in global memory: say so.
template <typename T>
__device__ __forceinline__ T* as_global(T* p) {
    // through an integer: a cast pair generic -> global -> generic would fold away
    return (T*)((__attribute__((address_space(1))) T*)reinterpret_cast<uintptr_t>(p));
}

template <int KIND, int D>
struct FormTraits {
    // G entries per cell; the symmetric geometry tensors keep each unordered index pair once
    static constexpr int n_alpha = KIND == K_MASS ? 1
                                 : KIND == K_LAPLACE || KIND == K_NEDELEC ? D * (D + 1) / 2
                                 : KIND == K_WLAPLACE ? (D + 1) * D * (D + 1) / 2
                                 : KIND == K_ELASTICITY ? D * D * (D * D + 1) / 2
                                 : KIND == K_PIOLA ? D * (D + 1) / 2
                                 : KIND == K_CURVED ? 0  // per form (quadrature points x pairs), at run time
                                                        : D * (D + 1) * D;
    static constexpr int n_coeff = KIND == K_WLAPLACE ? D + 1 : KIND == K_NS ? D * (D + 1) : 0;
};

// ------------------------------------------------------------------ geometry ----

// a*d - b*c to within about one rounding: the rounding error of b*c is recovered exactly
// with an FMA (Kahan's algorithm), so the cancellation of the two products on a badly
// shaped cell does not magnify it
__device__ __forceinline__ double diff_of_products(double a, double d, double b, double c) {
#pragma clang fp contract(off)
    const double w = b * c;
    const double e = fma(-b, c, w);  // w - b*c, exact
    const double f = fma(a, d, -w);
    return f + e;
}

// det J and g = J^{-1} (g_ab = dX_a / dx_b) of a Jacobian J_kb = dx_k / dX_b.  The
// cofactors are differences of products and det J a sum of three products that cancel
// on needles and slivers (det small against the products of edge lengths): both are
// compensated -- cofactors by diff_of_products, the cofactor expansion of det by an
// error-free transformation of every product and sum (Ogita, Rump and Oishi's Dot2) -- so det J
// and g keep a relative error of a few roundings up to aspect ratios ~1e3 instead of
// growing with the square of the aspect ratio.
template <int D>
__device__ __forceinline__ void invert_jacobian(const double (&J)[D][D], double& det, double (&g)[D][D]) {
    // no multiply may be fused into a following add: the error terms assume rounded products
#pragma clang fp contract(off)
    if constexpr (D == 2) {
        det = diff_of_products(J[0][0], J[1][1], J[0][1], J[1][0]);
        const double r = 1.0 / det;
        g[0][0] = J[1][1] * r;
        g[0][1] = -J[0][1] * r;
        g[1][0] = -J[1][0] * r;
        g[1][1] = J[0][0] * r;
    } else {
        const double c00 = diff_of_products(J[1][1], J[2][2], J[1][2], J[2][1]);
        const double c01 = diff_of_products(J[1][2], J[2][0], J[1][0], J[2][2]);
        const double c02 = diff_of_products(J[1][0], J[2][1], J[1][1], J[2][0]);
        // Dot2: p carries the rounded sum, s the exact errors of every product and sum
        double p = J[0][0] * c00;
        double s = fma(J[0][0], c00, -p);
        {
            const double h = J[0][1] * c01, r = fma(J[0][1], c01, -h);
            const double t = p + h, z = t - p;
            s += ((p - (t - z)) + (h - z)) + r;
            p = t;
        }
        {
            const double h = J[0][2] * c02, r = fma(J[0][2], c02, -h);
            const double t = p + h, z = t - p;
            s += ((p - (t - z)) + (h - z)) + r;
            p = t;
        }
        det = p + s;
        const double r = 1.0 / det;
        g[0][0] = c00 * r;
        g[1][0] = c01 * r;
        g[2][0] = c02 * r;
        g[0][1] = diff_of_products(J[0][2], J[2][1], J[0][1], J[2][2]) * r;
        g[1][1] = diff_of_products(J[0][0], J[2][2], J[0][2], J[2][0]) * r;
        g[2][1] = diff_of_products(J[0][1], J[2][0], J[0][0], J[2][1]) * r;
        g[0][2] = diff_of_products(J[0][1], J[1][2], J[0][2], J[1][1]) * r;
        g[1][2] = diff_of_products(J[0][2], J[1][0], J[0][0], J[1][2]) * r;
        g[2][2] = diff_of_products(J[0][0], J[1][1], J[0][1], J[1][0]) * r;
    }
}

template <int D>
__device__ __forceinline__ void affine_map(const double (&x)[D + 1][D], double& det, double (&g)[D][D]) {
    double J[D][D];
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
        for (int b = 0; b < D; ++b) J[k][b] = x[b + 1][k] - x[0][k];
    invert_jacobian<D>(J, det, g);
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

// Cells with P2 geometry (NG nodes): one lane per cell; at every quadrature point p,
// J(X_p) = sum_k x_k (grad Psi_k(X_p))^T, then G[(p, a <= b)] = |det J| (g g^T)_ab, SoA
// [n_pts * D(D+1)/2][gstride].  grad: [n_pts][NG][D] reference gradients of the geometry basis.
template <int D>
__global__ __launch_bounds__(256) void curved_geometry_kernel(int64_t cells, const double* __restrict__ coords,
                                                              int64_t cstride, int n_pts,
                                                              const double* __restrict__ grad, double* __restrict__ G,
                                                              int64_t gstride) {
    constexpr int NG = D == 2 ? 6 : 10;
    constexpr int NP = D * (D + 1) / 2;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (c >= cells) return;
    double x[NG][D];
#pragma unroll
    for (int k = 0; k < NG; ++k)
#pragma unroll
        for (int j = 0; j < D; ++j) x[k][j] = __builtin_nontemporal_load(&coords[(k * D + j) * cstride + c]);
    for (int p = 0; p < n_pts; ++p) {
        double J[D][D];
#pragma unroll
        for (int j = 0; j < D; ++j)
#pragma unroll
            for (int b = 0; b < D; ++b) J[j][b] = 0.0;
#pragma unroll
        for (int k = 0; k < NG; ++k)
#pragma unroll
            for (int b = 0; b < D; ++b) {
                const double gk = grad[(p * NG + k) * D + b];
#pragma unroll
                for (int j = 0; j < D; ++j) J[j][b] = fma(x[k][j], gk, J[j][b]);
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
                G[(p * NP + pr) * gstride + c] = adet * s;
            }
    }
}

hipError_t launch_curved_geometry(int dim, int64_t cells, const double* coords, int64_t cstride, int n_pts,
                                  const double* grad, double* G, int64_t gstride, hipStream_t stream) {
    if (cells <= 0) return hipSuccess;
    const unsigned grid = static_cast<unsigned>((cells + 255) / 256);
    if (dim == 2)
        curved_geometry_kernel<2><<<grid, 256, 0, stream>>>(cells, coords, cstride, n_pts, grad, G, gstride);
    else
        curved_geometry_kernel<3><<<grid, 256, 0, stream>>>(cells, coords, cstride, n_pts, grad, G, gstride);
    return hipGetLastError();
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

// Index pair (u, v), u <= v < N, of pair number p, pairs numbered row by row (row u
// starts at u*N - u*(u-1)/2).
template <int N>
__device__ __forceinline__ void upper_pair(int p, int& u, int& v) {
    int r = 0;
#pragma unroll
    for (int k = 1; k < N; ++k) r += p >= k * N - k * (k - 1) / 2;
    u = r;
    v = p - (r * N - r * (r - 1) / 2) + r;
}

template <int KIND, int D>
__device__ __forceinline__ double g_entry(const double* am, const double* cf, int CT, int c, int alpha) {
    const double adet = fabs(am[c]);
    auto g = [&](int a, int b) { return am[(1 + a * D + b) * CT + c]; };
    if constexpr (KIND == K_MASS) {
        return adet;
    } else if constexpr (KIND == K_LAPLACE || KIND == K_NEDELEC) {  // alpha = pair (a, b), a <= b
        // (Nedelec under the covariant Piola map: the same |det J| (g g^T)_ab)
        int a, b;
        upper_pair<D>(alpha, a, b);
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s += g(a, k) * g(b, k);
        return adet * s;
    } else if constexpr (KIND == K_WLAPLACE) {  // alpha = t * pairs + pair (a, b)
        constexpr int NP = D * (D + 1) / 2;
        const int t = alpha / NP;
        int a, b;
        upper_pair<D>(alpha - t * NP, a, b);
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s += g(a, k) * g(b, k);
        return cf[t * CT + c] * adet * s;
    } else if constexpr (KIND == K_PIOLA) {  // alpha = pair (a, b), a <= b
        // G = (J^T J)_ab / |det J| with J = g^{-1} = det J adj(g): G = |det J| sum_k adj_ka adj_kb
        int a, b;
        upper_pair<D>(alpha, a, b);
        auto adj = [&](int k, int m) -> double {  // adj(g)_km = cofactor (m, k) of g
            if constexpr (D == 2) {
                return k == m ? g(1 - m, 1 - k) : -g(k, m);
            } else {
                const int m1 = (m + 1) % 3, m2 = (m + 2) % 3, k1 = (k + 1) % 3, k2 = (k + 2) % 3;
                return g(m1, k1) * g(m2, k2) - g(m1, k2) * g(m2, k1);
            }
        };
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s += adj(k, a) * adj(k, b);
        return adet * s;
    } else if constexpr (KIND == K_ELASTICITY) {  // alpha = pair (a*D + j, b*D + l)
        int u, v;
        upper_pair<D * D>(alpha, u, v);
        const int a = u / D, j = u % D, b = v / D, l = v % D;
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

// ------------------------------------------------------ LDS plan and output write ---
// LDS of a contraction workgroup, in order (each part 16-byte aligned):
//   st   [CT][n_I] output values (double, or float in split modes) -- staged plans only
//   am   [1 + D*D][CT] affine map,  cf [n_coeff][CT] coefficients
//   G    FP64: [CT][n_alpha | 1] doubles;  split: [CT][kpad + 8] BF16 pieces
// A staged workgroup writes its whole output region -- CT consecutive cells, i.e. one
// contiguous run of CT * n_I values -- with 16-byte stores once every tile is done, so the
// HBM sees full aligned lines in streaming order whatever the order of the tiles.

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline int n_coeff_of(int dim, int kind) {
    return kind == K_WLAPLACE ? dim + 1 : kind == K_NS ? dim * (dim + 1) : 0;
}

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
template <typename T>
__device__ __forceinline__ void write_region(const T* __restrict__ st, T* __restrict__ out, int64_t n) {
    constexpr int V = 16 / sizeof(T);
    typedef T vec __attribute__((ext_vector_type(V)));
    const int64_t nv = n / V;
    const vec* s = reinterpret_cast<const vec*>(st);
    vec* o = reinterpret_cast<vec*>(out);
    for (int64_t i = threadIdx.x; i < nv; i += blockDim.x) o[i] = s[i];
    for (int64_t i = nv * V + threadIdx.x; i < n; i += blockDim.x) out[i] = st[i];
}

// ----------------------------------------------------------- FP64 contraction ---
// One cell tile of CT = 16*MT cells: G tile into LDS (row stride GS = n_alpha | 1, odd,
// so the 16 lanes reading one alpha column hit distinct banks), then every 16-entry output
// tile on the wave that owns it (tile t on wave t mod waves; tile loops are wave-uniform).
// MFMA operands: lane = 16*kq + r holds A[r][kq] = G[cell r][alpha of k row kq] and
// B[kq][r] = A^0[entry of column r][that alpha]; the 4 results of lane 16*kq + r are rows
// kq, kq + 4, kq + 8, kq + 12 of column r (the FP64 16x16x4 result layout on gfx950,
// which interleaves rows unlike the BF16 instruction below).
// Per k step: one scalar load of the 4 packed alpha indices and one 8-byte B load per
// lane, both fetched one step ahead; the MT LDS reads are issued before the MT MFMAs.
// Results go to the staging rows st (then one contiguous write of the whole tile), or
// straight to global memory when the tile's output does not fit in LDS (st == nullptr).

template <int D, int KIND, int MT>
__device__ __forceinline__ void contract_tile_f64(const double* am, const double* cf, double* Gs, double* st,
                                                  int64_t c0, int64_t cells, int nI, int n_tiles,
                                                  const int32_t* __restrict__ koff, const uint32_t* __restrict__ apack,
                                                  const int32_t* __restrict__ entry, const double* __restrict__ bvals,
                                                  double* __restrict__ out, int sym_n, int na_rt = 0,
                                                  const double* __restrict__ gmem = nullptr, int64_t gstride = 0) {
    using FT = FormTraits<KIND, D>;
    constexpr int CT = 16 * MT;
    // K_CURVED: G comes precomputed from memory (SoA [n_alpha][gstride]), n_alpha at run time
    const int NA = KIND == K_CURVED ? na_rt : FT::n_alpha;
    const int GS = NA | 1;
    if constexpr (KIND == K_CURVED) {  // (gmem == nullptr: the caller has built the G tile)
        if (gmem) {
            for (int i = threadIdx.x; i < CT * NA; i += blockDim.x) {
                const int al = i / CT, c = i - (i / CT) * CT;
                const int64_t cell = c0 + c;
                Gs[c * GS + al] = cell < cells ? gmem[al * gstride + cell] : 0.0;
            }
        }
    } else {
        for (int i = threadIdx.x; i < CT * NA; i += blockDim.x) {
            const int c = i / NA, al = i - c * NA;
            Gs[c * GS + al] = g_entry<KIND, D>(am, cf, CT, c, al);
        }
    }
    __syncthreads();
    const int waves = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const double* grow = Gs + lr * GS;
    for (int t = wave; t < n_tiles; t += waves) {
        d4 acc[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = d4{0.0, 0.0, 0.0, 0.0};
        const int k0 = koff[t];
        const int nk = (koff[t + 1] - k0) >> 2;
        const int e = entry[t * 16 + lr];
        if (nk > 0) {
            const uint32_t* ap = apack + (k0 >> 2);
            const double* bp = bvals + static_cast<int64_t>(k0 + lk) * 16 + lr;
            double bnext = bp[0];
            uint32_t wnext = ap[0];
            for (int kk = 0; kk < nk; ++kk) {
                const double bcur = bnext;
                const uint32_t w = wnext;
                if (kk + 1 < nk) {
                    bnext = bp[(kk + 1) * 64];
                    wnext = ap[kk + 1];
                }
                const int al = (w >> (8 * lk)) & 0xff;
                double av[MT];
#pragma unroll
                for (int m = 0; m < MT; ++m) av[m] = grow[m * 16 * GS + al];
#pragma unroll
                for (int m = 0; m < MT; ++m) acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[m], bcur, acc[m], 0, 0, 0);
            }
        }
        if (e >= 0) {
            // symmetric forms: the same value at the transposed entry (sym_n = element dofs)
            const int e2 = sym_n ? (e % sym_n) * sym_n + e / sym_n : e;
            if (st) {
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        st[(m * 16 + i * 4 + lk) * nI + e] = acc[m][i];
                        st[(m * 16 + i * 4 + lk) * nI + e2] = acc[m][i];
                    }
            } else {
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int64_t cell = c0 + m * 16 + i * 4 + lk;
                        if (cell < cells) {
                            out[cell * nI + e] = acc[m][i];
                            if (e2 != e) out[cell * nI + e2] = acc[m][i];
                        }
                    }
            }
        }
    }
    if (st && out) {
        __syncthreads();
        const int64_t nc = cells - c0 < CT ? cells - c0 : CT;
        write_region(st, out + c0 * nI, nc * nI);
    }
}

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
__device__ __forceinline__ void contract_tile_bf16(const double* am, const double* cf, unsigned short* Gp, float* st,
                                                   int64_t c0, int64_t cells, int nI, int n_tiles, int kpad,
                                                   const int* gpiece, const uint16_t* __restrict__ bb,
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
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int kchunks = kpad / 32;
    const unsigned short* grow = Gp + lr * KS + lk * 8;
    for (int t = wave; t < n_tiles; t += waves) {
        f4 acc[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = f4{0.f, 0.f, 0.f, 0.f};
        if (nonzero[t]) {
            const u16x8* bt = reinterpret_cast<const u16x8*>(bb) + static_cast<int64_t>(t) * (kpad / 8) * 16 + lk * 16 + lr;
            u16x8 bnext = bt[0];
            for (int kc = 0; kc < kchunks; ++kc) {
                const bf8 bv = __builtin_bit_cast(bf8, bnext);
                if (kc + 1 < kchunks) bnext = bt[(kc + 1) * 64];
                u16x8 av[MT];
#pragma unroll
                for (int m = 0; m < MT; ++m) av[m] = *reinterpret_cast<const u16x8*>(grow + m * 16 * KS + kc * 32);
#pragma unroll
                for (int m = 0; m < MT; ++m)
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, av[m]), bv, acc[m], 0, 0, 0);
            }
        }
        const int e = t * 16 + lr;
        if (e < nI) {
            if (st) {
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int i = 0; i < 4; ++i) st[(m * 16 + lk * 4 + i) * nI + e] = acc[m][i];
            } else {
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int64_t cell = c0 + m * 16 + lk * 4 + i;
                        if (cell < cells) out[cell * nI + e] = acc[m][i];
                    }
            }
        }
    }
    if (st) {
        __syncthreads();
        const int64_t nc = cells - c0 < CT ? cells - c0 : CT;
        write_region(st, out + c0 * nI, nc * nI);
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

// ------------------------------------------------------ persistent FP64 contraction ---
// Every 16-cell tile of a mesh runs the same contraction, so a persistent workgroup keeps
// it in registers: wave w owns a fixed set of the A^0 tiles (balanced by k steps on the
// host) and holds, per k step s, its B fragment breg[s] and one packed word preg[s] = LDS
// column of its alpha | (output entry of its column + 1) << 8 (the entry only at the last
// step of a tile, which bit s of the wave-uniform endmask flags).
// Per cell tile: affine map (prefetched one tile ahead in registers) -> LDS, G tile and the
// zero entries, then the MFMA chain straight from LDS and registers into the staged output
// rows, then one contiguous write of the 16 rows.

// Barrier for LDS traffic only: waits for this wave's LDS operations, then s_barrier.
// Unlike __syncthreads() it leaves global stores in flight, so the write-out of one cell
// tile overlaps the contraction of the next.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt left at their maxima
    __builtin_amdgcn_s_barrier();
}

// A cell tile of the persistent loop as the fetch and store steps see it: the mesh it
// belongs to (affine map, coefficients, output, cell count) and its index in that mesh.
struct MeshTile {
    const double* amap;
    int64_t astride;
    const double* coeffs;
    int64_t cstride;
    double* out;
    int64_t cells;
    int64_t ct;
};

// Tile source of a single-mesh launch: tile g of the sequence is tile g of the mesh.
struct OneMesh {
    const ContractArgs& A;
    __device__ __forceinline__ MeshTile at(int64_t g) const {
        return MeshTile{A.amap, A.astride, A.coeffs, A.cstride, static_cast<double*>(A.out), A.cells, g};
    }
};

// Tile source of a batch launch: the CT-cell tiles of items[0], then of items[1], ... (items
// in unit_begin order); queried with increasing g, so a cursor advances over the items.
template <int CT>
struct ItemCursor {
    const BatchItem* items;
    int n, idx;
    int64_t begin, end;
    MeshTile base;
    __device__ __forceinline__ MeshTile at(int64_t g) {
        while (g >= end && idx + 1 < n) {
            ++idx;
            const BatchItem& it = items[idx];
            begin = it.unit_begin;
            end = begin + (it.cells + CT - 1) / CT;
            base = MeshTile{as_global(it.amap), it.cells, as_global(it.coeffs), it.cells,
                            as_global(static_cast<double*>(it.out)), it.cells, 0};
        }
        MeshTile t = base;
        t.ct = g - begin;
        return t;
    }
};

// The tiles g, g + step, ... below g_end of a tile source (one mesh, or the items of a
// batch that share one form).  ACT (operator action, one mesh): the I/O waves prefetch the
// next tile's local vectors into registers, put them in LDS (two alternating buffers, so
// that one tile's products and the next tile's vectors never share one), and, once a
// tile's element tensors are staged, form y = A^K x there and store only y.
template <int D, int KIND, int KMAX, int IOS, bool ACT = false, class Src>
__device__ __forceinline__ void persistent_tiles(const ContractArgs& A, const PersistArgs& P, Src& src, int64_t ct,
                                                 const int64_t ct_end, const int64_t step, unsigned char* smem_raw) {
    using FT = FormTraits<KIND, D>;
    constexpr int CT = 16;
    constexpr int NA = FT::n_alpha;
    constexpr int NC = FT::n_coeff;
    constexpr int GS = NA | 1;
    constexpr int ROWS = 1 + D * D + NC;
    // One register file, two uses (the compiler cannot see that a wave only ever takes one
    // role, so separate arrays would both count): a compute lane keeps the B fragment of
    // step s in R[2s], R[2s+1] and its packed word in R[2*KMAX + s]; an I/O lane keeps
    // 16-byte slot j of a staged tile in R[4j .. 4j+3].
    // (the operator action keeps no staged tile in registers)
    constexpr int NR = (ACT || 3 * KMAX > 4 * IOS) ? 3 * KMAX : 4 * IOS;
    // Wave roles: the first blockDim/64 - kIoWaves waves ("compute waves") prefetch the next
    // tile's affine map and coefficients and run the MFMA steps; the last kIoWaves waves
    // move the staged output to global memory and nothing else.  On this architecture one
    // counter (vmcnt) tracks a wave's loads and stores in issue order, so a wave waiting for
    // its prefetched map would also wait for every store it issued before; keeping stores
    // out of the compute waves lets the write-out of one tile overlap the next contraction.
    double* st = reinterpret_cast<double*>(smem_raw);
    // [ROWS][AS]: map rows, then coefficients; the odd row stride AS = CT + 1 spreads the rows
    // of one cell over the LDS banks (the G build reads several rows of one cell per wave)
    constexpr int AS = CT + 1;
    double* am = reinterpret_cast<double*>(smem_raw + A.stage_bytes);
    double* cf = am + (1 + D * D) * AS;
    double* Gs = reinterpret_cast<double*>(smem_raw + A.stage_bytes + A.head_bytes);
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int nI = A.n_I;
    const int io_begin = blockDim.x - 64 * kIoWaves;
    const int io_lane = tid - io_begin;
    const int n_compute = (blockDim.x >> 6) - kIoWaves;
    const int s0 = wave < n_compute ? P.woff[wave] : 0;
    const int ns = wave < n_compute ? P.woff[wave + 1] - s0 : 0;

    uint32_t R[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) R[r] = 0;
    uint32_t endmask = 0;
    if (wave < n_compute) {
        // this wave's fragments and words, prepared per step and lane on the host:
        // independent coalesced loads, all in flight together
        const double* wb = P.wave_b + static_cast<int64_t>(wave) * KMAX * 64 + lane;
        const uint32_t* ww = P.wave_word + static_cast<int64_t>(wave) * KMAX * 64 + lane;
#pragma unroll
        for (int s = 0; s < KMAX; ++s) {
            const u32x2 bw = __builtin_bit_cast(u32x2, wb[s * 64]);
            R[2 * s] = bw[0];
            R[2 * s + 1] = bw[1];
            R[2 * KMAX + s] = ww[s * 64];
        }
        endmask = P.wave_mask[wave];
    }
    endmask = __builtin_amdgcn_readfirstlane(endmask);
    // the register-resident fragments have arrived before the tile loop starts: without this
    // the compiler, which cannot tell the loop's iterations apart, waits for every
    // outstanding vector memory operation (the affine-map prefetch included) before each
    // MFMA and each store
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)

    // thread r*CT + c (r < ROWS) fetches row r of cell c: affine map, then coefficients
    auto fetch = [&](const MeshTile& t) -> double {
        const int r = tid / CT, c = tid - (tid / CT) * CT;
        const int64_t cell = t.ct * CT + c;
        if (cell >= t.cells) return r == 0 ? 1.0 : 0.0;
        return r < 1 + D * D ? t.amap[r * t.astride + cell] : t.coeffs[(r - 1 - D * D) * t.cstride + cell];
    };
    // output run of a tile: start and length in doubles (element tensors, or y)
    const int nd = A.n_dof;
    auto out_run = [&](const MeshTile& t, double*& o, int64_t& n) {
        const int64_t c0 = t.ct * CT;
        const int64_t w = ACT ? nd : nI;
        o = t.out + c0 * w;
        n = (t.cells - c0 < CT ? t.cells - c0 : CT) * w;
    };
    // operator action: I/O lane l prefetches values l and l + 64 * kIoWaves of the tile's
    // local vectors (CT * nd <= 2 * 64 * kIoWaves doubles)
    double* xs = Gs + CT * GS;
    auto fetchx = [&](const MeshTile& t, int i) -> double {
        const int64_t g = t.ct * CT * nd + i;
        return i < CT * nd && g < t.cells * nd ? A.xloc[g] : 0.0;
    };
    double px0 = 0.0, px1 = 0.0;
    int xbuf = 0;
    double pre = 0.0;
    double* cur_out = nullptr;
    int64_t cur_n = 0;
    if (ct < ct_end) {
        const MeshTile t = src.at(ct);
        out_run(t, cur_out, cur_n);
        if (tid < ROWS * CT) pre = fetch(t);
        if (ACT && tid >= io_begin) {
            px0 = fetchx(t, io_lane);
            px1 = fetchx(t, io_lane + 64 * kIoWaves);
        }
    }
    const double* grow = Gs + lr * GS;
    double* io_out = nullptr;
    int64_t io_n = 0;
    // I/O lanes: store the tile held in R (slot j -> 16-byte pair io_lane + j * 64 * kIoWaves;
    // an odd last value rides in the last slot of lane 0, which the host keeps unused)
    auto io_store = [&]() {
        double* o = io_out;
        const int64_t nv = io_n / 2;
        const int jn = nv > io_lane ? static_cast<int>((nv - io_lane + 64 * kIoWaves - 1) / (64 * kIoWaves)) : 0;
        d2v* ov = reinterpret_cast<d2v*>(o) + io_lane;
#pragma unroll
        for (int j = 0; j < IOS; ++j) {
            if (j < jn) *ov = __builtin_bit_cast(d2v, u32x4{R[4 * j], R[4 * j + 1], R[4 * j + 2], R[4 * j + 3]});
            ov += 64 * kIoWaves;
        }
        if ((io_n & 1) && io_lane == 0)
            o[io_n - 1] = __builtin_bit_cast(double, u32x2{R[4 * (IOS - 1)], R[4 * (IOS - 1) + 1]});
    };
    for (; ct < ct_end; ct += step) {
        const bool more = ct + step < ct_end;
        double* nxt_out = nullptr;
        int64_t nxt_n = 0;
        if (tid < ROWS * CT) am[(tid / CT) * AS + tid % CT] = pre;
        if constexpr (ACT) {
            if (tid >= io_begin) {
                double* xb = xs + xbuf * CT * nd;
                if (io_lane < CT * nd) xb[io_lane] = px0;
                if (io_lane + 64 * kIoWaves < CT * nd) xb[io_lane + 64 * kIoWaves] = px1;
            }
        }
        if (more) {
            const MeshTile t = src.at(ct + step);
            out_run(t, nxt_out, nxt_n);
            if (tid < ROWS * CT) pre = fetch(t);
            if (ACT && tid >= io_begin) {
                px0 = fetchx(t, io_lane);
                px1 = fetchx(t, io_lane + 64 * kIoWaves);
            }
        }
        lds_barrier();
        for (int i = tid; i < CT * NA; i += blockDim.x) {
            const int c = i / NA, al = i - c * NA;
            Gs[c * GS + al] = g_entry<KIND, D>(am, cf, AS, c, al);
        }
        for (int i = tid; i < CT * P.n_zero && tid < io_begin; i += io_begin) {
            const int c = i / P.n_zero;
            st[c * nI + P.zero_entries[i - c * P.n_zero]] = 0.0;
        }
        lds_barrier();
        if (tid >= io_begin) {
            if (!ACT && io_n > 0) io_store();  // the previous tile, during this tile's MFMA phase
        } else {
            // compiler-only barrier (emits no instruction) on the row stride: keeps the
            // staging addresses of the steps from being precomputed outside the cell-tile
            // loop, which would cost 4 registers a step
            int nIs = nI;
            asm volatile("" : "+s"(nIs));
            d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < KMAX; ++s) {
                if (s < ns) {
                    const uint32_t word = R[2 * KMAX + s];
                    const double bv = __builtin_bit_cast(double, u32x2{R[2 * s], R[2 * s + 1]});
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(grow[word & 0xffu], bv, acc, 0, 0, 0);
                    if ((endmask >> s) & 1u) {
                        const int e = static_cast<int>((word >> 8) & 0xfffu) - 1;
                        if (e >= 0) {
#pragma unroll
                            for (int i = 0; i < 4; ++i) st[(i * 4 + lk) * nIs + e] = acc[i];
                        }
                        // symmetric forms: the transposed entry (none on the diagonal)
                        const int e2 = static_cast<int>(word >> 20) - 1;
                        if (e2 >= 0) {
#pragma unroll
                            for (int i = 0; i < 4; ++i) st[(i * 4 + lk) * nIs + e2] = acc[i];
                        }
                        acc = d4{0.0, 0.0, 0.0, 0.0};
                        // keeps the reset inside this branch (no select on every step that
                        // would wait for each MFMA's result)
                        asm volatile("" : "+v"(acc));
                    }
                }
            }
        }
        lds_barrier();
        if constexpr (ACT) {  // y = A^K x for this tile, by every wave, straight to global memory
            // lanes 2t and 2t + 1 sum the two halves of output t's dot product
            const double* xb = xs + xbuf * CT * nd;
            const int half = (nd + 1) >> 1;
            const int h = tid & 1;
            for (int t0 = 0; t0 < cur_n; t0 += blockDim.x >> 1) {
                const int t = t0 + (tid >> 1);
                double s = 0.0;
                if (t < cur_n) {
                    const int c = t / nd, i1 = t - c * nd;
                    const double* row = st + c * nI + i1 * nd;
                    const double* xc = xb + c * nd;
                    const int e = h ? nd : half;
#pragma unroll 1
                    for (int i2 = h * half; i2 < e; ++i2) s = fma(row[i2], xc[i2], s);
                }
                s += __shfl_xor(s, 1);
                if (t < cur_n && h == 0) cur_out[t] = s;
            }
            xbuf ^= 1;
        } else if (tid >= io_begin) {  // take this tile's rows into registers; st is free after the next barrier
            io_out = cur_out;
            io_n = cur_n;
            const int64_t nv = io_n / 2;
            const int jn = nv > io_lane ? static_cast<int>((nv - io_lane + 64 * kIoWaves - 1) / (64 * kIoWaves)) : 0;
            const d2v* sv = reinterpret_cast<const d2v*>(st) + io_lane;
#pragma unroll
            for (int j = 0; j < IOS; ++j) {
                if (j < jn) {
                    const u32x4 w = __builtin_bit_cast(u32x4, *sv);
                    R[4 * j] = w[0];
                    R[4 * j + 1] = w[1];
                    R[4 * j + 2] = w[2];
                    R[4 * j + 3] = w[3];
                }
                sv += 64 * kIoWaves;
            }
            if ((io_n & 1) && io_lane == 0) {
                const u32x2 w = __builtin_bit_cast(u32x2, st[io_n - 1]);
                R[4 * (IOS - 1)] = w[0];
                R[4 * (IOS - 1) + 1] = w[1];
            }
        }
        cur_out = nxt_out;
        cur_n = nxt_n;
    }
    if (!ACT && tid >= io_begin && io_n > 0) io_store();  // the last tile
}

template <int D, int KIND, int KMAX, int MAXT, int IOS, bool ACT = false>
__global__ __launch_bounds__(MAXT) void contract_f64_persistent(ContractArgs A, PersistArgs P) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    OneMesh src{A};
    persistent_tiles<D, KIND, KMAX, IOS, ACT>(A, P, src, blockIdx.x, (A.cells + 15) / 16, gridDim.x, smem_raw);
}

template <int D, int KIND, bool ACT>
static hipError_t launch_persistent_k(int kmax, int waves, int grid, size_t lds, const ContractArgs& a,
                                      const PersistArgs& p, hipStream_t s) {
    const unsigned block = 64u * waves;
    if (kmax <= 8)
        return launch_lds(contract_f64_persistent<D, KIND, 8, 1024, kIoSlots, ACT>, grid, block, lds, s, a, p);
    if (kmax <= 16)
        return launch_lds(contract_f64_persistent<D, KIND, 16, 1024, kIoSlots, ACT>, grid, block, lds, s, a, p);
    // the operator action stops at 16 register steps (past them its registers spill)
    if constexpr (ACT) return hipErrorInvalidValue;
    else return launch_lds(contract_f64_persistent<D, KIND, 24, 1024, kIoSlots, ACT>, grid, block, lds, s, a, p);
}

template <int D, bool ACT = false>
static hipError_t launch_persistent_d(int kind, int kmax, int waves, int grid, size_t lds, const ContractArgs& a,
                                      const PersistArgs& p, hipStream_t s) {
    switch (kind) {
    case K_MASS: return launch_persistent_k<D, K_MASS, ACT>(kmax, waves, grid, lds, a, p, s);
    case K_LAPLACE: return launch_persistent_k<D, K_LAPLACE, ACT>(kmax, waves, grid, lds, a, p, s);
    case K_WLAPLACE: return launch_persistent_k<D, K_WLAPLACE, ACT>(kmax, waves, grid, lds, a, p, s);
    case K_ELASTICITY: return launch_persistent_k<D, K_ELASTICITY, ACT>(kmax, waves, grid, lds, a, p, s);
    case K_PIOLA:
    case K_CURVED:
    case K_NEDELEC: return hipErrorInvalidValue;  // tile kernels only
    default: return launch_persistent_k<D, K_NS, ACT>(kmax, waves, grid, lds, a, p, s);
    }
}

hipError_t launch_contract_persistent(int dim, int kind, int kmax, int waves, int grid, ContractArgs a,
                                      const PersistArgs& p, hipStream_t stream) {
    if (a.cells <= 0) return hipSuccess;
    if (kmax > 24 || waves != 16 || (reinterpret_cast<uintptr_t>(a.out) & 15u) != 0) return hipErrorInvalidValue;
    // the staged rows of one tile must fit the I/O lanes' register slots, with lane 0's
    // last slot free for an odd tail
    const int64_t pairs = (16 * static_cast<int64_t>(a.n_I)) / 2;
    if (pairs > static_cast<int64_t>(kIoSlots) * 64 * kIoWaves - 64 * kIoWaves) return hipErrorInvalidValue;
    const LdsPlan pl = plan_lds(dim, kind, 16, a.n_I, a.n_alpha, 0, false, kLdsBudget);
    if (!pl.staged || (1 + dim * dim + n_coeff_of(dim, kind)) * 16 > 64 * (waves - kIoWaves)) return hipErrorInvalidValue;
    a.staged = 1;
    a.stage_bytes = pl.stage_bytes;
    a.head_bytes = pl.head_bytes;
    const int64_t ntiles = (a.cells + 15) / 16;
    if (grid > ntiles) grid = static_cast<int>(ntiles);
    return dim == 2 ? launch_persistent_d<2>(kind, kmax, waves, grid, pl.total, a, p, stream)
                    : launch_persistent_d<3>(kind, kmax, waves, grid, pl.total, a, p, stream);
}

hipError_t launch_apply_persistent(int dim, int kind, int kmax, int waves, int grid, ContractArgs a,
                                   const PersistArgs& p, hipStream_t stream) {
    if (a.cells <= 0) return hipSuccess;
    if (kmax > 16 || waves != 16 || !a.xloc || a.n_dof <= 0 || a.n_I != a.n_dof * a.n_dof ||
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

// ------------------------------------------------ persistent split-BF16 contraction ---
// The FP64 persistent pipeline for the split-BF16 mode, on cell tiles of CT = 16*MT cells:
// affine map one tile ahead, the G tile's BF16 pieces built in LDS (the K padding is zeroed
// once), the MFMA chain from LDS and registers into staged FP32 rows, and the write-out of a
// tile by the I/O waves during the next tile's MFMA phase.  Compute wave w (of W) owns the
// A^0 tiles w, w + W, w + 2W, ... and keeps their B fragments in registers: step s is the
// 32-wide K chunk s mod KC of its tile number s / KC (KC = kpad / 32 chunks per tile), 8 BF16
// values = 4 registers per lane; each step feeds MT MFMAs, one per 16-cell row block.

template <int MT>
struct Bf16PersistTraits {
    // 16-byte register slots per I/O lane holding one staged tile (CT rows of FP32)
    static constexpr int ios = MT == 1 ? 10 : 12;
};

template <int D, int KIND, int NSEG, int KS, int MT, class Src>
__device__ __forceinline__ void persistent_tiles_bf16(const ContractArgs& A, Src& src, int64_t ct,
                                                      const int64_t ct_end, const int64_t step,
                                                      unsigned char* smem_raw) {
    using FT = FormTraits<KIND, D>;
    constexpr int CT = 16 * MT;
    constexpr int NA = FT::n_alpha;
    constexpr int NC = FT::n_coeff;
    constexpr int ROWS = 1 + D * D + NC;
    constexpr int IOS = Bf16PersistTraits<MT>::ios;
    // one register file, two uses (as in the FP64 kernel): a compute lane keeps the B
    // fragment of step s in R[4s .. 4s+3]; an I/O lane keeps 16-byte slot j of a staged
    // tile in R[4j .. 4j+3]
    constexpr int NR = KS > IOS ? 4 * KS : 4 * IOS;
    float* st = reinterpret_cast<float*>(smem_raw);
    constexpr int AS = CT + 1;  // odd row stride of the map/coefficient rows (LDS banks)
    double* am = reinterpret_cast<double*>(smem_raw + A.stage_bytes);
    double* cf = am + (1 + D * D) * AS;
    unsigned short* Gp = reinterpret_cast<unsigned short*>(smem_raw + A.stage_bytes + A.head_bytes);
    const int kpad = A.kpad;
    const int GK = kpad + 8;  // row stride of the G pieces (BF16 values)
    const int KC = kpad / 32;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int nI = A.n_I;
    const int io_begin = blockDim.x - 64 * kIoWaves;
    const int io_lane = tid - io_begin;
    const int n_compute = (blockDim.x >> 6) - kIoWaves;
    const int my_tiles = wave < n_compute ? (A.n_tiles - wave + n_compute - 1) / n_compute : 0;
    const int ns = my_tiles * KC;

    uint32_t R[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) R[r] = 0;
    {
        int j = 0, kc = 0;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (s < ns) {
                const int t = wave + j * n_compute;
                const u32x4 bw = __builtin_bit_cast(
                    u32x4, reinterpret_cast<const u16x8*>(A.bb)[(static_cast<int64_t>(t) * (kpad / 8) + kc * 4 + lk) * 16 + lr]);
                R[4 * s] = bw[0];
                R[4 * s + 1] = bw[1];
                R[4 * s + 2] = bw[2];
                R[4 * s + 3] = bw[3];
                if (++kc == KC) kc = 0, ++j;
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): fragments in registers before the tile loop
    // K padding of the G pieces: zero once, no tile writes it
    {
        const int w = kpad - NSEG * NA;
        for (int i = tid; i < CT * w; i += blockDim.x) {
            const int c = i / w, k = NSEG * NA + (i - c * w);
            Gp[c * GK + k] = 0;
        }
    }

    // thread r*CT + c (r < ROWS) fetches row r of cell c: affine map, then coefficients
    auto fetch = [&](const MeshTile& t) -> double {
        const int r = tid / CT, c = tid - (tid / CT) * CT;
        const int64_t cell = t.ct * CT + c;
        if (cell >= t.cells) return r == 0 ? 1.0 : 0.0;
        return r < 1 + D * D ? t.amap[r * t.astride + cell] : t.coeffs[(r - 1 - D * D) * t.cstride + cell];
    };
    // output run of a tile (floats)
    auto out_run = [&](const MeshTile& t, float*& o, int64_t& n) {
        const int64_t c0 = t.ct * CT;
        o = reinterpret_cast<float*>(t.out) + c0 * nI;
        n = (t.cells - c0 < CT ? t.cells - c0 : CT) * nI;
    };
    double pre = 0.0;
    float* cur_out = nullptr;
    int64_t cur_n = 0;
    if (ct < ct_end) {
        const MeshTile t = src.at(ct);
        out_run(t, cur_out, cur_n);
        if (tid < ROWS * CT) pre = fetch(t);
    }
    const unsigned short* grow = Gp + lr * GK + lk * 8;
    float* io_out = nullptr;
    int64_t io_n = 0;
    // I/O lanes: 16-byte slot j of lane l holds floats 4 (l + j * 64 * kIoWaves) .. + 3
    auto io_store = [&]() {
        const int64_t nv = io_n / 4;
        const int jn = nv > io_lane ? static_cast<int>((nv - io_lane + 64 * kIoWaves - 1) / (64 * kIoWaves)) : 0;
        u32x4* ov = reinterpret_cast<u32x4*>(io_out) + io_lane;
#pragma unroll
        for (int j = 0; j < IOS; ++j) {
            if (j < jn) *ov = u32x4{R[4 * j], R[4 * j + 1], R[4 * j + 2], R[4 * j + 3]};
            ov += 64 * kIoWaves;
        }
    };
    for (; ct < ct_end; ct += step) {
        const bool more = ct + step < ct_end;
        float* nxt_out = nullptr;
        int64_t nxt_n = 0;
        if (tid < ROWS * CT) am[(tid / CT) * AS + tid % CT] = pre;
        if (more) {
            const MeshTile t = src.at(ct + step);
            out_run(t, nxt_out, nxt_n);
            if (tid < ROWS * CT) pre = fetch(t);
        }
        lds_barrier();
        for (int i = tid; i < CT * NA; i += blockDim.x) {
            const int c = i / NA, al = i - c * NA;
            const double gv = g_entry<KIND, D>(am, cf, AS, c, al);
            double piece[3];
            piece[0] = rn_bf16(gv);
            piece[1] = rn_bf16(gv - piece[0]);
            piece[2] = rn_bf16((gv - piece[0]) - piece[1]);
#pragma unroll
            for (int sg = 0; sg < NSEG; ++sg) Gp[c * GK + sg * NA + al] = bf16_of(piece[A.gpiece[sg]]);
        }
        lds_barrier();
        if (tid >= io_begin) {
            if (io_n > 0) io_store();  // the previous tile, during this tile's MFMA phase
        } else {
            f4 acc[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) acc[m] = f4{0.f, 0.f, 0.f, 0.f};
            int j = 0, kc = 0;
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                if (s < ns) {
                    const bf8 bv =
                        __builtin_bit_cast(bf8, u32x4{R[4 * s], R[4 * s + 1], R[4 * s + 2], R[4 * s + 3]});
                    u16x8 av[MT];
#pragma unroll
                    for (int m = 0; m < MT; ++m) av[m] = *reinterpret_cast<const u16x8*>(grow + m * 16 * GK + kc * 32);
#pragma unroll
                    for (int m = 0; m < MT; ++m)
                        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, av[m]), bv, acc[m], 0,
                                                                         0, 0);
                    if (++kc == KC) {
                        const int e = (wave + j * n_compute) * 16 + lr;
                        if (e < nI) {
#pragma unroll
                            for (int m = 0; m < MT; ++m)
#pragma unroll
                                for (int i = 0; i < 4; ++i) st[(m * 16 + lk * 4 + i) * nI + e] = acc[m][i];
                        }
#pragma unroll
                        for (int m = 0; m < MT; ++m) {
                            acc[m] = f4{0.f, 0.f, 0.f, 0.f};
                            asm volatile("" : "+v"(acc[m]));
                        }
                        kc = 0;
                        ++j;
                    }
                }
            }
        }
        lds_barrier();
        if (tid >= io_begin) {  // take this tile's rows into registers; st is free after the next barrier
            io_out = cur_out;
            io_n = cur_n;
            const int64_t nv = io_n / 4;
            const int jn = nv > io_lane ? static_cast<int>((nv - io_lane + 64 * kIoWaves - 1) / (64 * kIoWaves)) : 0;
            const u32x4* sv = reinterpret_cast<const u32x4*>(st) + io_lane;
#pragma unroll
            for (int j = 0; j < IOS; ++j) {
                if (j < jn) {
                    const u32x4 w = *sv;
                    R[4 * j] = w[0];
                    R[4 * j + 1] = w[1];
                    R[4 * j + 2] = w[2];
                    R[4 * j + 3] = w[3];
                }
                sv += 64 * kIoWaves;
            }
            // a tail of fewer than 4 floats (a last, partial cell tile): stored right away
            const int64_t tail = io_n - nv * 4;
            if (io_lane < tail) io_out[nv * 4 + io_lane] = st[nv * 4 + io_lane];
        }
        cur_out = nxt_out;
        cur_n = nxt_n;
    }
    if (tid >= io_begin && io_n > 0) io_store();  // the last tile
}

template <int D, int KIND, int NSEG, int KS, int MT>
__global__ __launch_bounds__(1024) void contract_bf16_persistent(ContractArgs A) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    OneMesh src{A};
    persistent_tiles_bf16<D, KIND, NSEG, KS, MT>(A, src, blockIdx.x, (A.cells + 16 * MT - 1) / (16 * MT), gridDim.x,
                                                smem_raw);
}

// Register budget (128 per lane at 1024 threads): at most 16 register-resident steps, and 8
// for 32-cell tiles with the 6-product split (its G build needs more registers).
int bf16_persistent_max_steps(int tile_cells, int n_seg) { return tile_cells == 32 && n_seg == 6 ? 8 : 16; }

template <int D, int KIND, int NSEG, int MT>
static hipError_t launch_bf16_persistent_m(int ks, int grid, size_t lds, const ContractArgs& a, hipStream_t s) {
    if (ks <= 8) return launch_lds(contract_bf16_persistent<D, KIND, NSEG, 8, MT>, grid, 1024u, lds, s, a);
    if constexpr (MT == 1 || NSEG == 3)
        return launch_lds(contract_bf16_persistent<D, KIND, NSEG, 16, MT>, grid, 1024u, lds, s, a);
    return hipErrorInvalidValue;
}

template <int D, int KIND, int NSEG>
static hipError_t launch_bf16_persistent_k(int mt, int ks, int grid, size_t lds, const ContractArgs& a,
                                           hipStream_t s) {
    return mt == 1 ? launch_bf16_persistent_m<D, KIND, NSEG, 1>(ks, grid, lds, a, s)
                   : launch_bf16_persistent_m<D, KIND, NSEG, 2>(ks, grid, lds, a, s);
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
    const int ios = tile_cells == 16 ? Bf16PersistTraits<1>::ios : Bf16PersistTraits<2>::ios;
    const int64_t units = (tile_cells * static_cast<int64_t>(n_I) + 3) / 4;
    const bool fits = (tile_cells == 16 || tile_cells == 32) && p.staged &&
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

// --------------------------------------------------------------- mixed batches ---
// Tile launch: workgroup u runs tile u of the launch, cell tile 16*MT of item unit_item[u]
// (one launch per tile size, so each kernel's register count is that of its own tile),
// geometry computed in place (one lane per cell), then the FP64 or split-BF16 contraction of
// the single-mesh kernel.  LDS per the item's own plan: staged rows [stage_bytes], affine
// map and coefficients [head_bytes], G tile; the launch reserves the largest item plan.


template <int D, int KIND, int MT, int NSEG>
__device__ __forceinline__ void batch_tile(const BatchItem& it, int64_t c0, unsigned char* smem) {
    constexpr int NC = FormTraits<KIND, D>::n_coeff;
    constexpr int CT = 16 * MT;
    // the item's own LDS plan: staged rows, affine map and coefficients, G tile
    double* am = reinterpret_cast<double*>(smem + it.stage_bytes);
    double* cf = am + (1 + D * D) * CT;
    unsigned char* g = smem + it.stage_bytes + it.head_bytes;
    stage_tile_from_coords<D, NC>(as_global(it.coords), as_global(it.coeffs), it.cells, c0, CT, am, cf);
    __syncthreads();
    if constexpr (NSEG > 0) {
        contract_tile_bf16<D, KIND, MT, NSEG>(am, cf, reinterpret_cast<unsigned short*>(g),
                                              it.staged ? reinterpret_cast<float*>(smem) : nullptr, c0, it.cells,
                                              it.n_I, it.n_tiles, it.kpad, it.gpiece, as_global(it.bb),
                                              as_global(it.nonzero), as_global(static_cast<float*>(it.out)));
    } else {
        contract_tile_f64<D, KIND, MT>(am, cf, reinterpret_cast<double*>(g),
                                       it.staged ? reinterpret_cast<double*>(smem) : nullptr, c0, it.cells, it.n_I,
                                       it.n_tiles, as_global(it.koff), as_global(it.apack), as_global(it.entry),
                                       as_global(it.b), as_global(static_cast<double*>(it.out)), it.sym_n);
    }
}

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

template <int D, int KIND, int KMAX>
__global__ __launch_bounds__(1024) void batch_persistent_kernel(const BatchItem* __restrict__ items, int n_items,
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
    ItemCursor<16> src{items, n_items, -1, 0, 0, MeshTile{}};
    persistent_tiles<D, KIND, KMAX, kIoSlots>(A, P, src, blockIdx.x, total_tiles, gridDim.x, smem_raw);
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
    if constexpr (MT == 1 || NSEG == 3)
        return launch_lds(batch_persistent_bf16_kernel<D, KIND, NSEG, 16, MT>, grid, 1024u, lds, s, items, n_items,
                          tiles);
    return hipErrorInvalidValue;
}

template <int D, int NSEG>
static hipError_t launch_batch_bf16_d(int kind, int mt, int ks, const BatchItem* items, int n_items, int64_t tiles,
                                      int grid, size_t lds, hipStream_t s) {
#define FFC_BATCH_BF16_KIND(K)                                                                \
    return mt == 1 ? launch_batch_bf16_m<D, K, NSEG, 1>(ks, items, n_items, tiles, grid, lds, s) \
                   : launch_batch_bf16_m<D, K, NSEG, 2>(ks, items, n_items, tiles, grid, lds, s)
    switch (kind) {
    case K_MASS: FFC_BATCH_BF16_KIND(K_MASS);
    case K_LAPLACE: FFC_BATCH_BF16_KIND(K_LAPLACE);
    case K_WLAPLACE: FFC_BATCH_BF16_KIND(K_WLAPLACE);
    case K_ELASTICITY: FFC_BATCH_BF16_KIND(K_ELASTICITY);
    default: FFC_BATCH_BF16_KIND(K_NS);
    }
#undef FFC_BATCH_BF16_KIND
}

template <int D, int KIND>
static hipError_t launch_batch_persistent_k(int kmax, const BatchItem* items, int n_items, int64_t tiles, int grid,
                                            size_t lds, hipStream_t s) {
    if (kmax <= 8)
        return launch_lds(batch_persistent_kernel<D, KIND, 8>, grid, 1024u, lds, s, items, n_items, tiles);
    if (kmax <= 16)
        return launch_lds(batch_persistent_kernel<D, KIND, 16>, grid, 1024u, lds, s, items, n_items, tiles);
    return launch_lds(batch_persistent_kernel<D, KIND, 24>, grid, 1024u, lds, s, items, n_items, tiles);
}

template <int D>
static hipError_t launch_batch_persistent_d(int kind, int kmax, const BatchItem* items, int n_items, int64_t tiles,
                                            int grid, size_t lds, hipStream_t s) {
    switch (kind) {
    case K_MASS: return launch_batch_persistent_k<D, K_MASS>(kmax, items, n_items, tiles, grid, lds, s);
    case K_LAPLACE: return launch_batch_persistent_k<D, K_LAPLACE>(kmax, items, n_items, tiles, grid, lds, s);
    case K_WLAPLACE: return launch_batch_persistent_k<D, K_WLAPLACE>(kmax, items, n_items, tiles, grid, lds, s);
    case K_ELASTICITY: return launch_batch_persistent_k<D, K_ELASTICITY>(kmax, items, n_items, tiles, grid, lds, s);
    default: return launch_batch_persistent_k<D, K_NS>(kmax, items, n_items, tiles, grid, lds, s);
    }
}

hipError_t launch_batch_persistent(int dim, int kind, int kmax, int nseg, int mt, const BatchItem* items, int n_items,
                                   int64_t tiles, int grid, size_t lds, hipStream_t stream) {
    if (tiles <= 0 || n_items <= 0) return hipSuccess;
    if (grid > tiles) grid = static_cast<int>(tiles);
    if (nseg == 3)
        return dim == 2 ? launch_batch_bf16_d<2, 3>(kind, mt, kmax, items, n_items, tiles, grid, lds, stream)
                        : launch_batch_bf16_d<3, 3>(kind, mt, kmax, items, n_items, tiles, grid, lds, stream);
    if (nseg == 6)
        return dim == 2 ? launch_batch_bf16_d<2, 6>(kind, mt, kmax, items, n_items, tiles, grid, lds, stream)
                        : launch_batch_bf16_d<3, 6>(kind, mt, kmax, items, n_items, tiles, grid, lds, stream);
    return dim == 2 ? launch_batch_persistent_d<2>(kind, kmax, items, n_items, tiles, grid, lds, stream)
                    : launch_batch_persistent_d<3>(kind, kmax, items, n_items, tiles, grid, lds, stream);
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
    // elasticity: enough cells that the 256 threads all get a 2 x 2 block of function pairs;
    // below 8 dofs (one entry per thread): enough cells for one entry per thread
    int cap = 8;
    const int n = kind == K_ELASTICITY || kind == K_NS ? dim * ns : ns;
    if (kind == K_ELASTICITY) {
        const int pairs = ((ns + 1) / 2) * ((ns + 1) / 2);
        cap = std::max(8, (256 + pairs - 1) / pairs);
    } else if (n < 8) {
        cap = std::max(8, (256 + n * n - 1) / (n * n));
    }
    if (qc > cap) qc = cap;
    if (qc < 1) qc = 1;
    return qc;
}

// Entries of the quadrature kernel: each thread takes a block of QR rows (test functions) by
// QE consecutive columns (trial functions), so each function's values at a point are read
// from LDS once for the block (mass, Laplacian, weighted Laplacian, NS convection).  slots:
// per cell |det|, g, then per point the weight, the physical gradients [point][function][D]
// and (NS) the convection term [point][function].
template <int D, int KIND, int QR, int QE>
__device__ __forceinline__ void quad_entries(const QuadArgs& A, const double* phis, const double* slots, int slot,
                                             int64_t c0) {
    const int ns = A.ns, n = A.n, nI = A.n_I, NQ = A.npts, QC = A.cells_per_block;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int rblocks = (n + QR - 1) / QR, runs = (n + QE - 1) / QE;
    for (int i = tid; i < QC * rblocks * runs; i += nthr) {
        const int c = i / (rblocks * runs), r = i - c * (rblocks * runs);
        const int rb = r / runs, j0 = (r - rb * runs) * QE, i0 = rb * QR;
        const int64_t cell = c0 + c;
        if (cell >= A.cells) continue;
        const double* geo = slots + c * slot;
        const double* W = geo + 1 + D * D;
        const double* grad = W + NQ;
        // rows and columns past n repeat the last function (computed, never stored)
        int fr[QR], fc[QE];  // scalar basis function of each row / column
        int cr[QR], cc[QE];  // vector component (vector forms)
#pragma unroll
        for (int a = 0; a < QR; ++a) {
            const int i1 = i0 + a < n ? i0 + a : n - 1;
            cr[a] = i1 / ns;
            fr[a] = i1 - cr[a] * ns;
        }
#pragma unroll
        for (int j = 0; j < QE; ++j) {
            const int i2 = j0 + j < n ? j0 + j : n - 1;
            cc[j] = i2 / ns;
            fc[j] = i2 - cc[j] * ns;
        }
        double acc[QR][QE];
#pragma unroll
        for (int a = 0; a < QR; ++a)
#pragma unroll
            for (int j = 0; j < QE; ++j) acc[a][j] = 0.0;
        for (int q = 0; q < NQ; ++q) {
            const double wq = W[q];
            if constexpr (KIND == K_MASS || KIND == K_NS) {
                const double* conv = grad + NQ * ns * D;  // NS: (w . grad) phi at the points
                double rv[QR], cv[QE];
#pragma unroll
                for (int a = 0; a < QR; ++a) rv[a] = wq * phis[q * ns + fr[a]];
#pragma unroll
                for (int j = 0; j < QE; ++j) cv[j] = KIND == K_MASS ? phis[q * ns + fc[j]] : conv[q * ns + fc[j]];
#pragma unroll
                for (int a = 0; a < QR; ++a)
#pragma unroll
                    for (int j = 0; j < QE; ++j)
                        if (KIND == K_MASS || cr[a] == cc[j]) acc[a][j] += rv[a] * cv[j];
            } else {
                double rv[QR][D], cv[QE][D];
#pragma unroll
                for (int a = 0; a < QR; ++a)
#pragma unroll
                    for (int k = 0; k < D; ++k) rv[a][k] = grad[(q * ns + fr[a]) * D + k];
#pragma unroll
                for (int j = 0; j < QE; ++j)
#pragma unroll
                    for (int k = 0; k < D; ++k) cv[j][k] = grad[(q * ns + fc[j]) * D + k];
#pragma unroll
                for (int a = 0; a < QR; ++a) {
#pragma unroll
                    for (int j = 0; j < QE; ++j) {
                        double dot = 0.0;
#pragma unroll
                        for (int k = 0; k < D; ++k) dot += rv[a][k] * cv[j][k];
                        acc[a][j] += wq * dot;
                    }
                }
            }
        }
#pragma unroll
        for (int a = 0; a < QR; ++a) {
            if (i0 + a >= n) break;
            double* o = A.out + cell * nI + (i0 + a) * n + j0;
#pragma unroll
            for (int j = 0; j < QE; ++j)
                if (j0 + j < n) o[j] = acc[a][j];
        }
    }
}

// Elasticity entries: a thread takes ER x EC pairs of scalar functions (s1, s2) and forms all
// D x D component pairs of each from one table of products of their gradients.
template <int D>
__device__ __forceinline__ void quad_entries_elasticity(const QuadArgs& A, const double* slots, int slot,
                                                        int64_t c0) {
    constexpr int ER = 2, EC = 2;
    const int ns = A.ns, n = A.n, nI = A.n_I, NQ = A.npts, QC = A.cells_per_block;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int sb = (ns + ER - 1) / ER, sr = (ns + EC - 1) / EC;
    const double mu = A.mu, lam = A.lambda;
    for (int i = tid; i < QC * sb * sr; i += nthr) {
        const int c = i / (sb * sr), r = i - c * (sb * sr);
        const int s10 = (r / sr) * ER, s20 = (r - (r / sr) * sr) * EC;
        const int64_t cell = c0 + c;
        if (cell >= A.cells) continue;
        const double* geo = slots + c * slot;
        const double* W = geo + 1 + D * D;
        const double* grad = W + NQ;
        int f1[ER], f2[EC];  // functions past ns repeat the last one (computed, never stored)
#pragma unroll
        for (int a = 0; a < ER; ++a) f1[a] = s10 + a < ns ? s10 + a : ns - 1;
#pragma unroll
        for (int b = 0; b < EC; ++b) f2[b] = s20 + b < ns ? s20 + b : ns - 1;
        double acc[ER][EC][D][D];
#pragma unroll
        for (int a = 0; a < ER; ++a)
#pragma unroll
            for (int b = 0; b < EC; ++b)
#pragma unroll
                for (int k = 0; k < D; ++k)
#pragma unroll
                    for (int l = 0; l < D; ++l) acc[a][b][k][l] = 0.0;
        for (int q = 0; q < NQ; ++q) {
            const double wq = W[q];
            double g1[ER][D], g2[EC][D];
#pragma unroll
            for (int a = 0; a < ER; ++a)
#pragma unroll
                for (int k = 0; k < D; ++k) g1[a][k] = grad[(q * ns + f1[a]) * D + k];
#pragma unroll
            for (int b = 0; b < EC; ++b)
#pragma unroll
                for (int k = 0; k < D; ++k) g2[b][k] = grad[(q * ns + f2[b]) * D + k];
#pragma unroll
            for (int a = 0; a < ER; ++a) {
#pragma unroll
                for (int b = 0; b < EC; ++b) {
                    double P[D][D];  // P[k][l] = d phi_s1 / dx_k * d phi_s2 / dx_l
                    double dot = 0.0;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
#pragma unroll
                        for (int l = 0; l < D; ++l) P[k][l] = g1[a][k] * g2[b][l];
                        dot += P[k][k];
                    }
                    // entry ((c1, s1), (c2, s2)): mu d_c2 phi_s1 d_c1 phi_s2 + lambda d_c1 phi_s1
                    // d_c2 phi_s2, plus mu grad phi_s1 . grad phi_s2 when c1 = c2
#pragma unroll
                    for (int c1 = 0; c1 < D; ++c1)
#pragma unroll
                        for (int c2 = 0; c2 < D; ++c2) {
                            double v = mu * P[c2][c1] + lam * P[c1][c2];
                            if (c1 == c2) v += mu * dot;
                            acc[a][b][c1][c2] += wq * v;
                        }
                }
            }
        }
#pragma unroll
        for (int a = 0; a < ER; ++a) {
            if (s10 + a >= ns) break;
#pragma unroll
            for (int c1 = 0; c1 < D; ++c1) {
                double* o = A.out + cell * nI + static_cast<int64_t>(c1 * ns + s10 + a) * n;
#pragma unroll
                for (int c2 = 0; c2 < D; ++c2)
#pragma unroll
                    for (int b = 0; b < EC; ++b)
                        if (s20 + b < ns) o[c2 * ns + s20 + b] = acc[a][b][c1][c2];
            }
        }
    }
}

template <int D, int KIND>
__global__ __launch_bounds__(256) void quadrature_kernel(QuadArgs A) {
    extern __shared__ double smem[];
    const int ns = A.ns, n = A.n, NQ = A.npts, QC = A.cells_per_block;
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
    // entry blocks, shapes measured on P2-P4 meshes: 2 x 4 for the gradient forms (their
    // per-cell gradient tables leave few cells per block, so smaller blocks keep more lanes
    // busy), 4 x 4 for mass and convection, one entry per thread below 8 dofs
    if constexpr (KIND == K_ELASTICITY) quad_entries_elasticity<D>(A, slots, slot, c0);
    else if (n < 8) quad_entries<D, KIND, 1, 1>(A, phis, slots, slot, c0);
    else if constexpr (KIND == K_LAPLACE || KIND == K_WLAPLACE) quad_entries<D, KIND, 2, 4>(A, phis, slots, slot, c0);
    else quad_entries<D, KIND, 4, 4>(A, phis, slots, slot, c0);
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
    if (kind == K_PIOLA || kind == K_CURVED || kind == K_NEDELEC) return hipErrorInvalidValue;  // affine Lagrange forms only
    return dim == 2 ? launch_quad_d<2>(kind, a, stream) : launch_quad_d<3>(kind, a, stream);
}

}  // namespace ffc
