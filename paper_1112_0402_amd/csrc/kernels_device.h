// Device code shared by the kernel translation units (kernels_*.hip): the geometry, the
// G_K build, the tile contractions and the persistent pipelines, as inline templates.
//
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
//  contract_*_persistent  one workgroup per CU (12 or 16 waves) walking cell tiles: each compute
//                      wave keeps its share of the A^0 tiles in registers, dedicated I/O
//                      waves write the staged rows of one tile during the next tile's MFMA
//                      steps (also the operator action y_K = A^K x_K, and mixed batches)
//  curved_geometry_kernel  cells with P2 geometry: |det J| g g^T at every quadrature point
//                      (Sec. 3.4: the integral becomes a sum over points, still a contraction)
//  quadrature_kernel   the quadrature comparison (Sec. 4.3 / Sec. 6): per cell, physical
//                      basis gradients at the points of a collapsed Gauss-Jacobi rule, then
//                      every entry summed over the points, register-blocked over entries
#pragma once

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
// Regions of 32 KB and more are written with non-temporal stores (streamed to HBM without
// allocating in the caches): measured on MI355X 20% faster for 16-cell tiles of large
// tensors (Laplacian P4 on tetrahedra, convection P2 in split x6), ~5% slower for the small
// regions of tiny tensors, which keep ordinary stores.
template <typename T>
__device__ __forceinline__ void write_region(const T* __restrict__ st, T* __restrict__ out, int64_t n) {
    constexpr int V = 16 / sizeof(T);
    typedef T vec __attribute__((ext_vector_type(V)));
    const int64_t nv = n / V;
    const vec* s = reinterpret_cast<const vec*>(st);
    vec* o = reinterpret_cast<vec*>(out);
    if (n * static_cast<int64_t>(sizeof(T)) >= 32768) {
        for (int64_t i = threadIdx.x; i < nv; i += blockDim.x) __builtin_nontemporal_store(s[i], &o[i]);
    } else {
        for (int64_t i = threadIdx.x; i < nv; i += blockDim.x) o[i] = s[i];
    }
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
    const double* coords;  // SoA [(d+1)*d][cells] (kernels that compute the affine map)
};

// Tile source of a single-mesh launch: tile g of the sequence is tile g of the mesh.
struct OneMesh {
    const ContractArgs& A;
    __device__ __forceinline__ MeshTile at(int64_t g) const {
        return MeshTile{A.amap, A.astride, A.coeffs, A.cstride, static_cast<double*>(A.out), A.cells, g, A.coords};
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
    // the item's fields go to scalar registers: kept in vector registers, the compiler
    // reloaded them from the item array at every tile, and the wait for that load made the
    // I/O waves wait for their own stores once per tile
    static __device__ __forceinline__ int64_t uniform(int64_t v) {
        const uint64_t u = static_cast<uint64_t>(v);
        const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
        const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
        return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
    }
    template <class T>
    static __device__ __forceinline__ T* uniform_ptr(T* p) {
        return as_global(reinterpret_cast<T*>(uniform(static_cast<int64_t>(reinterpret_cast<uintptr_t>(p)))));
    }
    __device__ __forceinline__ MeshTile at(int64_t g) {
        while (g >= end && idx + 1 < n) {
            ++idx;
            const BatchItem& it = items[idx];
            begin = uniform(it.unit_begin);
            const int64_t cells = uniform(it.cells);
            end = begin + (cells + CT - 1) / CT;
            base = MeshTile{uniform_ptr(it.amap), cells, uniform_ptr(it.coeffs), cells,
                            uniform_ptr(static_cast<double*>(it.out)), cells, 0, uniform_ptr(it.coords)};
        }
        MeshTile t = base;
        t.ct = g - begin;
        return t;
    }
};

// Affine map of cell c of a tile from its coordinates staged in LDS (xs: [(D+1)*D][AS],
// row v*D + k = coordinate k of vertex v) into am ([1 + D*D][AS]: det J, then g_ab).
template <int D>
__device__ __forceinline__ void tile_affine_map(const double* xs, int AS, int c, double* am) {
    double J[D][D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double x0 = xs[k * AS + c];
#pragma unroll
        for (int b = 0; b < D; ++b) J[k][b] = xs[((b + 1) * D + k) * AS + c] - x0;
    }
    double det, g[D][D];
    invert_jacobian<D>(J, det, g);
    am[c] = det;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) am[(1 + a * D + b) * AS + c] = g[a][b];
}

// Coordinate (v, k) of a cell past the end of a mesh: the reference simplex (J = I), so the
// padding rows of a last, partial tile stay finite.
__device__ __forceinline__ double reference_vertex(int v, int k) { return v == k + 1 ? 1.0 : 0.0; }

// The tiles g, g + step, ... below g_end of a tile source (one mesh, or the items of a
// batch that share one form).  ACT (operator action, one mesh): the I/O waves prefetch the
// next tile's local vectors into registers, put them in LDS (two alternating buffers, so
// that one tile's products and the next tile's vectors never share one), and, once a
// tile's element tensors are staged, form y = A^K x there and store only y.  GEO: the
// affine map is computed here from the coordinates (no geometry pass, no affine-map round
// trip through HBM): coordinates are prefetched two tiles ahead, staged in LDS at the top of
// the next iteration, and turned into the following tile's map by the last compute wave
// after its MFMA steps -- while the I/O waves store -- into the second of two map blocks.
// MT: cell tiles of 16*MT cells (MT row blocks of the MFMA per register-resident B fragment),
// for element tensors small enough that a 16-cell tile would carry too little output per
// pass of the pipeline.
template <int D, int KIND, int KMAX, int IOS, bool ACT = false, bool GEO = false, int MT = 1, class Src>
__device__ __forceinline__ void persistent_tiles(const ContractArgs& A, const PersistArgs& P, Src& src, int64_t ct,
                                                 const int64_t ct_end, const int64_t step, unsigned char* smem_raw) {
    using FT = FormTraits<KIND, D>;
    constexpr int CT = 16 * MT;
    static_assert(!(ACT && MT > 1), "the operator action runs 16-cell tiles");
    constexpr int NA = FT::n_alpha;
    constexpr int NC = FT::n_coeff;
    constexpr int GS = NA | 1;
    constexpr int ROWS = 1 + D * D + NC;
    constexpr int XR = (D + 1) * D;  // coordinate rows (GEO)
    static_assert(!(ACT && GEO), "the operator action reads a precomputed affine map");
    // values each fetching thread prefetches per tile (at least 6 compute waves fetch)
    constexpr int FROWS = GEO ? NC + XR : ROWS;
    constexpr int FR = (FROWS * CT + 383) / 384;
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
    // of one cell over the LDS banks (the G build reads several rows of one cell per wave).
    // GEO: map rows of the current tile, map rows of the next tile, coefficients, then the
    // coordinate rows [XR][AS] of the next tile.
    constexpr int AS = CT + 1;
    double* am = reinterpret_cast<double*>(smem_raw + A.stage_bytes);
    double* am_next = GEO ? am + (1 + D * D) * AS : am;
    double* cf = am_next + (1 + D * D) * AS;
    double* xc = cf + NC * AS;
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

    // value i = r*CT + c (r < ROWS) of a tile is row r of cell c: affine map, then
    // coefficients; GEO: values [0, NC*CT) are coefficient rows, [NC*CT, (NC+XR)*CT) coordinate
    // rows.  Thread tid fetches values tid + f * (64 * compute waves), f < FR (compute waves
    // only: they never store)
    const int nft = 64 * n_compute;
    auto fetch_i = [&](const MeshTile& t, int i) -> double {
        const int r = i / CT, c = i - (i / CT) * CT;
        const int64_t cell = t.ct * CT + c;
        if constexpr (GEO) {
            if (r < NC) return cell < t.cells ? t.coeffs[r * t.cstride + cell] : 0.0;
            const int rx = r - NC;
            return cell < t.cells ? t.coords[rx * t.cells + cell] : reference_vertex(rx / D, rx - (rx / D) * D);
        }
        if (cell >= t.cells) return r == 0 ? 1.0 : 0.0;
        return r < 1 + D * D ? t.amap[r * t.astride + cell] : t.coeffs[(r - 1 - D * D) * t.cstride + cell];
    };
    auto fidx = [&](int f) { return tid + f * nft; };
    auto is_coef = [&](int i) { return tid < io_begin && i < NC * CT; };
    auto is_coord = [&](int i) { return GEO && tid < io_begin && i >= NC * CT && i < (NC + XR) * CT; };
    auto is_row = [&](int i) { return tid < io_begin && i < ROWS * CT; };
    Src srcx = src;  // GEO: a cursor for the coordinates, which run one tile ahead
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
    double pre[FR];
#pragma unroll
    for (int f = 0; f < FR; ++f) pre[f] = 0.0;
    double* cur_out = nullptr;
    int64_t cur_n = 0;
    if (ct < ct_end) {
        const MeshTile t = src.at(ct);
        out_run(t, cur_out, cur_n);
        if constexpr (GEO) {
            // the first tile's map, built before the loop; the second tile's coordinates in flight
            const MeshTile tx = srcx.at(ct);
#pragma unroll
            for (int f = 0; f < FR; ++f) {
                const int i = fidx(f);
                if (is_coef(i)) pre[f] = fetch_i(t, i);
                if (is_coord(i)) {
                    const int k = i - NC * CT;
                    xc[(k / CT) * AS + k % CT] = fetch_i(tx, i);
                }
            }
            __syncthreads();
            if (tid < CT) tile_affine_map<D>(xc, AS, tid, am);
            if (ct + step < ct_end) {
                const MeshTile tx1 = srcx.at(ct + step);
#pragma unroll
                for (int f = 0; f < FR; ++f)
                    if (is_coord(fidx(f))) pre[f] = fetch_i(tx1, fidx(f));
            }
            __syncthreads();
        } else {
#pragma unroll
            for (int f = 0; f < FR; ++f)
                if (is_row(fidx(f))) pre[f] = fetch_i(t, fidx(f));
        }
        if (ACT && tid >= io_begin) {
            px0 = fetchx(t, io_lane);
            px1 = fetchx(t, io_lane + 64 * kIoWaves);
        }
    }
    const double* grow = Gs + lr * GS;
    double* io_out = nullptr;
    int64_t io_n = 0;
    // I/O lanes: store the tile held in R (slot j -> 16-byte pair io_lane + j * 64 * kIoWaves;
    // an odd last value rides in the last slot of lane 0, which the host keeps unused), with
    // non-temporal stores (measured on MI355X: 7-20% faster for the mid-size tensors, neutral
    // for elasticity P2)
    auto io_store = [&]() {
        double* o = io_out;
        const int64_t nv = io_n / 2;
        const int jn = nv > io_lane ? static_cast<int>((nv - io_lane + 64 * kIoWaves - 1) / (64 * kIoWaves)) : 0;
        d2v* ov = reinterpret_cast<d2v*>(o) + io_lane;
#pragma unroll
        for (int j = 0; j < IOS; ++j) {
            if (j < jn)
                __builtin_nontemporal_store(__builtin_bit_cast(d2v, u32x4{R[4 * j], R[4 * j + 1], R[4 * j + 2], R[4 * j + 3]}),
                                            ov);
            ov += 64 * kIoWaves;
        }
        if ((io_n & 1) && io_lane == 0)
            o[io_n - 1] = __builtin_bit_cast(double, u32x2{R[4 * (IOS - 1)], R[4 * (IOS - 1) + 1]});
    };
    // the staged entries no step writes (zero A^0 rows) stay zero from tile to tile: nothing
    // else is ever written there
    for (int i = tid; i < CT * P.n_zero && tid < io_begin; i += io_begin) {
        const int c = i / P.n_zero;
        st[c * nI + P.zero_entries[i - c * P.n_zero]] = 0.0;
    }
    // The fetching below sits in a branch on the wave (uniform): a wait for the previous
    // prefetch that the compiler places in code every wave runs would make the I/O waves wait
    // for their stores, i.e. for the write-out of the previous tile to reach memory, once per
    // tile.
    const bool fetcher = wave < n_compute;
    for (; ct < ct_end; ct += step) {
        const bool more = ct + step < ct_end;
        double* nxt_out = nullptr;
        int64_t nxt_n = 0;
        MeshTile tn{};
        if (more) {
            tn = src.at(ct + step);
            out_run(tn, nxt_out, nxt_n);
        }
        if (fetcher) {
#pragma unroll
            for (int f = 0; f < FR; ++f) {
                const int i = fidx(f);
                if constexpr (GEO) {
                    // this tile's coefficients, the next tile's coordinates
                    if (is_coef(i)) cf[(i / CT) * AS + i % CT] = pre[f];
                    if (is_coord(i)) {
                        const int k = i - NC * CT;
                        xc[(k / CT) * AS + k % CT] = pre[f];
                    }
                } else {
                    if (is_row(i)) am[(i / CT) * AS + i % CT] = pre[f];
                }
            }
            if (more) {
#pragma unroll
                for (int f = 0; f < FR; ++f) {
                    const int i = fidx(f);
                    if (GEO ? is_coef(i) : is_row(i)) pre[f] = fetch_i(tn, i);
                }
            }
            if constexpr (GEO) {
                if (ct + 2 * step < ct_end) {
                    const MeshTile tx = srcx.at(ct + 2 * step);
#pragma unroll
                    for (int f = 0; f < FR; ++f)
                        if (is_coord(fidx(f))) pre[f] = fetch_i(tx, fidx(f));
                }
            }
        }
        if constexpr (ACT) {
            if (tid >= io_begin) {
                double* xb = xs + xbuf * CT * nd;
                if (io_lane < CT * nd) xb[io_lane] = px0;
                if (io_lane + 64 * kIoWaves < CT * nd) xb[io_lane + 64 * kIoWaves] = px1;
                if (more) {
                    px0 = fetchx(tn, io_lane);
                    px1 = fetchx(tn, io_lane + 64 * kIoWaves);
                }
            }
        }
        lds_barrier();
        for (int i = tid; i < CT * NA; i += blockDim.x) {
            const int c = i / NA, al = i - c * NA;
            Gs[c * GS + al] = g_entry<KIND, D>(am, cf, AS, c, al);
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
            d4 acc[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) acc[m] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < KMAX; ++s) {
                if (s < ns) {
                    const uint32_t word = R[2 * KMAX + s];
                    const double bv = __builtin_bit_cast(double, u32x2{R[2 * s], R[2 * s + 1]});
                    double av[MT];
#pragma unroll
                    for (int m = 0; m < MT; ++m) av[m] = grow[m * 16 * GS + (word & 0xffu)];
#pragma unroll
                    for (int m = 0; m < MT; ++m)
                        acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[m], bv, acc[m], 0, 0, 0);
                    if ((endmask >> s) & 1u) {
                        const int e = static_cast<int>((word >> 8) & 0xfffu) - 1;
                        if (e >= 0) {
#pragma unroll
                            for (int m = 0; m < MT; ++m)
#pragma unroll
                                for (int i = 0; i < 4; ++i) st[(m * 16 + i * 4 + lk) * nIs + e] = acc[m][i];
                        }
                        // symmetric forms: the transposed entry (none on the diagonal)
                        const int e2 = static_cast<int>(word >> 20) - 1;
                        if (e2 >= 0) {
#pragma unroll
                            for (int m = 0; m < MT; ++m)
#pragma unroll
                                for (int i = 0; i < 4; ++i) st[(m * 16 + i * 4 + lk) * nIs + e2] = acc[m][i];
                        }
#pragma unroll
                        for (int m = 0; m < MT; ++m) {
                            acc[m] = d4{0.0, 0.0, 0.0, 0.0};
                            // keeps the reset inside this branch (no select on every step that
                            // would wait for each MFMA's result)
                            asm volatile("" : "+v"(acc[m]));
                        }
                    }
                }
            }
            if constexpr (GEO) {
                // the next tile's affine map from the coordinates staged at the top of this
                // iteration, while the I/O waves store
                if (wave == n_compute - 1 && lane < CT && more) tile_affine_map<D>(xc, AS, lane, am_next);
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
        if constexpr (GEO) {
            double* t = am;
            am = am_next;
            am_next = t;
        }
    }
    if (!ACT && tid >= io_begin && io_n > 0) io_store();  // the last tile
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
    static constexpr int ios = MT == 1 ? 10 : MT == 2 ? 12 : 17;
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
            if (j < jn) __builtin_nontemporal_store(u32x4{R[4 * j], R[4 * j + 1], R[4 * j + 2], R[4 * j + 3]}, ov);
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
            // compiler-only barrier (emits no instruction) on the row stride: keeps the staging
            // addresses of the result rows from being precomputed outside the cell-tile loop,
            // where they would hold registers across it (and spill with 32-cell tiles)
            int nIs = nI;
            asm volatile("" : "+s"(nIs));
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
                        if (e < nIs) {
#pragma unroll
                            for (int m = 0; m < MT; ++m)
#pragma unroll
                                for (int i = 0; i < 4; ++i) st[(m * 16 + lk * 4 + i) * nIs + e] = acc[m][i];
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

}  // namespace ffc
