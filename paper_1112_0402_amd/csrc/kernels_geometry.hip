// Geometry kernels: the affine map (one lane per cell) and, for curvilinear cells, G at the points.
#include "kernels_device.h"

namespace ffc {

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

// Validation of the affine maps, off the hot path: cell c is degenerate when |det J| <=
// tol * h^D, h its longest edge (scale-free: the ratio is the cell's volume against that of a
// cube on its longest edge), or when det J is not finite.  out[0] counts degenerate cells,
// out[1] holds the smallest degenerate index: per wave a ballot, then one lane (the first
// degenerate one) updates both with global atomics.
template <int D>
__global__ __launch_bounds__(256) void degenerate_cells_kernel(int64_t cells, const double* __restrict__ coords,
                                                              double tol, unsigned long long* __restrict__ out) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    bool bad = false;
    if (c < cells) {
        double x[D + 1][D];
#pragma unroll
        for (int v = 0; v <= D; ++v)
#pragma unroll
            for (int k = 0; k < D; ++k) x[v][k] = coords[(v * D + k) * cells + c];
        double det, g[D][D];
        affine_map<D>(x, det, g);
        double h2 = 0.0;
#pragma unroll
        for (int v = 0; v <= D; ++v)
#pragma unroll
            for (int w = v + 1; w <= D; ++w) {
                double e2 = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k) e2 = fma(x[w][k] - x[v][k], x[w][k] - x[v][k], e2);
                h2 = fmax(h2, e2);
            }
        const double h = sqrt(h2);
        double bound = tol;
#pragma unroll
        for (int k = 0; k < D; ++k) bound *= h;
        bad = !(fabs(det) > bound);  // also true for a NaN det
    }
    const unsigned long long m = __ballot(bad);
    if (m != 0ull && static_cast<int>(threadIdx.x & 63u) == __builtin_ctzll(m)) {
        atomicAdd(&out[0], static_cast<unsigned long long>(__popcll(m)));
        atomicMin(&out[1], static_cast<unsigned long long>(c));
    }
}

__global__ void degenerate_init_kernel(unsigned long long* out) {
    out[0] = 0ull;
    out[1] = ~0ull;
}

hipError_t launch_degenerate_cells(int dim, int64_t cells, const double* coords, double tol, unsigned long long* out,
                                   hipStream_t stream) {
    degenerate_init_kernel<<<1, 1, 0, stream>>>(out);
    if (cells > 0) {
        const unsigned grid = static_cast<unsigned>((cells + 255) / 256);
        if (dim == 2)
            degenerate_cells_kernel<2><<<grid, 256, 0, stream>>>(cells, coords, tol, out);
        else
            degenerate_cells_kernel<3><<<grid, 256, 0, stream>>>(cells, coords, tol, out);
    }
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

}  // namespace ffc
