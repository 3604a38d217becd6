// The quadrature comparison kernel.
#include "kernels_device.h"

namespace ffc {

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
