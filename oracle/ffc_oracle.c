/*
 * Element-tensor oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark load
 * this library.  The product path never calls it, links it or reads its tables.
 *
 * What it computes: the element tensor of a bilinear form on one affine simplex K,
 *     A^K_{i1 i2} = a_K(phi_{i1}, phi_{i2}) = int_K integrand(v = phi_{i1}, u = phi_{i2}) dx
 * (element matrix, Sec. 2.2 "Assembly"; element tensor of a multilinear form, Sec. 3.1),
 * evaluated straight from that definition on the physical cell: the integral is pulled
 * back to the reference simplex by the affine map F_K(X) = x^0 + J X (Sec. 3.2 and the
 * affine-map figure), physical gradients are grad phi = J^{-T} grad Phi, and the
 * pulled-back integrand is integrated by a product Gauss-Legendre rule in collapsed
 * (Duffy) coordinates with enough points to be exact for the integrand's degree.
 * Nothing here uses the tensor representation A^0 : G_K; that is what it checks.
 *
 * Conventions (written out here, shared with the product only as a written convention):
 *  - reference simplex K0: vertex 0 at the origin, vertex k at the k-th unit vector
 *    (Sec. 3.2, affine-map figure, for d = 2; the same pattern for d = 3);
 *  - Lagrange P_q nodes at the equispaced points (barycentric multi-index a / q), basis by
 *    the barycentric product formula (nodes given by point evaluation, Sec. 5.3);
 *  - dof order: vertices; then edges (triangle: edge k opposite vertex k; tetrahedron:
 *    (2,3),(1,3),(1,2),(0,3),(0,2),(0,1)), points running from the lower to the higher
 *    vertex; then faces (tetrahedron, face k opposite vertex k); then the interior.
 *    Inside an edge/face/interior with sorted vertices s_0<...<s_m, points are ordered
 *    lexicographically ascending in (b_1, ..., b_m), b_j = barycentric index of s_j;
 *  - vector elements are component-blocked: dof (c, s) -> c * n_scalar + s;
 *  - output row = test function v (first argument), column = trial function u;
 *    out[cell * n * n + i1 * n + i2];
 *  - the determinant enters as |det J| (the paper writes det F'_K for a positively
 *    oriented map).
 *
 * Forms (integrands, v = test, u = trial):
 *  0 mass        v u                                  (test case 1, eq. mass)
 *  1 laplace     grad v . grad u                      (test case 2, eq. poisson)
 *  2 wlaplace    w grad v . grad u,  w in P1          (variable-coefficient diffusion, Sec. 3.1)
 *  3 elasticity  sigma(u) : eps(v), sigma = 2 mu eps + lambda tr(eps) I, vector P_q
 *                (test case 4 generalised from the strain-strain term)
 *  4 ns          v . ((w . grad) u), u, v vector P_q, w vector P1   (test case 3, eq. navierstokes)
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAX_NODES 64 /* scalar P4 on a tetrahedron has 35 nodes */
#define OR_MAX_QP 4096

enum { OR_MASS = 0, OR_LAPLACE = 1, OR_WLAPLACE = 2, OR_ELASTICITY = 3, OR_NS = 4 };

/* ------------------------------------------------------------------ nodes ---- */

/* Append the points strictly inside the sub-simplex with sorted vertices s[0..m] to
 * nodes (barycentric multi-indices of length d+1), lexicographically ascending in
 * (b_1, ..., b_m); b_0 = q - sum.  Returns the new count. */
static int interior_points(int d, int q, const int* s, int m, int (*nodes)[4], int count) {
    int b[4];
    /* odometer over (b_1, ..., b_m) in [1, q-1]^m with b_m fastest, i.e. ascending
     * lexicographic order with b_1 most significant; points with b_0 < 1 are skipped */
    for (int j = 1; j <= m; ++j) b[j] = 1;
    for (;;) {
        int sum = 0;
        for (int j = 1; j <= m; ++j) sum += b[j];
        int b0 = q - sum;
        if (b0 >= 1) {
            for (int v = 0; v <= d; ++v) nodes[count][v] = 0;
            nodes[count][s[0]] = b0;
            for (int j = 1; j <= m; ++j) nodes[count][s[j]] = b[j];
            ++count;
        }
        int j = m;
        while (j >= 1) {
            if (b[j] < q - 1) { b[j]++; break; }
            b[j] = 1;
            --j;
        }
        if (j < 1) break;
    }
    return count;
}

static int lagrange_nodes(int d, int q, int (*nodes)[4]) {
    int count = 0;
    if (q == 0) { /* not used by the forms here */
        return 0;
    }
    for (int v = 0; v <= d; ++v) {
        for (int u = 0; u <= d; ++u) nodes[count][u] = 0;
        nodes[count][v] = q;
        ++count;
    }
    if (d == 2) {
        static const int edges[3][2] = {{1, 2}, {0, 2}, {0, 1}};
        for (int e = 0; e < 3; ++e) count = interior_points(d, q, edges[e], 1, nodes, count);
        static const int cell[3] = {0, 1, 2};
        count = interior_points(d, q, cell, 2, nodes, count);
    } else {
        static const int edges[6][2] = {{2, 3}, {1, 3}, {1, 2}, {0, 3}, {0, 2}, {0, 1}};
        for (int e = 0; e < 6; ++e) count = interior_points(d, q, edges[e], 1, nodes, count);
        static const int faces[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
        for (int f = 0; f < 4; ++f) count = interior_points(d, q, faces[f], 2, nodes, count);
        static const int cell[4] = {0, 1, 2, 3};
        count = interior_points(d, q, cell, 3, nodes, count);
    }
    return count;
}

/* f_m(t) = prod_{k<m} (q t - k)/(k+1) and its derivative. */
static void silvester_factor(int q, int m, double t, double* f, double* df) {
    double val = 1.0, der = 0.0;
    for (int k = 0; k < m; ++k) {
        double factor = (q * t - k) / (k + 1);
        double dfactor = (double)q / (k + 1);
        der = der * factor + val * dfactor;
        val = val * factor;
    }
    *f = val;
    *df = der;
}

/* Values and reference gradients (d/dX_b, b < d) of all scalar basis functions at the
 * reference point X. */
static void eval_basis(int d, int q, int nn, const int (*nodes)[4], const double* X,
                       double* phi, double* dphi /* [nn][d] */) {
    double lam[4];
    lam[0] = 1.0;
    for (int b = 0; b < d; ++b) {
        lam[b + 1] = X[b];
        lam[0] -= X[b];
    }
    for (int i = 0; i < nn; ++i) {
        double f[4], df[4];
        for (int v = 0; v <= d; ++v) silvester_factor(q, nodes[i][v], lam[v], &f[v], &df[v]);
        double dl[4];
        double val = 1.0;
        for (int v = 0; v <= d; ++v) val *= f[v];
        for (int v = 0; v <= d; ++v) {
            double p = df[v];
            for (int u = 0; u <= d; ++u)
                if (u != v) p *= f[u];
            dl[v] = p;
        }
        phi[i] = val;
        for (int b = 0; b < d; ++b) dphi[i * d + b] = dl[b + 1] - dl[0];
    }
}

/* ------------------------------------------------------------- quadrature ---- */

/* Legendre polynomial P_m(z) and its derivative by the three-term recurrence. */
static void legendre(int m, double z, double* pm, double* dpm) {
    double p0 = 1.0, p1 = z;
    if (m == 0) {
        *pm = 1.0;
        *dpm = 0.0;
        return;
    }
    for (int k = 2; k <= m; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    *pm = p1;
    /* (z^2 - 1) P_m' = m (z P_m - P_{m-1}) */
    *dpm = (m == 1) ? 1.0 : m * (z * p1 - p0) / (z * z - 1.0);
}

/* Gauss-Legendre rule with m points on [0,1]: roots of P_m by Newton's method from the
 * usual cosine guesses, weights 2 / ((1 - z^2) P_m'(z)^2), then the map z -> (1 - z)/2. */
static void gauss_legendre01(int m, double* x, double* w) {
    for (int i = 0; i < m; ++i) {
        double z = cos(M_PI * (i + 0.75) / (m + 0.5));
        double pm, dpm;
        for (int it = 0; it < 100; ++it) {
            legendre(m, z, &pm, &dpm);
            double dz = pm / dpm;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        legendre(m, z, &pm, &dpm);
        x[i] = 0.5 * (1.0 - z);
        w[i] = 0.5 * 2.0 / ((1.0 - z * z) * dpm * dpm);
    }
}

/* Collapsed-coordinate product rule on the reference simplex, m points per direction.
 * triangle: X1 = s1 (1 - s2), X2 = s2, dX = (1 - s2) ds
 * tetrahedron: X1 = s1 (1-s2)(1-s3), X2 = s2 (1-s3), X3 = s3, dX = (1-s2)(1-s3)^2 ds
 * Returns the number of points. */
int oracle_simplex_rule(int d, int m, double* pts, double* wts) {
    double x[64], w[64];
    if (m < 1 || m > 16 || (d != 2 && d != 3)) return -1;
    gauss_legendre01(m, x, w);
    int n = 0;
    if (d == 2) {
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                double s1 = x[i], s2 = x[j];
                pts[2 * n + 0] = s1 * (1.0 - s2);
                pts[2 * n + 1] = s2;
                wts[n] = w[i] * w[j] * (1.0 - s2);
                ++n;
            }
    } else {
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j)
                for (int k = 0; k < m; ++k) {
                    double s1 = x[i], s2 = x[j], s3 = x[k];
                    pts[3 * n + 0] = s1 * (1.0 - s2) * (1.0 - s3);
                    pts[3 * n + 1] = s2 * (1.0 - s3);
                    pts[3 * n + 2] = s3;
                    wts[n] = w[i] * w[j] * w[k] * (1.0 - s2) * (1.0 - s3) * (1.0 - s3);
                    ++n;
                }
    }
    return n;
}

/* ------------------------------------------------------------------ forms ---- */

static int is_vector(int kind) { return kind == OR_ELASTICITY || kind == OR_NS; }

int oracle_n_scalar_dofs(int dim, int degree) {
    int nodes[OR_MAX_NODES][4];
    if ((dim != 2 && dim != 3) || degree < 1 || degree > 4) return -1;
    return lagrange_nodes(dim, degree, nodes);
}

int oracle_n_dofs(int kind, int dim, int degree) {
    int ns = oracle_n_scalar_dofs(dim, degree);
    if (ns < 0 || kind < 0 || kind > 4) return -1;
    return is_vector(kind) ? dim * ns : ns;
}

int oracle_n_coeffs(int kind, int dim) {
    if (kind == OR_WLAPLACE) return dim + 1;
    if (kind == OR_NS) return dim * (dim + 1);
    return 0;
}

/* polynomial degree of the pulled-back integrand */
static int integrand_degree(int kind, int q) {
    switch (kind) {
    case OR_MASS: return 2 * q;
    case OR_LAPLACE: return 2 * q - 2;
    case OR_WLAPLACE: return 2 * q - 1;
    case OR_ELASTICITY: return 2 * q - 2;
    case OR_NS: return 2 * q;
    }
    return 2 * q;
}

/* Scalar-node multi-indices in dof order, for tests: nodes_out[n][4]. */
int oracle_nodes(int dim, int degree, int* nodes_out) {
    int nodes[OR_MAX_NODES][4];
    if ((dim != 2 && dim != 3) || degree < 1 || degree > 4) return -1;
    int nn = lagrange_nodes(dim, degree, nodes);
    for (int i = 0; i < nn; ++i)
        for (int v = 0; v < 4; ++v) nodes_out[4 * i + v] = (v <= dim) ? nodes[i][v] : 0;
    return nn;
}

/* Reference basis values / gradients at given reference points, for tests. */
int oracle_basis(int dim, int degree, int npts, const double* X, double* phi, double* dphi) {
    int nodes[OR_MAX_NODES][4];
    if ((dim != 2 && dim != 3) || degree < 1 || degree > 4) return -1;
    int nn = lagrange_nodes(dim, degree, nodes);
    for (int p = 0; p < npts; ++p)
        eval_basis(dim, degree, nn, (const int(*)[4])nodes, X + p * dim, phi + p * nn,
                   dphi + p * nn * dim);
    return nn;
}

static void element_tensor(int kind, int d, int q, double lam_, double mu_, int nn,
                           const int (*nodes)[4], int nq, const double* qp, const double* qw,
                           const double* x /* [d+1][d] vertices */, const double* wc,
                           double* A, double* phi, double* dphi, double* gphys) {
    /* Jacobian J[k][b] = dx_k / dX_b, columns = edge vectors from vertex 0 */
    double J[3][3] = {{0}}, G[3][3] = {{0}}, det;
    for (int k = 0; k < d; ++k)
        for (int b = 0; b < d; ++b) J[k][b] = x[(b + 1) * d + k] - x[k];
    if (d == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        G[0][0] = J[1][1] / det;
        G[0][1] = -J[0][1] / det;
        G[1][0] = -J[1][0] / det;
        G[1][1] = J[0][0] / det;
    } else {
        double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        /* inverse = adjugate / det, adj = cofactor^T */
        G[0][0] = c00 / det;
        G[1][0] = c01 / det;
        G[2][0] = c02 / det;
        G[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        G[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        G[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        G[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        G[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        G[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    }
    double adet = fabs(det);
    int n = is_vector(kind) ? d * nn : nn;
    for (int e = 0; e < n * n; ++e) A[e] = 0.0;

    for (int p = 0; p < nq; ++p) {
        const double* X = qp + p * d;
        eval_basis(d, q, nn, nodes, X, phi, dphi);
        /* physical gradients: d phi / d x_k = sum_b (dX_b/dx_k) dPhi/dX_b, G = J^{-1} */
        for (int i = 0; i < nn; ++i)
            for (int k = 0; k < d; ++k) {
                double s = 0.0;
                for (int b = 0; b < d; ++b) s += G[b][k] * dphi[i * d + b];
                gphys[i * d + k] = s;
            }
        /* barycentric coordinates of the point = P1 basis */
        double lam[4];
        lam[0] = 1.0;
        for (int b = 0; b < d; ++b) {
            lam[b + 1] = X[b];
            lam[0] -= X[b];
        }
        double W = qw[p] * adet;

        if (kind == OR_MASS || kind == OR_LAPLACE || kind == OR_WLAPLACE) {
            double coef = 1.0;
            if (kind == OR_WLAPLACE) {
                coef = 0.0;
                for (int t = 0; t <= d; ++t) coef += wc[t] * lam[t];
            }
            for (int i = 0; i < nn; ++i)
                for (int j = 0; j < nn; ++j) {
                    double val;
                    if (kind == OR_MASS) {
                        val = phi[i] * phi[j];
                    } else {
                        val = 0.0;
                        for (int k = 0; k < d; ++k) val += gphys[i * d + k] * gphys[j * d + k];
                        val *= coef;
                    }
                    A[i * n + j] += W * val;
                }
        } else if (kind == OR_ELASTICITY) {
            for (int c1 = 0; c1 < d; ++c1)
                for (int s1 = 0; s1 < nn; ++s1)
                    for (int c2 = 0; c2 < d; ++c2)
                        for (int s2 = 0; s2 < nn; ++s2) {
                            /* grad v: row c1 holds grad phi_s1; grad u: row c2 holds grad phi_s2 */
                            double gv[3][3] = {{0}}, gu[3][3] = {{0}};
                            for (int k = 0; k < d; ++k) {
                                gv[c1][k] = gphys[s1 * d + k];
                                gu[c2][k] = gphys[s2 * d + k];
                            }
                            double ev[3][3], eu[3][3], sg[3][3];
                            double tr = 0.0;
                            for (int a = 0; a < d; ++a)
                                for (int b = 0; b < d; ++b) {
                                    ev[a][b] = 0.5 * (gv[a][b] + gv[b][a]);
                                    eu[a][b] = 0.5 * (gu[a][b] + gu[b][a]);
                                }
                            for (int a = 0; a < d; ++a) tr += eu[a][a];
                            double val = 0.0;
                            for (int a = 0; a < d; ++a)
                                for (int b = 0; b < d; ++b) {
                                    sg[a][b] = 2.0 * mu_ * eu[a][b] + (a == b ? lam_ * tr : 0.0);
                                    val += sg[a][b] * ev[a][b];
                                }
                            A[(c1 * nn + s1) * n + (c2 * nn + s2)] += W * val;
                        }
        } else if (kind == OR_NS) {
            double wv[3];
            for (int k = 0; k < d; ++k) {
                wv[k] = 0.0;
                for (int t = 0; t <= d; ++t) wv[k] += wc[k * (d + 1) + t] * lam[t];
            }
            for (int c1 = 0; c1 < d; ++c1)
                for (int s1 = 0; s1 < nn; ++s1)
                    for (int c2 = 0; c2 < d; ++c2)
                        for (int s2 = 0; s2 < nn; ++s2) {
                            /* v = phi_s1 e_c1, u = phi_s2 e_c2: sum_c v_c sum_k w_k du_c/dx_k */
                            double val = 0.0;
                            for (int c = 0; c < d; ++c) {
                                double vc = (c == c1) ? phi[s1] : 0.0;
                                double conv = 0.0;
                                for (int k = 0; k < d; ++k) {
                                    double duck = (c == c2) ? gphys[s2 * d + k] : 0.0;
                                    conv += wv[k] * duck;
                                }
                                val += vc * conv;
                            }
                            A[(c1 * nn + s1) * n + (c2 * nn + s2)] += W * val;
                        }
        }
    }
}

/* Evaluate the element tensors of `cells` cells.
 *  coords: SoA, coords[(v * dim + k) * cells + c] = coordinate k of vertex v of cell c
 *  coeffs: SoA, coeffs[j * cells + c] (wlaplace: j = vertex; ns: j = comp * (dim+1) + vertex),
 *          NULL for forms without coefficients
 *  out:    [cells][n][n] row-major, row = test function.
 * Returns 0, or -1 for an unsupported form. */
int oracle_tabulate(int kind, int dim, int degree, double lam_, double mu_, long long cells,
                    const double* coords, const double* coeffs, double* out, int nthreads) {
    int nodes[OR_MAX_NODES][4];
    if ((dim != 2 && dim != 3) || degree < 1 || degree > 4 || kind < 0 || kind > 4) return -1;
    if (oracle_n_coeffs(kind, dim) > 0 && coeffs == NULL) return -1;
    int nn = lagrange_nodes(dim, degree, nodes);
    int n = is_vector(kind) ? dim * nn : nn;
    int p = integrand_degree(kind, degree);
    int m = (p + dim) / 2 + 1;
    double* qp = (double*)malloc(sizeof(double) * OR_MAX_QP * 3);
    double* qw = (double*)malloc(sizeof(double) * OR_MAX_QP);
    int nq = oracle_simplex_rule(dim, m, qp, qw);
    if (nq <= 0) {
        free(qp);
        free(qw);
        return -1;
    }
    int ncoef = oracle_n_coeffs(kind, dim);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        double phi[OR_MAX_NODES], dphi[OR_MAX_NODES * 3], gphys[OR_MAX_NODES * 3];
        double x[12], wc[12];
#pragma omp for schedule(static)
        for (long long c = 0; c < cells; ++c) {
            for (int j = 0; j < (dim + 1) * dim; ++j) x[j] = coords[(long long)j * cells + c];
            for (int j = 0; j < ncoef; ++j) wc[j] = coeffs[(long long)j * cells + c];
            element_tensor(kind, dim, degree, lam_, mu_, nn, (const int(*)[4])nodes, nq, qp, qw,
                           x, wc, out + c * (long long)n * n, phi, dphi, gphys);
        }
    }
    free(qp);
    free(qw);
    return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
