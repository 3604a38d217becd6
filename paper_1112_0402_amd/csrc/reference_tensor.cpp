// Compile step: reference tensors A^0 (Sec. 3.2, "Evaluation by tensor representation";
// per-form expressions in Sec. 3.3; integrals computed once per form, Sec. 5.3), their
// matrix-core tiling, BF16 split pieces, and the plain-quadrature tables (Sec. 6).
//
// Construction (independent of any quadrature): the Lagrange basis is obtained by
// inverting the monomial Vandermonde matrix at the equispaced nodes in long double, and
// every entry of A^0 is an integral of a polynomial over K0, summed exactly term by term
// with int_K0 X^e dX = e_1! ... e_d! / (|e| + d)!.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>

#include "reference_tensor.h"

namespace ffc {

namespace {

using ld = long double;

// ------------------------------------------------------------------ nodes -------

// Points strictly inside the sub-simplex with sorted vertices s_0 < ... < s_m, in
// ascending lexicographic order of (b_1, ..., b_m) (b_1 most significant); b_0 = q - sum.
void interior_rec(int j, int q, const std::vector<int>& s, std::vector<int>& cur,
                  std::vector<std::array<int, 4>>* nodes) {
    const int m = static_cast<int>(s.size()) - 1;
    if (j > m) {
        int sum = 0;
        for (int t = 1; t <= m; ++t) sum += cur[t];
        const int b0 = q - sum;
        if (b0 < 1) return;
        std::array<int, 4> a{0, 0, 0, 0};
        a[s[0]] = b0;
        for (int t = 1; t <= m; ++t) a[s[t]] = cur[t];
        nodes->push_back(a);
        return;
    }
    for (int v = 1; v <= q - 1; ++v) {
        cur[j] = v;
        interior_rec(j + 1, q, s, cur, nodes);
    }
}

void append_interior(int q, const std::vector<int>& s, std::vector<std::array<int, 4>>* nodes) {
    std::vector<int> cur(s.size(), 0);
    interior_rec(1, q, s, cur, nodes);
}

std::vector<std::array<int, 4>> lagrange_nodes(int d, int q) {
    std::vector<std::array<int, 4>> nodes;
    for (int v = 0; v <= d; ++v) {
        std::array<int, 4> a{0, 0, 0, 0};
        a[v] = q;
        nodes.push_back(a);
    }
    if (d == 2) {
        for (auto e : std::vector<std::vector<int>>{{1, 2}, {0, 2}, {0, 1}}) append_interior(q, e, &nodes);
        append_interior(q, {0, 1, 2}, &nodes);
    } else {
        for (auto e : std::vector<std::vector<int>>{{2, 3}, {1, 3}, {1, 2}, {0, 3}, {0, 2}, {0, 1}})
            append_interior(q, e, &nodes);
        for (auto f : std::vector<std::vector<int>>{{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}})
            append_interior(q, f, &nodes);
        append_interior(q, {0, 1, 2, 3}, &nodes);
    }
    return nodes;
}

// -------------------------------------------------------------- polynomials ------
// Sparse polynomial in X_1..X_d: key = e1 + 32 e2 + 1024 e3.

using Poly = std::map<int, ld>;

inline int key_of(const std::array<int, 3>& e) { return e[0] + 32 * e[1] + 1024 * e[2]; }
inline std::array<int, 3> exp_of(int k) { return {k & 31, (k >> 5) & 31, (k >> 10) & 31}; }

Poly mul(const Poly& p, const Poly& r) {
    Poly out;
    for (const auto& a : p)
        for (const auto& b : r) out[a.first + b.first] += a.second * b.second;
    return out;
}

Poly diff(const Poly& p, int b) {
    Poly out;
    for (const auto& t : p) {
        auto e = exp_of(t.first);
        if (e[b] == 0) continue;
        ld c = t.second * e[b];
        e[b] -= 1;
        out[key_of(e)] += c;
    }
    return out;
}

ld factorial(int n) {
    ld f = 1;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

// int_K0 X^e dX = prod e_b! / (|e| + d)!
ld integrate(const Poly& p, int d) {
    ld s = 0;
    for (const auto& t : p) {
        auto e = exp_of(t.first);
        int tot = 0;
        ld num = 1;
        for (int b = 0; b < d; ++b) {
            num *= factorial(e[b]);
            tot += e[b];
        }
        s += t.second * num / factorial(tot + d);
    }
    return s;
}

// P1 basis psi_t = barycentric coordinate t: psi_0 = 1 - sum X, psi_t = X_{t-1}.
Poly p1(int d, int t) {
    Poly p;
    if (t == 0) {
        p[0] = 1;
        for (int b = 0; b < d; ++b) {
            std::array<int, 3> e{0, 0, 0};
            e[b] = 1;
            p[key_of(e)] = -1;
        }
    } else {
        std::array<int, 3> e{0, 0, 0};
        e[t - 1] = 1;
        p[key_of(e)] = 1;
    }
    return p;
}

// Gauss-Jordan inverse with partial pivoting, in place, n x n row-major.
bool invert(std::vector<ld>& A, int n) {
    std::vector<ld> I(n * n, 0);
    for (int i = 0; i < n; ++i) I[i * n + i] = 1;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabsl(A[r * n + c]) > fabsl(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0) return false;
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(A[c * n + k], A[piv * n + k]);
                std::swap(I[c * n + k], I[piv * n + k]);
            }
        ld inv = 1 / A[c * n + c];
        for (int k = 0; k < n; ++k) {
            A[c * n + k] *= inv;
            I[c * n + k] *= inv;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            ld f = A[r * n + c];
            if (f == 0) continue;
            for (int k = 0; k < n; ++k) {
                A[r * n + k] -= f * A[c * n + k];
                I[r * n + k] -= f * I[c * n + k];
            }
        }
    }
    A.swap(I);
    return true;
}

ld eval(const Poly& p, const std::array<ld, 3>& X) {
    ld v = 0;
    for (const auto& t : p) {
        const auto e = exp_of(t.first);
        ld m = t.second;
        for (int b = 0; b < 3; ++b)
            for (int k = 0; k < e[b]; ++k) m *= X[b];
        v += m;
    }
    return v;
}

std::vector<Poly> basis_polys(const LagrangeBasis& B) {
    std::vector<Poly> out(B.n);
    const int nm = static_cast<int>(B.exps.size());
    for (int i = 0; i < B.n; ++i)
        for (int m = 0; m < nm; ++m) {
            ld c = B.coef[m * B.n + i];
            if (c != 0) out[i][key_of(B.exps[m])] += c;
        }
    return out;
}

}  // namespace

// ---------------------------------------------------------------- public -------

int n_scalar_dofs(int dim, int degree) {
    if (dim == 2) return (degree + 1) * (degree + 2) / 2;
    if (dim == 3) return (degree + 1) * (degree + 2) * (degree + 3) / 6;
    return -1;
}

int integrand_degree(int kind, int q) {
    switch (kind) {
    case MASS: return 2 * q;
    case LAPLACE: return 2 * q - 2;
    case WLAPLACE: return 2 * q - 1;
    case ELASTICITY: return 2 * q - 2;
    case NS: return 2 * q;
    case PIOLA: return 2;
    case CURVED: return 2 * q - 2;
    case NEDELEC: return 2;
    }
    return 2 * q;
}

bool supported(const FormSpec& s, std::string* why) {
    if (s.dim != 2 && s.dim != 3) {
        *why = "dim must be 2 or 3";
        return false;
    }
    if (s.kind < MASS || s.kind > NEDELEC) {
        *why = "unknown form kind";
        return false;
    }
    if ((s.kind == PIOLA || s.kind == NEDELEC) && s.degree != 1) {
        *why = "Raviart-Thomas and Nedelec elements of the lowest order only (degree 1)";
        return false;
    }
    int qmax = (s.kind == ELASTICITY || s.kind == NS) ? 3 : s.kind == CURVED ? 2 : 4;
    if (s.degree < 1 || s.degree > qmax) {
        *why = "degree out of range (1.." + std::to_string(qmax) + " for this form)";
        return false;
    }
    return true;
}

LagrangeBasis make_basis(int d, int q) {
    LagrangeBasis B;
    B.dim = d;
    B.degree = q;
    B.nodes = lagrange_nodes(d, q);
    B.n = static_cast<int>(B.nodes.size());
    for (int tot = 0; tot <= q; ++tot)
        for (int e0 = tot; e0 >= 0; --e0)
            for (int e1 = tot - e0; e1 >= 0; --e1) {
                int e2 = tot - e0 - e1;
                if (d == 2 && e2 != 0) continue;
                if (d == 2 && e0 + e1 != tot) continue;
                B.exps.push_back({e0, e1, d == 3 ? e2 : 0});
            }
    const int n = B.n;
    // V[k][m] = X_k^{e_m}, X_k = (a_1/q, ..., a_d/q)
    std::vector<ld> V(n * n);
    for (int k = 0; k < n; ++k)
        for (int m = 0; m < n; ++m) {
            ld v = 1;
            for (int b = 0; b < d; ++b) v *= powl(static_cast<ld>(B.nodes[k][b + 1]) / q, B.exps[m][b]);
            V[k * n + m] = v;
        }
    invert(V, n);  // V^{-1}: coef[m][i] so that phi_i(X_k) = delta_ik
    B.coef = V;
    return B;
}

bool build_reference_tensor(const FormSpec& s, ReferenceTensor* rt, std::string* err) {
    if (!supported(s, err)) return false;
    const int d = s.dim, q = s.degree;
    LagrangeBasis B = make_basis(d, q);
    if (static_cast<int>(B.exps.size()) != B.n) {
        *err = "internal: monomial count mismatch";
        return false;
    }
    std::vector<Poly> phi = basis_polys(B);
    std::vector<std::vector<Poly>> dphi(B.n, std::vector<Poly>(d));
    for (int i = 0; i < B.n; ++i)
        for (int b = 0; b < d; ++b) dphi[i][b] = diff(phi[i], b);

    rt->spec = s;
    rt->ns = B.n;
    const bool vec = (s.kind == ELASTICITY || s.kind == NS);
    rt->n = vec ? d * B.n : B.n;  // (PIOLA: the d + 1 vertices of P1 are also its d + 1 facets)
    if (s.kind == NEDELEC) rt->n = d * (d + 1) / 2;  // one dof per edge
    rt->n_I = rt->n * rt->n;
    switch (s.kind) {
    case MASS: rt->n_alpha = 1; rt->n_coeff = 0; break;
    case LAPLACE: rt->n_alpha = d * d; rt->n_coeff = 0; break;
    case WLAPLACE: rt->n_alpha = (d + 1) * d * d; rt->n_coeff = d + 1; break;
    case ELASTICITY: rt->n_alpha = d * d * d * d; rt->n_coeff = 0; break;
    case NS: rt->n_alpha = d * (d + 1) * d; rt->n_coeff = d * (d + 1); break;
    case PIOLA: rt->n_alpha = d * d; rt->n_coeff = 0; break;
    case CURVED: rt->n_alpha = 0; rt->n_coeff = 0; break;  // set below, with the rule
    case NEDELEC: rt->n_alpha = d * d; rt->n_coeff = 0; break;
    }
    // CURVED: the Laplacian on cells mapped by P2 geometry (Sec. 3.4, curvilinear elements),
    // integration replaced by a sum over the points X_p of a collapsed Gauss-Jacobi rule with
    // m = q + 1 points per direction: A^K = sum_p w_p |det J(X_p)| grad(phi_i1) . grad(phi_i2),
    // a contraction of A^0[(i1,i2)][(p, a, b)] = w_p dPhi_i1/dX_a dPhi_i2/dX_b (X_p) with
    // G_K[(p, a, b)] = |det J(X_p)| (g g^T)_ab(X_p); the (a, b) pairs are kept once, a <= b.
    std::vector<std::array<ld, 3>> cpts;
    std::vector<ld> cwts;
    if (s.kind == CURVED) {
        collapsed_rule(d, q + 1, &cpts, &cwts);
        rt->n_pts = static_cast<int>(cpts.size());
        rt->n_alpha = rt->n_pts * d * (d + 1) / 2;
        LagrangeBasis G2 = make_basis(d, 2);
        std::vector<Poly> psi = basis_polys(G2);
        rt->n_geo = G2.n;
        rt->geo_grad.assign(static_cast<size_t>(rt->n_pts) * G2.n * d, 0.0);
        for (int p = 0; p < rt->n_pts; ++p)
            for (int k = 0; k < G2.n; ++k)
                for (int b = 0; b < d; ++b)
                    rt->geo_grad[(static_cast<size_t>(p) * G2.n + k) * d + b] =
                        static_cast<double>(eval(diff(psi[k], b), cpts[p]));
    }
    const int ns = B.n, n = rt->n, na = rt->n_alpha;
    std::vector<ld> A(static_cast<size_t>(rt->n_I) * na, 0);
    auto at = [&](int i1, int i2, int alpha) -> ld& { return A[(static_cast<size_t>(i1) * n + i2) * na + alpha]; };

    if (s.kind == MASS) {
        for (int i = 0; i < ns; ++i)
            for (int j = 0; j < ns; ++j) at(i, j, 0) = integrate(mul(phi[i], phi[j]), d);
    } else if (s.kind == LAPLACE) {
        for (int i = 0; i < ns; ++i)
            for (int j = 0; j < ns; ++j)
                for (int a = 0; a < d; ++a)
                    for (int b = 0; b < d; ++b) at(i, j, a * d + b) = integrate(mul(dphi[i][a], dphi[j][b]), d);
    } else if (s.kind == WLAPLACE) {
        for (int t = 0; t <= d; ++t) {
            Poly psi = p1(d, t);
            for (int i = 0; i < ns; ++i)
                for (int a = 0; a < d; ++a) {
                    Poly pa = mul(psi, dphi[i][a]);
                    for (int j = 0; j < ns; ++j)
                        for (int b = 0; b < d; ++b) at(i, j, (t * d + a) * d + b) = integrate(mul(pa, dphi[j][b]), d);
                }
        }
    } else if (s.kind == ELASTICITY) {
        // A^0[(c1,s1),(c2,s2)][(a,j,b,l)] = C_{c1 j c2 l} int dPhi_s1/dX_a dPhi_s2/dX_b
        // C_ijkl = mu (d_ik d_jl + d_il d_jk) + lambda d_ij d_kl
        std::vector<ld> L(static_cast<size_t>(ns) * ns * d * d);
        for (int s1 = 0; s1 < ns; ++s1)
            for (int s2 = 0; s2 < ns; ++s2)
                for (int a = 0; a < d; ++a)
                    for (int b = 0; b < d; ++b)
                        L[((s1 * ns + s2) * d + a) * d + b] = integrate(mul(dphi[s1][a], dphi[s2][b]), d);
        const ld lam = s.lambda, mu = s.mu;
        auto C = [&](int i, int j, int k, int l) -> ld {
            return mu * ((i == k && j == l) + (i == l && j == k)) + lam * (i == j && k == l);
        };
        for (int c1 = 0; c1 < d; ++c1)
            for (int s1 = 0; s1 < ns; ++s1)
                for (int c2 = 0; c2 < d; ++c2)
                    for (int s2 = 0; s2 < ns; ++s2)
                        for (int a = 0; a < d; ++a)
                            for (int j = 0; j < d; ++j)
                                for (int b = 0; b < d; ++b)
                                    for (int l = 0; l < d; ++l) {
                                        ld c = C(c1, j, c2, l);
                                        if (c == 0) continue;
                                        at(c1 * ns + s1, c2 * ns + s2, ((a * d + j) * d + b) * d + l) =
                                            c * L[((s1 * ns + s2) * d + a) * d + b];
                                    }
    } else if (s.kind == CURVED) {
        const int np = d * (d + 1) / 2;
        for (int p = 0; p < rt->n_pts; ++p)
            for (int i = 0; i < ns; ++i)
                for (int j = 0; j < ns; ++j) {
                    int pr = 0;
                    for (int a = 0; a < d; ++a)
                        for (int b = a; b < d; ++b, ++pr) {
                            ld v = eval(dphi[i][a], cpts[p]) * eval(dphi[j][b], cpts[p]);
                            if (a != b) v += eval(dphi[i][b], cpts[p]) * eval(dphi[j][a], cpts[p]);
                            at(i, j, p * np + pr) = cwts[p] * v;
                        }
                }
    } else if (s.kind == NEDELEC) {
        // Psi_(a,b) = lambda_a grad lambda_b - lambda_b grad lambda_a, edges in the P2 edge order;
        // A^0[(i,j)][(a1,a2)] = int_K0 Psi_i,a1 Psi_j,a2
        static const int E2[3][2] = {{1, 2}, {0, 2}, {0, 1}};
        static const int E3[6][2] = {{2, 3}, {1, 3}, {1, 2}, {0, 3}, {0, 2}, {0, 1}};
        auto dlam = [&](int v, int a) -> ld { return v == 0 ? -1 : (v - 1 == a ? 1 : 0); };
        auto psi = [&](int e, int a) {
            const int va = d == 2 ? E2[e][0] : E3[e][0], vb = d == 2 ? E2[e][1] : E3[e][1];
            Poly p;
            for (const auto& t : p1(d, va)) p[t.first] += t.second * dlam(vb, a);
            for (const auto& t : p1(d, vb)) p[t.first] -= t.second * dlam(va, a);
            return p;
        };
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                for (int a1 = 0; a1 < d; ++a1)
                    for (int a2 = 0; a2 < d; ++a2) at(i, j, a1 * d + a2) = integrate(mul(psi(i, a1), psi(j, a2)), d);
    } else if (s.kind == PIOLA) {
        // Psi_i = (X - V_i) / (d |K0|) = (d-1)! (X - V_i), V_0 = 0, V_k = e_k;
        // A^0[(i,j)][(a1,a2)] = int_K0 Psi_i,a1 Psi_j,a2
        auto psi = [&](int i, int a) {
            Poly p;
            std::array<int, 3> e{0, 0, 0};
            e[a] = 1;
            const ld c = factorial(d - 1);
            p[key_of(e)] = c;
            if (i > 0 && i - 1 == a) p[0] -= c;
            return p;
        };
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                for (int a1 = 0; a1 < d; ++a1)
                    for (int a2 = 0; a2 < d; ++a2) at(i, j, a1 * d + a2) = integrate(mul(psi(i, a1), psi(j, a2)), d);
    } else if (s.kind == NS) {
        // A^0[(c1,s1),(c2,s2)][(k,t,a)] = delta_{c1 c2} int Phi_s1 psi_t dPhi_s2/dX_a
        for (int t = 0; t <= d; ++t) {
            Poly psi = p1(d, t);
            for (int s1 = 0; s1 < ns; ++s1) {
                Poly ps = mul(phi[s1], psi);
                for (int s2 = 0; s2 < ns; ++s2)
                    for (int a = 0; a < d; ++a) {
                        ld v = integrate(mul(ps, dphi[s2][a]), d);
                        for (int c = 0; c < d; ++c)
                            for (int k = 0; k < d; ++k) at(c * ns + s1, c * ns + s2, (k * (d + 1) + t) * d + a) = v;
                    }
            }
        }
    }
    // round to FP64; entries that are zero up to the rounding of the construction are
    // set to exactly zero (true nonzeros of these rational tensors are far larger)
    ld amax = 0;
    for (ld v : A) amax = std::max(amax, fabsl(v));
    rt->A0.resize(A.size());
    rt->nnz = 0;
    for (size_t k = 0; k < A.size(); ++k) {
        ld v = A[k];
        if (fabsl(v) <= 1e-12L * amax) v = 0;
        rt->A0[k] = static_cast<double>(v);
        rt->nnz += (v != 0);
    }
    return true;
}

int folded_n_alpha(int kind, int d) {
    switch (kind) {
    case LAPLACE: return d * (d + 1) / 2;
    case PIOLA: return d * (d + 1) / 2;
    case NEDELEC: return d * (d + 1) / 2;
    case WLAPLACE: return (d + 1) * d * (d + 1) / 2;
    case ELASTICITY: return d * d * (d * d + 1) / 2;
    case MASS: return 1;
    default: return d * (d + 1) * d;
    }
}

ReferenceTensor fold_symmetric_g(const ReferenceTensor& rt) {
    const int kind = rt.spec.kind, d = rt.spec.dim;
    if (kind != LAPLACE && kind != WLAPLACE && kind != ELASTICITY && kind != PIOLA && kind != NEDELEC) return rt;
    // pair index space: N indices per side, `outer` independent copies (weight dofs)
    const int N = kind == ELASTICITY ? d * d : d;
    const int outer = kind == WLAPLACE ? d + 1 : 1;
    const int np = N * (N + 1) / 2;
    ReferenceTensor f = rt;
    f.n_alpha = outer * np;
    f.A0.assign(static_cast<size_t>(rt.n_I) * f.n_alpha, 0.0);
    double amax = 0;
    for (double v : rt.A0) amax = std::max(amax, std::fabs(v));
    f.nnz = 0;
    for (int i = 0; i < rt.n_I; ++i)
        for (int t = 0; t < outer; ++t) {
            int p = 0;
            for (int u = 0; u < N; ++u)
                for (int v = u; v < N; ++v, ++p) {
                    const double* row = &rt.A0[static_cast<size_t>(i) * rt.n_alpha + t * N * N];
                    double x = u == v ? row[u * N + v] : row[u * N + v] + row[v * N + u];
                    if (std::fabs(x) <= 1e-12 * amax) x = 0;  // cancellation to rounding level
                    f.A0[static_cast<size_t>(i) * f.n_alpha + t * np + p] = x;
                    f.nnz += (x != 0);
                }
        }
    return f;
}

// ------------------------------------------------------------ MFMA tiles -------

namespace {

using Mask = std::array<uint64_t, 4>;  // nonzero alpha columns of a row (n_alpha <= 256)

int popcount(const Mask& m) {
    int c = 0;
    for (uint64_t w : m) c += __builtin_popcountll(w);
    return c;
}
Mask mask_and_not(const Mask& a, const Mask& b) {
    Mask r{};
    for (int k = 0; k < 4; ++k) r[k] = a[k] & ~b[k];
    return r;
}
Mask mask_and(const Mask& a, const Mask& b) {
    Mask r{};
    for (int k = 0; k < 4; ++k) r[k] = a[k] & b[k];
    return r;
}
void mask_or(Mask& a, const Mask& b) {
    for (int k = 0; k < 4; ++k) a[k] |= b[k];
}

// Greedy clustering of `rows` into groups of at most 16: seed = remaining row with the most
// nonzero columns, then repeatedly add the row that grows the union least (ties: the row
// that shares most columns with the union, then the lower row index).
std::vector<std::vector<int>> cluster_rows(const std::vector<int>& rows, const std::vector<Mask>& mask) {
    std::vector<std::vector<int>> groups;
    std::vector<int> rem(rows);
    while (!rem.empty()) {
        size_t seed = 0;
        for (size_t i = 1; i < rem.size(); ++i)
            if (popcount(mask[rem[i]]) > popcount(mask[rem[seed]])) seed = i;
        std::vector<int> g{rem[seed]};
        Mask u = mask[rem[seed]];
        rem.erase(rem.begin() + seed);
        while (g.size() < 16 && !rem.empty()) {
            size_t best = 0;
            int best_inc = 1 << 30, best_ov = -1;
            for (size_t i = 0; i < rem.size(); ++i) {
                const Mask& m = mask[rem[i]];
                const Mask inc = mask_and_not(m, u);
                const Mask ov = mask_and(m, u);
                const int ci = popcount(inc), co = popcount(ov);
                if (ci < best_inc || (ci == best_inc && co > best_ov)) {
                    best = i;
                    best_inc = ci;
                    best_ov = co;
                }
            }
            mask_or(u, mask[rem[best]]);
            g.push_back(rem[best]);
            rem.erase(rem.begin() + best);
        }
        std::sort(g.begin(), g.end());
        groups.push_back(g);
    }
    return groups;
}

}  // namespace

TilesF64 make_tiles_f64(const ReferenceTensor& rt, int window, bool sym) {
    TilesF64 T;
    const int nI = rt.n_I, na = rt.n_alpha;
    T.window = window;
    T.sym = sym;
    T.n = rt.n;
    T.koff.assign(1, 0);
    if (na > 256) return T;  // alpha indices are packed in one byte: no tiles (supported() keeps forms below)
    std::vector<Mask> mask(nI, Mask{});
    for (int r = 0; r < nI; ++r)
        for (int a = 0; a < na; ++a)
            if (rt.A0[static_cast<size_t>(r) * na + a] != 0) mask[r][a >> 6] |= uint64_t(1) << (a & 63);
    // the entries to compute: all, or those with i1 <= i2 (entry = i1 * n + i2)
    std::vector<int> todo;
    for (int r = 0; r < nI; ++r)
        if (!sym || r / rt.n <= r % rt.n) todo.push_back(r);
    const int nT = static_cast<int>(todo.size());
    std::vector<std::vector<int>> groups;
    const int W = window <= 0 ? nT : window;
    for (int w0 = 0; w0 < nT; w0 += W) {
        std::vector<int> rows;
        for (int q = w0; q < std::min(nT, w0 + W); ++q) rows.push_back(todo[q]);
        if (W == 16) {
            groups.push_back(rows);
        } else {
            auto g = cluster_rows(rows, mask);
            groups.insert(groups.end(), g.begin(), g.end());
        }
    }
    T.n_tiles = static_cast<int>(groups.size());
    T.koff.assign(T.n_tiles + 1, 0);
    T.entry.assign(static_cast<size_t>(T.n_tiles) * 16, -1);
    for (int t = 0; t < T.n_tiles; ++t) {
        const auto& g = groups[t];
        Mask u{};
        for (size_t e = 0; e < g.size(); ++e) {
            T.entry[static_cast<size_t>(t) * 16 + e] = g[e];
            mask_or(u, mask[g[e]]);
        }
        std::vector<int> cols;
        for (int a = 0; a < na; ++a)
            if (u[a >> 6] >> (a & 63) & 1) cols.push_back(a);
        const int kpad = (static_cast<int>(cols.size()) + 3) / 4 * 4;
        for (int k = 0; k < kpad; ++k) {
            const bool real = k < static_cast<int>(cols.size());
            const int a = real ? cols[k] : (cols.empty() ? 0 : cols[0]);
            if (k % 4 == 0) T.apack.push_back(0);
            T.apack.back() |= static_cast<uint32_t>(a) << (8 * (k % 4));
            for (int e = 0; e < 16; ++e) {
                const int row = T.entry[static_cast<size_t>(t) * 16 + e];
                T.b.push_back((real && row >= 0) ? rt.A0[static_cast<size_t>(row) * na + a] : 0.0);
            }
        }
        T.koff[t + 1] = T.koff[t] + kpad;
    }
    return T;
}

WaveSchedule make_wave_schedule(const TilesF64& T, int waves) {
    WaveSchedule S;
    S.waves = waves;
    std::vector<int> tiles;
    for (int t = 0; t < T.n_tiles; ++t) {
        if (T.koff[t + 1] > T.koff[t]) {
            tiles.push_back(t);
        } else {
            for (int e = 0; e < 16; ++e) {
                const int x = T.entry[static_cast<size_t>(t) * 16 + e];
                if (x < 0) continue;
                S.zero_entries.push_back(x);
                if (T.sym && (x % T.n) * T.n + x / T.n != x) S.zero_entries.push_back((x % T.n) * T.n + x / T.n);
            }
        }
    }
    std::stable_sort(tiles.begin(), tiles.end(), [&](int a, int b) {
        return (T.koff[a + 1] - T.koff[a]) > (T.koff[b + 1] - T.koff[b]);
    });
    std::vector<std::vector<int>> own(waves);
    std::vector<int> load(waves, 0);
    for (int t : tiles) {
        int w = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
        own[w].push_back(t);
        load[w] += (T.koff[t + 1] - T.koff[t]) / 4;
    }
    S.woff.assign(waves + 1, 0);
    for (int w = 0; w < waves; ++w) {
        std::sort(own[w].begin(), own[w].end());
        for (int t : own[w]) {
            const int k0 = T.koff[t] / 4, k1 = T.koff[t + 1] / 4;
            for (int k = k0; k < k1; ++k) {
                S.step_kstep.push_back(k);
                S.step_end.push_back(k == k1 - 1 ? t : -1);
            }
        }
        S.woff[w + 1] = static_cast<int>(S.step_kstep.size());
        S.max_steps = std::max(S.max_steps, S.woff[w + 1] - S.woff[w]);
    }
    return S;
}

double round_bf16(double x) {
    // keep the top 7 explicit mantissa bits of the double, round to nearest even on the
    // remaining 45; values here are far inside the BF16 normal range
    if (x == 0.0 || !std::isfinite(x)) return x;
    uint64_t u;
    std::memcpy(&u, &x, 8);
    const uint64_t drop = 45;
    uint64_t lsb = (u >> drop) & 1u;
    u += ((uint64_t(1) << (drop - 1)) - 1) + lsb;
    u &= ~((uint64_t(1) << drop) - 1);
    double r;
    std::memcpy(&r, &u, 8);
    return r;
}

uint16_t bf16_bits(double representable) {
    float f = static_cast<float>(representable);  // exact: 8 significant bits
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return static_cast<uint16_t>(u >> 16);
}

TilesBF16 make_tiles_bf16(const ReferenceTensor& rt, int products) {
    TilesBF16 T;
    const int nI = rt.n_I, na = rt.n_alpha;
    T.n_tiles = (nI + 15) / 16;
    // pieces 0 = hi, 1 = lo, 2 = lo2
    if (products == 3) {
        T.n_seg = 3;
        const int g[3] = {0, 0, 1}, a[3] = {0, 1, 0};
        for (int s = 0; s < 3; ++s) {
            T.gpiece[s] = g[s];
            T.apiece[s] = a[s];
        }
    } else {
        T.n_seg = 6;
        const int g[6] = {0, 0, 1, 0, 1, 2}, a[6] = {0, 1, 0, 2, 1, 0};
        for (int s = 0; s < 6; ++s) {
            T.gpiece[s] = g[s];
            T.apiece[s] = a[s];
        }
    }
    const int K = T.n_seg * na;
    T.kpad = (K + 31) / 32 * 32;
    // pieces of A^0
    std::vector<double> P[3];
    for (int p = 0; p < 3; ++p) P[p].resize(rt.A0.size());
    for (size_t k = 0; k < rt.A0.size(); ++k) {
        double x = rt.A0[k];
        double hi = round_bf16(x);
        double lo = round_bf16(x - hi);
        double lo2 = round_bf16((x - hi) - lo);
        P[0][k] = hi;
        P[1][k] = lo;
        P[2][k] = lo2;
    }
    T.b.assign(static_cast<size_t>(T.n_tiles) * T.kpad * 16, 0);
    T.nonzero.assign(T.n_tiles, 0);
    for (int t = 0; t < T.n_tiles; ++t) {
        for (int kk = 0; kk < T.kpad; ++kk) {
            int s = kk / na, a = kk % na;
            for (int e = 0; e < 16; ++e) {
                int row = t * 16 + e;
                double v = 0.0;
                if (kk < K && row < nI) v = P[T.apiece[s]][static_cast<size_t>(row) * na + a];
                if (kk < K && row < nI && rt.A0[static_cast<size_t>(row) * na + a] != 0) T.nonzero[t] = 1;
                // layout [tile][kk/8][e][kk%8]
                size_t idx = ((static_cast<size_t>(t) * (T.kpad / 8) + kk / 8) * 16 + e) * 8 + kk % 8;
                T.b[idx] = bf16_bits(v);
            }
        }
    }
    return T;
}

// ----------------------------------------------------------- quadrature --------

// Golub-Welsch: nodes = eigenvalues of the Jacobi matrix of the monic Jacobi
// polynomials for weight (1-x)^a (1+x)^0 on [-1,1], weights = mu_0 * (first component of
// the normalised eigenvector)^2; eigenproblem by cyclic Jacobi rotations; then mapped to
// [0,1] with weight (1-xi)^a.
void gauss_jacobi01(int m, int a, std::vector<long double>* x, std::vector<long double>* w) {
    const ld al = a, be = 0;
    std::vector<ld> M(m * m, 0), V(m * m, 0);
    for (int i = 0; i < m; ++i) {
        V[i * m + i] = 1;
        ld k = i;
        ld diag;
        if (i == 0)
            diag = (be - al) / (al + be + 2);
        else
            diag = (be * be - al * al) / ((2 * k + al + be) * (2 * k + al + be + 2));
        M[i * m + i] = diag;
        if (i + 1 < m) {
            ld kk = i + 1;
            ld num = 4 * kk * (kk + al) * (kk + be) * (kk + al + be);
            ld s = 2 * kk + al + be;
            ld den = s * s * (s + 1) * (s - 1);
            ld off = sqrtl(num / den);
            M[i * m + i + 1] = off;
            M[(i + 1) * m + i] = off;
        }
    }
    for (int sweep = 0; sweep < 100; ++sweep) {
        ld offn = 0;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) offn += M[p * m + q] * M[p * m + q];
        if (offn < 1e-40L) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                ld apq = M[p * m + q];
                if (fabsl(apq) < 1e-300L) continue;
                ld theta = (M[q * m + q] - M[p * m + p]) / (2 * apq);
                ld t = (theta >= 0 ? 1 : -1) / (fabsl(theta) + sqrtl(theta * theta + 1));
                ld c = 1 / sqrtl(t * t + 1), s = t * c;
                for (int k = 0; k < m; ++k) {  // M <- M R
                    ld mkp = M[k * m + p], mkq = M[k * m + q];
                    M[k * m + p] = c * mkp - s * mkq;
                    M[k * m + q] = s * mkp + c * mkq;
                }
                for (int k = 0; k < m; ++k) {  // M <- R^T M
                    ld mpk = M[p * m + k], mqk = M[q * m + k];
                    M[p * m + k] = c * mpk - s * mqk;
                    M[q * m + k] = s * mpk + c * mqk;
                }
                for (int k = 0; k < m; ++k) {  // V <- V R
                    ld vkp = V[k * m + p], vkq = V[k * m + q];
                    V[k * m + p] = c * vkp - s * vkq;
                    V[k * m + q] = s * vkp + c * vkq;
                }
            }
    }
    // mu_0 = int_{-1}^1 (1-x)^a dx = 2^{a+1}/(a+1)
    ld mu0 = powl(2.0L, a + 1) / (a + 1);
    std::vector<std::pair<ld, ld>> nw;
    for (int i = 0; i < m; ++i) {
        ld xi = M[i * m + i];
        ld wi = mu0 * V[0 * m + i] * V[0 * m + i];
        // to [0,1]: xi' = (1 + x)/2, (1 - xi') = (1 - x)/2, dxi' = dx/2
        nw.push_back({(1 + xi) / 2, wi / powl(2.0L, a + 1)});
    }
    std::sort(nw.begin(), nw.end());
    x->clear();
    w->clear();
    for (auto& p : nw) {
        x->push_back(p.first);
        w->push_back(p.second);
    }
}

void collapsed_rule(int d, int m, std::vector<std::array<ld, 3>>* pts, std::vector<ld>* wts) {
    std::vector<ld> x0, w0, x1, w1, x2, w2;
    gauss_jacobi01(m, 0, &x0, &w0);
    gauss_jacobi01(m, 1, &x1, &w1);
    gauss_jacobi01(m, 2, &x2, &w2);
    pts->clear();
    wts->clear();
    if (d == 2) {
        // X1 = s1 (1 - s2), X2 = s2, dX = (1 - s2) ds, the (1 - s2) factor in the
        // Jacobi weight of the second direction
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                pts->push_back({x0[i] * (1 - x1[j]), x1[j], 0});
                wts->push_back(w0[i] * w1[j]);
            }
    } else {
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j)
                for (int k = 0; k < m; ++k) {
                    pts->push_back({x0[i] * (1 - x1[j]) * (1 - x2[k]), x1[j] * (1 - x2[k]), x2[k]});
                    wts->push_back(w0[i] * w1[j] * w2[k]);
                }
    }
}

QuadTables make_quad_tables(const FormSpec& s) {
    QuadTables Q;
    const int d = s.dim;
    int p = std::max(0, integrand_degree(s.kind, s.degree));
    int m = (p + 2) / 2;  // ceil((p + 1) / 2)
    if (m < 1) m = 1;
    Q.m = m;
    Q.dim = d;
    std::vector<std::array<ld, 3>> pts;
    std::vector<ld> wts;
    collapsed_rule(d, m, &pts, &wts);
    Q.npts = static_cast<int>(pts.size());
    LagrangeBasis B = make_basis(d, s.degree);
    Q.ns = B.n;
    std::vector<Poly> phi = basis_polys(B);
    Q.pts.resize(Q.npts * d);
    Q.wts.resize(Q.npts);
    Q.phi.resize(Q.npts * B.n);
    Q.dphi.resize(Q.npts * B.n * d);
    for (int qp = 0; qp < Q.npts; ++qp) {
        for (int b = 0; b < d; ++b) Q.pts[qp * d + b] = static_cast<double>(pts[qp][b]);
        Q.wts[qp] = static_cast<double>(wts[qp]);
        for (int i = 0; i < B.n; ++i) {
            ld v = 0;
            ld g[3] = {0, 0, 0};
            for (const auto& t : phi[i]) {
                auto e = exp_of(t.first);
                ld mono = 1;
                for (int b = 0; b < d; ++b) mono *= powl(pts[qp][b], e[b]);
                v += t.second * mono;
                for (int b = 0; b < d; ++b) {
                    if (e[b] == 0) continue;
                    ld dm = e[b];
                    for (int c = 0; c < d; ++c) dm *= powl(pts[qp][c], e[c] - (c == b ? 1 : 0));
                    g[b] += t.second * dm;
                }
            }
            Q.phi[qp * B.n + i] = static_cast<double>(v);
            for (int b = 0; b < d; ++b) Q.dphi[(qp * B.n + i) * d + b] = static_cast<double>(g[b]);
        }
    }
    return Q;
}

}  // namespace ffc
