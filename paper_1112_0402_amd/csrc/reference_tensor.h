// Compile step (host, FP64 results from long-double arithmetic): the reference tensor
// A^0 of each supported form, its tiling for the matrix-core contraction, its BF16
// split pieces, and the tables of the plain quadrature kernel.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace ffc {

enum Kind { MASS = 0, LAPLACE = 1, WLAPLACE = 2, ELASTICITY = 3, NS = 4, PIOLA = 5, CURVED = 6, NEDELEC = 7 };

struct FormSpec {
    int kind = 0, dim = 2, degree = 1;
    double lambda = 1.0, mu = 1.0;
};

// Scalar Lagrange basis on K0 in the monomial basis: phi_i(X) = sum_m coef[m][i] X^exp[m].
struct LagrangeBasis {
    int dim = 0, degree = 0, n = 0;
    std::vector<std::array<int, 3>> exps;   // monomials of total degree <= q
    std::vector<long double> coef;          // [n_mono][n]
    std::vector<std::array<int, 4>> nodes;  // barycentric multi-indices in dof order
};

struct ReferenceTensor {
    FormSpec spec;
    int ns = 0;       // scalar dofs
    int n = 0;        // element dofs (d * ns for vector forms)
    int n_I = 0;      // n * n
    int n_alpha = 0;  // entries of G_K
    int n_coeff = 0;  // coefficient doubles per cell
    int64_t nnz = 0;
    std::vector<double> A0;  // [n_I][n_alpha]
    // CURVED (quadrature as contraction on cells with P2 geometry): quadrature points, the P2
    // geometry nodes per cell, and the reference gradients of the P2 geometry basis at the
    // points, [n_pts][n_geo][dim]
    int n_pts = 0, n_geo = 0;
    std::vector<double> geo_grad;
};

// Contraction tiles for 16 x 16 x 4 FP64 MFMA.  The n_I output entries are grouped into
// tiles of 16 (the MFMA N dimension); each tile keeps only the alpha columns that are
// nonzero in one of its rows (zeros of A^0 are skipped), padded to a multiple of 4 (the
// MFMA K step) with zero B values.  Grouping: within windows of `window` consecutive
// entries, rows are clustered greedily so that each tile's union of nonzero columns
// stays small; window == 16 keeps tiles contiguous, window <= 0 clusters over all rows.
struct TilesF64 {
    int n_tiles = 0;
    int window = 16;
    std::vector<int32_t> koff;    // [n_tiles + 1], in k rows (multiples of 4)
    std::vector<uint32_t> apack;  // [koff[n_tiles] / 4]: the 4 alpha indices of a k step, one byte each
    std::vector<double> b;        // [koff[n_tiles]][16] A^0 values, 0 for padding
    std::vector<int32_t> entry;   // [n_tiles][16] output entry of each tile column, -1 = padding
    // symmetric forms: only the entries i1 <= i2 of the element tensor are computed; each
    // result also lands at the transposed entry (n = element dofs)
    bool sym = false;
    int n = 0;
};

// Split-BF16 contraction: concatenated K = n_seg segments of n_alpha, segment s pairs
// G piece gpiece[s] with A^0 piece apiece[s]; padded to a multiple of 32.
struct TilesBF16 {
    int n_tiles = 0;
    int n_seg = 0;
    int kpad = 0;                  // padded concatenated K (multiple of 32)
    int gpiece[6] = {0}, apiece[6] = {0};
    std::vector<uint16_t> b;       // [n_tiles][kpad / 8][16][8] bf16 bits
    std::vector<uint8_t> nonzero;  // [n_tiles] 0 if the tile's rows of A^0 are all zero
};

struct QuadTables {
    int npts = 0, ns = 0, dim = 0, m = 0;
    std::vector<double> pts, wts;  // [npts][dim], [npts]
    std::vector<double> phi;       // [npts][ns]
    std::vector<double> dphi;      // [npts][ns][dim]
};

int n_scalar_dofs(int dim, int degree);
// collapsed Gauss-Jacobi rule on K0 with m points per direction (exact for degree 2m - 1)
void collapsed_rule(int dim, int m, std::vector<std::array<long double, 3>>* pts, std::vector<long double>* wts);
int integrand_degree(int kind, int degree);
bool supported(const FormSpec& s, std::string* why);

LagrangeBasis make_basis(int dim, int degree);
bool build_reference_tensor(const FormSpec& s, ReferenceTensor* out, std::string* err);
// Symmetric geometry tensors (Sec. 3.3): G^{ab} = G^{ba} for the Laplacian and, per weight
// dof, for the weighted Laplacian; G^{(aj)(bl)} = G^{(bl)(aj)} for elasticity.  The
// contraction then needs each unordered pair once, against the sum of its two A^0 columns.
// Returns A^0 with the columns folded that way -- pairs (u, v), u <= v, row by row; the
// weighted Laplacian keeps the weight dof as the outer index -- and every other form as it is.
ReferenceTensor fold_symmetric_g(const ReferenceTensor& rt);
// G entries per cell after the fold
int folded_n_alpha(int kind, int dim);
TilesF64 make_tiles_f64(const ReferenceTensor& rt, int window, bool sym = false);

// Static schedule of the FP64 tiles over the waves of a persistent workgroup: the tiles
// with a nonzero contraction are dealt to `waves` waves, longest first onto the least
// loaded wave (balancing k steps); each wave's steps are listed in order.  Entries whose
// rows of A^0 are all zero are listed apart (they are written as zeros).
struct WaveSchedule {
    int waves = 0;
    int max_steps = 0;                  // largest number of k steps of one wave
    std::vector<int32_t> woff;          // [waves + 1] step range of each wave
    std::vector<int32_t> step_kstep;    // [steps] k step (index into apack, and into b in units of 4 k rows)
    std::vector<int32_t> step_end;      // [steps] the tile if the step is its last, else -1
    std::vector<int32_t> zero_entries;  // entries whose A^0 row is zero
};
WaveSchedule make_wave_schedule(const TilesF64& T, int waves);
TilesBF16 make_tiles_bf16(const ReferenceTensor& rt, int products /* 3 or 6 */);
QuadTables make_quad_tables(const FormSpec& s);

// Gauss-Jacobi rule for weight (1-x)^a on [0,1], m points (Golub-Welsch).
void gauss_jacobi01(int m, int a, std::vector<long double>* x, std::vector<long double>* w);

// Round-to-nearest-even of a double to BF16 (returned as the double it represents).
double round_bf16(double x);
uint16_t bf16_bits(double representable);

}  // namespace ffc
