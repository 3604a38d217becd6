/*
 * ffc_hip -- element tensors in the tensor representation A^K = A^0 : G_K on AMD
 * Instinct MI355X (gfx950).
 *
 * The element tensor of a bilinear form on an affine simplex K (element matrix, Sec. 2.2;
 * element tensor of a multilinear form, Sec. 3.1) is evaluated as the contraction
 *     A^K_i = A^0_{i alpha} G_K^alpha                      (eq. tensorproduct, Sec. 3.2)
 * of a reference tensor A^0, integrated once per form on the reference simplex K0 in FP64
 * on the host (the compile step: "Evaluation of integrals", Sec. 5.3), with a geometry
 * tensor G_K built per cell from det F'_K, the inverse Jacobian g_ab = dX_a/dx_b and the
 * coefficient dofs (Sec. 3.2 and test cases 1-4, Sec. 3.3).  On the device:
 *   1. a geometry kernel, one lane per cell, FP64: coords -> (det J, J^{-1});
 *   2. a contraction kernel: G_K tile built in LDS, A^0 tiles on the matrix cores
 *      (MFMA), cells x |alpha| times |alpha| x |i| -- the level-3 BLAS batching the
 *      paper proposes (Sec. 3.5, "Optimization");
 * and, as the in-GPU comparison, a plain quadrature kernel (pretabulated basis at the
 * points of a collapsed-coordinate Gauss-Jacobi rule exact for the integrand, Sec. 6).
 * Also here: split-BF16 contraction modes, mixed batches in a short fixed launch sequence
 * (ffc_batch_*), global assembly into CSR (ffc_assembly_*, ffc_assemble; Algorithm 2),
 * the operator action without writing element tensors (ffc_apply_tensor,
 * ffc_operator_apply), the H(div) / H(curl) and curvilinear extensions of Sec. 3.4 as
 * form kinds, and the kernel selector network's kernels (ffc_mlp_*, ffc_adam_step).
 *
 * Conventions shared by every entry point
 *  - Reference simplex K0: vertex 0 at the origin, vertex k at the k-th unit vector
 *    (affine-map figure, Sec. 3.2).  J = [x^1 - x^0, ..., x^d - x^0] (columns).
 *  - Lagrange P_q dofs: point evaluation at the equispaced nodes (Sec. 5.3), ordered
 *    vertices, edges (triangle: edge k opposite vertex k; tetrahedron: (2,3),(1,3),(1,2),
 *    (0,3),(0,2),(0,1), points from the lower to the higher vertex), faces (face k
 *    opposite vertex k), interior; inside a sub-simplex with sorted vertices s_0<..<s_m,
 *    ascending lexicographic order of (b_1..b_m).  Vector elements are component-blocked:
 *    dof (c, s) -> c * n_scalar + s.
 *  - Element tensor layout: out[cell][i1 * n + i2], row i1 = test function (first
 *    argument of a(v, u)), n = element dofs.
 *  - |det J| is used (the paper's det F'_K for positively oriented cells).
 *  - coords (device, FP64, SoA): coords[(v * d + k) * cells + c] = coordinate k of local
 *    vertex v of cell c (FFC_CURVED_LAPLACE: v runs over the cell's P2 nodes).
 *  - coeffs (device, FP64, SoA): coeffs[j * cells + c]; weighted Laplacian: j = vertex
 *    (w in P1); Navier-Stokes: j = comp * (d + 1) + vertex (w in vector P1).  NULL for
 *    forms without coefficients.
 *  - All device pointers are caller-owned (for example torch tensors) and must stay
 *    valid until the work enqueued on the form's stream has finished.
 *
 * Errors: every int-returning call returns FFC_OK (0) or a negative ffc_status; the
 * message of the last failure on the calling thread is ffc_last_error().  Argument
 * errors are detected before anything is enqueued.  Device faults surface as
 * FFC_E_DEVICE from the call that observes them.
 */
#ifndef FFC_HIP_H
#define FFC_HIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque form handle: the compiled reference tensor, its device tables and workspace. */
typedef struct ffc_form ffc_form;

typedef enum {
    FFC_OK = 0,
    FFC_E_INVALID = -1,     /* bad argument (NULL pointer, negative size, wrong mode) */
    FFC_E_UNSUPPORTED = -2, /* form / dimension / degree / precision not supported   */
    FFC_E_DEVICE = -3,      /* HIP runtime error, or no usable gfx950 device        */
    FFC_E_DEGENERATE = -4,  /* ffc_check_cells found degenerate cells                */
    FFC_E_NOMEM = -5        /* host or device allocation failed (create calls, and
                               the validation call's counters)                       */
} ffc_status;

/* Forms (v = test, u = trial):
 *  FFC_MASS          int v u                              (test case 1, eq. mass)
 *  FFC_LAPLACE       int grad v . grad u                  (test case 2, eq. poisson)
 *  FFC_WLAPLACE      int w grad v . grad u, w in P1       (variable-coefficient diffusion, Sec. 3.1)
 *  FFC_ELASTICITY    int sigma(u) : eps(v), sigma = 2 mu eps + lambda tr(eps) I, vector P_q
 *                    (test case 4; the paper's strain-strain term is mu = 1/2, lambda = 0)
 *  FFC_NS_CONVECTION int v . ((w . grad) u), u, v vector P_q, w vector P1 (test case 3)
 *  FFC_PIOLA_MASS    int v . u for Raviart-Thomas functions of the lowest order mapped by
 *                    the contravariant Piola transform (the H(div) example of Sec. 3.4):
 *                    degree 1 only; d + 1 dofs, reference basis Psi_i = (X - V_i) / (d |K0|)
 *                    (unit flux through the facet opposite vertex i); A^0 = int Psi_i,a1
 *                    Psi_j,a2, G^{a1 a2} = (1 / |det J|) (J^T J)_{a1 a2}; tensor kernel only
 *                    (no quadrature kernel, no batches)
 *  FFC_NEDELEC_MASS  int v . u for Nedelec (Whitney edge) functions of the lowest order
 *                    mapped by the covariant Piola transform (the H(curl) side of Sec. 3.4):
 *                    degree 1 only; one dof per edge, edges in the P2 edge order below,
 *                    oriented from the lower to the higher vertex, reference basis
 *                    Psi_(a,b) = lambda_a grad lambda_b - lambda_b grad lambda_a; A^0 =
 *                    int Psi_i,a1 Psi_j,a2 and G = |det J| (g g^T) -- the Laplacian's G; tensor
 *                    kernel only (no quadrature kernel, no batches)
 *  FFC_CURVED_LAPLACE int grad u . grad v, u, v in P_q (q = 1, 2), on cells mapped by P2
 *                    geometry (the curvilinear elements of Sec. 3.4): the Jacobian varies
 *                    inside the cell, so the integral becomes a sum over the points X_p of a
 *                    collapsed Gauss-Jacobi rule with q + 1 points per direction, contracted as
 *                    A^0[(i1,i2)][(p,a,b)] = w_p dPhi_i1/dX_a dPhi_i2/dX_b (X_p) with
 *                    G_K[(p,a,b)] = |det J(X_p)| (g g^T)_ab(X_p) (pairs a <= b, b's summed
 *                    into A^0).  coords: SoA [n_geo * d][cells] with the n_geo = 6 (d = 2)
 *                    or 10 (d = 3) P2 nodes of each cell in the P2 dof order below; each
 *                    cell tile builds its G at the points in LDS (with geometry = PASS, a
 *                    geometry kernel writes G into the form's workspace first).  FP64 tensor
 *                    kernel only (no quadrature kernel, split modes, batches, operator action
 *                    or affine-map entry). */
typedef enum {
    FFC_MASS = 0, FFC_LAPLACE = 1, FFC_WLAPLACE = 2, FFC_ELASTICITY = 3, FFC_NS_CONVECTION = 4, FFC_PIOLA_MASS = 5,
    FFC_CURVED_LAPLACE = 6, FFC_NEDELEC_MASS = 7
} ffc_kind;

/* Arithmetic of the contraction.  FP64: FP64 MFMA, FP64 output.  Split modes: G and A^0
 * are split into BF16 pieces (hi = RN(x), lo = RN(x - hi), [lo2 = RN(x - hi - lo)]) with
 * the subtractions in FP64, multiplied on BF16 MFMA with FP32 accumulation, FP32 output;
 * geometry stays FP64.  3 products: hi*hi + hi*lo + lo*hi.  6 products: additionally
 * hi*lo2 + lo*lo + lo2*hi. */
typedef enum { FFC_FP64 = 0, FFC_SPLIT_BF16_3 = 1, FFC_SPLIT_BF16_6 = 2 } ffc_precision;

/* Which kernel evaluates A^K.  QUADRATURE is FP64 only.
 * AUTO: the automatic choice between tensor representation and quadrature (and among the
 * tensor kernel's launch shapes) that Sec. 4.4 leaves open, made by the learned selector
 * network (ffc_mlp_* below; it predicts each candidate launch's run time relative to the
 * library default from the form's rank, degree, |i|, |alpha|, dimension and the cell
 * count).  ffc_form_create reads the trained network from the file named by the
 * environment variable FFC_SELECTOR ("none": no file), else from
 * data/selector_mi355x_fp64.txt in the directory of this library; evaluates it on the host
 * for every cell count 2^0 .. 2^40 (a launch other than the default is picked only when
 * predicted faster by more than the file's decision margin); and creates one internal form
 * per launch it picks, so
 * ffc_tabulate_tensor only dispatches (to the pick for round(log2 cells)) and still never
 * allocates.  The network decides for FP64 Lagrange forms (FFC_MASS .. FFC_NS_CONVECTION),
 * the forms it was trained on; elsewhere, and when no file is found, every cell count takes
 * the library default tensor launch.  A file named by FFC_SELECTOR that cannot be read is
 * an error (FFC_E_INVALID).  Entry points other than ffc_tabulate_tensor, and
 * ffc_form_get_info, use the default tensor launch. */
typedef enum { FFC_KERNEL_AUTO = 0, FFC_KERNEL_TENSOR = 1, FFC_KERNEL_QUADRATURE = 2 } ffc_kernel;
typedef enum { FFC_GEOMETRY_PASS = 1, FFC_GEOMETRY_FUSED = 2 } ffc_geometry;

typedef struct {
    int32_t kind;        /* ffc_kind */
    int32_t dim;         /* 2 (triangles) or 3 (tetrahedra) */
    int32_t degree;      /* Lagrange degree q of u and v: 1..4 (vector forms: 1..3) */
    int32_t precision;   /* ffc_precision */
    int32_t kernel;      /* ffc_kernel */
    int32_t tile_cells;  /* cells per workgroup tile of the contraction: 0 = default, else 16, 32 or 64
                            (with persistent = 1: the persistent kernel's cell tile; 32 and 64
                            in FP64 take 12 waves) */
    int32_t waves;       /* waves per workgroup of the contraction: 0 = default, else 1, 2, 4, 8,
                            12 or 16 (the persistent FP64 kernel: 12 = 6 compute + 6 I/O
                            waves, which also computes the affine maps; 16 = 10 + 6 with a
                            geometry pass) */
    int32_t tile_window; /* FP64 tensor kernel: grouping of the n_I output entries into the
                            16-entry MFMA tiles.  0 = default; 16 = consecutive entries; a
                            multiple of 16 = rows clustered greedily (smallest union of nonzero
                            A^0 columns) inside windows of that many consecutive entries;
                            -1 = clustered over all entries.  Ignored by the other kernels. */
    int32_t persistent;  /* tensor kernel: 0 = auto (persistent workgroups with the A^0 tiles
                            in registers for element tensors of at least 100 entries in FP64
                            -- 12 waves on 16-, 32- or 64-cell tiles below 576 entries, 16-cell
                            tiles from 576 -- and 144 in the split modes, 100 for forms with
                            coefficients, when they fit; FP64 forms without coefficients of 400
                            entries and more build that schedule for the operator action and
                            batches but tabulate on one 16-cell tile per workgroup after a
                            geometry pass, measured faster there),
                            1 = persistent whenever it fits, -1 = one workgroup per cell tile.
                            Default tile launches: the cell tile and workgroup size measured
                            fastest for the element tensor's size (one or two waves for
                            tensors of at most 36 entries); ffc_form_get_info reports them */
    int32_t geometry;    /* tensor kernel, ffc_tabulate_tensor: where the affine map is
                            computed.  FFC_GEOMETRY_PASS = a geometry kernel writes it to a
                            form-owned workspace that the contraction reads;
                            FFC_GEOMETRY_FUSED = the contraction computes it from the
                            coordinates (one launch, no workspace round trip): the per-tile
                            kernels per cell tile in LDS, the persistent FP64 kernel one tile
                            ahead of the contraction.  The persistent split-BF16 kernel always
                            uses the pass, and so does the 16-wave persistent FP64 kernel.
                            0 = default = fused where available, except FP64 tile launches of
                            16-cell tiles (large tensors), which take the pass. */
    int32_t symmetry;    /* FP64 tensor kernel: 0 = auto (for the symmetric forms -- all but
                            FFC_NS_CONVECTION -- compute only the entries i1 <= i2 on the
                            matrix cores and write each also at (i2, i1): half the MFMA
                            work; used where it saves MFMA steps and the output rows are
                            staged in LDS, i.e. the persistent kernel or a staged tile
                            launch), -1 = compute every entry */
    double lambda, mu;   /* Lame parameters (FFC_ELASTICITY only) */
    void* stream;        /* hipStream_t the form's work is enqueued on; NULL = default stream */
} ffc_form_desc;

typedef struct {
    int64_t n_dofs;           /* n: element dofs per argument */
    int64_t n_entries;        /* n_I = n * n entries per element tensor */
    int64_t n_alpha;          /* |alpha|: entries of G_K per cell */
    int64_t nnz_a0;           /* nonzero entries of A^0 */
    int64_t n_coords;         /* (d + 1) * d doubles per cell */
    int64_t n_coeffs;         /* coefficient doubles per cell (0 if none) */
    int64_t out_bytes;        /* bytes per output entry: 8 (FP64) or 4 (split modes) */
    int64_t mfma_k_per_tile;  /* sum over the 16-entry output tiles of their padded contraction
                                 length: one tile of 16 cells executes mfma_k_per_tile * 512
                                 FP64 MFMA flops (split modes: * 512 BF16 flops) */
    int64_t n_tiles;          /* 16-entry output tiles */
    int64_t quad_points;      /* points of the quadrature kernel's rule */
    int64_t persistent_waves; /* waves of the persistent contraction, FP64 or split BF16 (0 = not used) */
    int64_t persistent_kmax;  /* register-resident k steps per wave of that kernel */
    int64_t tile_cells;       /* cells per workgroup tile of the contraction */
    int64_t waves;            /* waves per workgroup of the (non-persistent) contraction */
    int64_t fused_geometry;   /* 1: ffc_tabulate_tensor computes the affine map inside the
                                 contraction (one launch); 0: geometry pass first */
    int64_t g_entries;        /* G_K entries computed per cell: n_alpha, or fewer for the
                                 symmetric geometry tensors (Laplacian, weighted Laplacian,
                                 elasticity), whose two A^0 columns per unordered index pair
                                 are summed in the compile step */
    int64_t symmetric;        /* 1: the FP64 tiles hold the entries i1 <= i2 only, each result
                                 written at (i1, i2) and (i2, i1) -- the element matrices are
                                 exactly symmetric; 0: every entry computed */
    int64_t auto_launches;    /* FFC_KERNEL_AUTO forms: distinct launches the selector uses over
                                 all cell counts (the other fields describe the default tensor
                                 launch); 0 for other forms */
} ffc_form_info;

/* Compile step only, host only, touches no device: the reference tensor A^0 of the form
 * (A^0_{i alpha} = int_K0 prod dPhi/dX, Sec. 3.2; per-form expressions in Sec. 3.3).
 * Writes n_I and n_alpha; if A0 != NULL also writes A^0 row-major [n_I][n_alpha] (FP64,
 * caller-owned host buffer of n_I * n_alpha doubles).  Index conventions of alpha:
 *   mass: alpha = 0                       G = |det J|
 *   laplace: alpha = a*d + b              G = |det J| sum_k g_ak g_bk
 *   wlaplace: alpha = (t*d + a)*d + b     G = w_t |det J| sum_k g_ak g_bk
 *   elasticity: alpha = ((a*d + j)*d + b)*d + l     G = |det J| g_aj g_bl
 *   ns: alpha = (k*(d+1) + t)*d + a       G = |det J| g_ak w_{k,t}
 * with g = J^{-1} (g_ab = dX_a/dx_b). */
int ffc_compile_reference_tensor(const ffc_form_desc* desc, int64_t* n_I, int64_t* n_alpha, double* A0);

/* Compile step + upload: builds A^0, its MFMA tiles (and BF16 pieces in split modes) and
 * the quadrature tables, copies them to the current device and returns an opaque form
 * handle owned by the library (release with ffc_form_destroy).  The handle also owns a
 * geometry workspace of fixed capacity; longer tabulations are processed in chunks, so
 * the tabulation calls never allocate. */
int ffc_form_create(const ffc_form_desc* desc, ffc_form** form);
int ffc_form_get_info(const ffc_form* form, ffc_form_info* info);
void ffc_form_destroy(ffc_form* form);

/* FFC_KERNEL_AUTO forms: the candidate launch that ffc_tabulate_tensor uses for `cells`
 * cells -- its index in the selector file's candidate list (0 = the library default tensor
 * launch) -- and whether a selector file was loaded (1) or the default is used for lack of
 * one (0; from_selector may be NULL).  FFC_E_INVALID for other forms. */
int ffc_form_select(const ffc_form* form, int64_t cells, int32_t* candidate, int32_t* from_selector);

/* Enqueue the evaluation of `cells` element tensors on the form's stream and return
 * (asynchronous).  coords: device SoA as above; coeffs: device SoA or NULL; out: device
 * buffer of cells * n_I entries, double (FP64 and quadrature) or float (split modes),
 * aligned to its element size; a 16-byte aligned out takes the staged launches (whole
 * contiguous regions), any other the tile launch with direct stores (the same values;
 * FP64 bit for bit).  Nothing outside the cells * n_I entries is written.
 * cells == 0 is a no-op.  Not safe for concurrent calls on one form (shared workspace). */
int ffc_tabulate_tensor(const ffc_form* form, int64_t cells, const double* coords, const double* coeffs, void* out);

/* The contraction alone (kernel 2 above) from a precomputed affine map: affine_map is
 * the device SoA [1 + d*d][cells] that ffc_compute_geometry writes (row 0 = det J, row
 * 1 + a*d + b = g_ab).  Lets several forms on one mesh share one geometry pass (the
 * paper's eval reads the same AffineMap for every form, Sec. 5.5).  Tensor kernel only
 * (FFC_E_INVALID for a quadrature form).  Same asynchrony and layouts as
 * ffc_tabulate_tensor. */
int ffc_tabulate_tensor_affine(const ffc_form* form, int64_t cells, const double* affine_map, const double* coeffs,
                               void* out);

/* Operator action (matrix-free): y_K = A^K x_K for every cell, A^K = A^0 : G_K as in
 * ffc_tabulate_tensor (rows = test functions, Sec. 2.1), the element tensors built and used
 * on chip and never written to memory -- the matrix-free use of the tensor representation
 * that the paper points to as related work (Sec. 1).  x: device [cells][n] local vectors
 * (n = element dofs, the trial-function dofs of each cell in the element's dof order), y:
 * device [cells][n], overwritten.  FP64 tensor-kernel forms only (FFC_E_UNSUPPORTED
 * otherwise, or when the element tensors of a 16-cell tile do not fit the LDS of a CU).
 * Asynchronous on the form's stream, like ffc_tabulate_tensor; results equal A^K x_K
 * computed from ffc_tabulate_tensor's output to FP64 rounding.  Launch: the persistent
 * kernel where the form has one on 16-cell tiles, else a per-tile kernel on the form's own
 * tile_cells and waves when both were given and the tile fits, else on a shape chosen for
 * the element tensor's size.
 * Linear forms: the source term L(v) = int f v dx, f in the element's own space (Sec. 5.5),
 * has the tensor representation b_K,i = A^0_{ia} |det J| f_a with the mass form's A^0, so
 * its element vectors are this call on an FFC_MASS form with x = the cells' f dofs. */
int ffc_apply_tensor(const ffc_form* form, int64_t cells, const double* coords, const double* coeffs, const double* x,
                     double* y);

/* The geometry pass alone (kernel 1 above), for inspection: affine map of each cell as
 * SoA [1 + d*d][cells] FP64 into caller-owned device memory: row 0 = det J, row
 * 1 + a*d + b = g_ab = (J^{-1})_ab.  Asynchronous on `stream` (hipStream_t, NULL =
 * default). */
int ffc_compute_geometry(int32_t dim, int64_t cells, const double* coords, double* affine_map, void* stream);

/* Validation mode, off the hot path (which never checks the cells): the affine map of a
 * cell (Sec. 3.2, the map from the reference cell) must be invertible for its element
 * tensor to exist.  Counts the cells whose map is degenerate, |det J| <= tol * h^d with h
 * the cell's longest edge (the ratio of its volume to that of the cube on that edge, so
 * tol is scale-free; tol = 0 flags det J == 0 exactly), or whose det J is not finite.
 * coords: device SoA [(d+1)*d][cells] as for ffc_tabulate_tensor.  count, first (host, each
 * may be NULL): the number of degenerate cells and the smallest such index (-1 if none).
 * Returns FFC_E_DEGENERATE when any cell is degenerate, FFC_OK otherwise; FFC_E_INVALID
 * for cells < 0, tol < 0 or not finite, coords NULL with cells > 0; FFC_E_UNSUPPORTED for
 * dim not 2 or 3.  Allocates two device words per call and waits for `stream` (hipStream_t,
 * NULL = default) before returning. */
int ffc_check_cells(int32_t dim, int64_t cells, const double* coords, double tol, int64_t* count, int64_t* first,
                    void* stream);

/* Mixed batches (many meshes of uneven size, mixed forms and degrees; the level-3 BLAS
 * batching of Sec. 3.5 taken across meshes).  A batch is built from `n` (form, cells,
 * coords, coeffs, out) items; all forms must share one precision and use the tensor
 * kernel.  ffc_batch_run enqueues a fixed, short sequence of launches on `stream` (fit
 * for graph capture; no memset, no allocation):
 *   - items whose form uses a persistent contraction (FP64 or split BF16): one geometry
 *     pass each into a batch-owned workspace, then one persistent launch per form over
 *     the cell tiles of all its items in sequence (workgroup w takes tiles w, w + grid,
 *     ...; the form's A^0 fragments stay in registers across items);
 *   - every other item: one launch per group of items sharing a workgroup size, a cell
 *     tile size and an LDS size class, one workgroup per cell tile, geometry computed in
 *     place from the coordinates.
 * Results equal those of ffc_tabulate_tensor on each item.  The arrays are copied; the
 * device pointers must stay valid while the batch exists; runs of one batch must not
 * overlap (they share the geometry workspace).  ffc_batch_info: total cells, work units
 * (cell tiles) and the number of kernel launches one run enqueues. */
typedef struct ffc_batch ffc_batch;
int ffc_batch_create(int32_t n, const ffc_form* const* forms, const int64_t* cells, const double* const* coords,
                     const double* const* coeffs, void* const* outs, void* stream, ffc_batch** batch);
int ffc_batch_run(ffc_batch* batch);
int ffc_batch_info(const ffc_batch* batch, int64_t* total_cells, int64_t* work_units, int32_t* launches);
void ffc_batch_destroy(ffc_batch* batch);

/* Global assembly (Sec. 2.2: the element-by-element algorithm, Algorithm 2's insertion
 * step): A = sum over cells K of P_K^T A^K P_K into a CSR matrix, with the same
 * local-to-global map for test and trial functions.
 *
 * ffc_assembly_create: symbolic phase, once per mesh.  dofmap is a HOST array
 * [cells][n_local] of global dof indices in [0, n_global) (local order = the element
 * tensor's row/column order); the library builds the CSR pattern (row r = every dof sharing
 * a cell with dof r, columns ascending) and the CSR index of every element-tensor entry, on
 * the device of the current HIP context.  Fails with FFC_E_UNSUPPORTED if the pattern
 * would have 2^31 entries or more.  `stream` (hipStream_t, NULL = default) is used by
 * ffc_assemble.
 * ffc_assembly_info: rows (= n_global) and nonzeros.
 * ffc_assembly_pattern: copies the pattern to HOST arrays row_ptr [n_global + 1] (int64)
 * and col_idx [nnz] (int32).
 * ffc_assemble: numeric phase.  element_tensors: device [cells][n_local][n_local], FP64
 * (tensor_bytes 8) or FP32 (4, the split modes' output), row = test function; values:
 * device [nnz] FP64, overwritten, or added to if accumulate != 0.  Asynchronous on the
 * stream; no allocation, no memset (graph-capturable).  Each matrix row is summed by one
 * wave in a fixed order (cells ascending), without atomics: results are reproducible.
 * n_local <= 64; rows of at most 1024 entries. */
typedef struct ffc_assembly ffc_assembly;
int ffc_assembly_create(int64_t cells, int32_t n_local, const int32_t* dofmap, int64_t n_global, void* stream,
                        ffc_assembly** assembly);
int ffc_assembly_info(const ffc_assembly* assembly, int64_t* n_rows, int64_t* nnz);
int ffc_assembly_pattern(const ffc_assembly* assembly, int64_t* row_ptr, int32_t* col_idx);
int ffc_assemble(ffc_assembly* assembly, const void* element_tensors, int32_t tensor_bytes, double* values,
                 int32_t accumulate);
/* Matrix-free operator: y = A x, A = sum_K P_K^T A^K P_K the matrix ffc_assemble would
 * build from `form`'s element tensors on this assembly's mesh (Algorithm 2), without
 * forming A or the element tensors: x_K = P_K x (gather through the dofmap), y_K = A^K x_K
 * (ffc_apply_tensor), then y[r] = sum of the y_K entries of dof r in a fixed order (cells
 * ascending; no atomics).  coords / coeffs: the mesh as for ffc_tabulate_tensor, with the
 * assembly's cell count; x, y: device [n_global] FP64 (y overwritten; dofs no cell touches
 * get 0); work: caller-owned device scratch of 2 * cells * n_local doubles.  The form must
 * be an FP64 tensor-kernel form with n_local element dofs.  Asynchronous on the form's
 * stream; no allocation. */
int ffc_operator_apply(const ffc_assembly* assembly, const ffc_form* form, const double* coords, const double* coeffs,
                       const double* x, double* y, double* work);
/* ffc_operator_apply for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and the
 * same result, bit for bit, but the 2 * cells * n_local doubles of scratch (the gathered
 * local vectors and their products) live in a fixed library-owned device array of 2^24
 * doubles (128 MiB) instead of a caller's `work` buffer.  Each device the library runs on
 * holds its own copy of the array until the process ends; its address is looked up on the
 * first call on a device.  The call allocates and frees nothing.  FFC_E_UNSUPPORTED (before
 * anything is enqueued) if 2 * cells * n_local exceeds 2^24; FFC_E_INVALID if the form's
 * device is not the current device.  Every call on one device shares the array and each call
 * overwrites the part it uses: calls that overlap on one device (other streams, other
 * threads) race and must be serialised by the caller. */
int ffc_operator_apply_noalloc(const ffc_assembly* assembly, const ffc_form* form, const double* coords,
                               const double* coeffs, const double* x, double* y);
void ffc_assembly_destroy(ffc_assembly* assembly);

/* Kernel selector network.  A multilayer perceptron that predicts the log run time of each
 * candidate launch (tensor or quadrature kernel, launch shape) of a tabulation from its
 * features (form rank, degree, |i|, |alpha|, dimension, cells); the candidate with the
 * smallest prediction is chosen -- the automatic choice between tensor representation
 * and quadrature that Sec. 4.4 leaves to future work.  It is trained on the GPU with these
 * kernels (FP32):
 *   y = relu(relu(x W1 + b1) W2 + b2) W3 + b3,
 * parameters in one flat array: W1 [n_in][n_hidden], b1 [n_hidden], W2 [n_hidden][n_hidden],
 * b2 [n_hidden], W3 [n_hidden][n_out], b3 [n_out] (ffc_mlp_param_count floats).
 * All pointers are device pointers, caller-owned; calls are asynchronous on `stream`. */
int64_t ffc_mlp_param_count(int32_t n_in, int32_t n_hidden, int32_t n_out);
/* x [batch][n_in] -> y [batch][n_out]; act (workspace, 2*batch*n_hidden floats) keeps the two
 * hidden activations for the backward pass. */
int ffc_mlp_forward(int32_t n_in, int32_t n_hidden, int32_t n_out, int64_t batch, const float* params,
                    const float* x, float* act, float* y, void* stream);
/* Gradient of a loss with dL/dy = dy [batch][n_out] w.r.t. the parameters, written to grad
 * (ffc_mlp_param_count floats); act from the forward pass; work: 2*batch*n_hidden floats. */
int ffc_mlp_backward(int32_t n_in, int32_t n_hidden, int32_t n_out, int64_t batch, const float* params,
                     const float* x, const float* act, const float* dy, float* grad, float* work, void* stream);
/* Masked mean squared error over n values: loss[0] = sum m (y - t)^2 / sum m,
 * dy = 2 m (y - t) / sum m. */
int ffc_mlp_mse(int64_t n, const float* y, const float* target, const float* mask, float* dy, float* loss,
                void* stream);
/* One Adam step (bias-corrected, step >= 1) on n parameters with gradient g and moments m, v;
 * weight_decay adds the L2 term weight_decay * params to the gradient first (0 = plain Adam). */
int ffc_adam_step(int64_t n, float* params, const float* grad, float* m, float* v, float lr, float beta1,
                  float beta2, float eps, float weight_decay, int32_t step, void* stream);

/* Message of the last failing call on this thread ("" if none). */
const char* ffc_last_error(void);

/* Library version string. */
const char* ffc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FFC_HIP_H */
