/*
 * h2mg.h -- C ABI of the MI355X H2 matrix and H2-MG solver library.
 *
 * The library builds an H2 approximation A_H2 of a dense SPD kernel matrix
 * A_ij = k(|p_i - p_j|) (+ shift on the diagonal) from points and a kernel,
 * multiplies by it, and solves A_H2 x = b by the H2-MG V-cycle.
 *
 * Paper: Sushnikova, Turkiyyah, Chow, Keyes, "H2-MG: A multigrid method for
 * hierarchical rank structured matrices".
 *   - H2 representation and matvec: Section 3.1 (eq. f, eq. h20, eq. s1,
 *     eq. h2, and the matvec recursion that follows eq. h2).
 *   - Restricted operators: Section 3.3 (eq. a2_str).
 *   - V-cycle: Section 3.3, Algorithm 1; smoother Iter = CG.
 *   - Kernels: Section 4 (eq. a_gau, eq. a_exp).
 *
 * Conventions shared by every entry point
 *   - Every call returns an h2mg_status; no exception crosses the ABI.  On
 *     failure h2mg_last_error() returns a thread-local message that stays
 *     valid until the next call on the same thread.
 *   - "device" pointers are HIP device allocations on the current device;
 *     "host" pointers are ordinary host memory.  The caller owns every
 *     pointer it passes; the library copies what it keeps.
 *   - Points are n x dim row-major FP64 in user order.  Vectors passed to
 *     h2mg_matvec / h2mg_solve are length-n FP64 in user order (the library
 *     permutes to tree order internally).
 *   - Coefficient vectors of coarse level k >= 2 (tree depth d = L - k + 2)
 *     are cluster-major: 2^d clusters of r coefficients each, clusters in
 *     tree order.
 *   - Device work is enqueued on the given stream (0 = null stream).
 *     h2mg_matvec, h2mg_level_apply, h2mg_restrict and h2mg_prolong do not
 *     block the host.  h2mg_build, h2mg_setup_mg, h2mg_vcycle and
 *     h2mg_solve synchronise the stream before returning.
 *   - A handle is not thread-safe: calls on one handle must not overlap.
 */
#ifndef H2MG_H_
#define H2MG_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum h2mg_status {
  H2MG_OK = 0,
  H2MG_ERR_INVALID_ARG = 1,   /* bad size, parameter, null or non-finite input */
  H2MG_ERR_OOM = 2,           /* device or host allocation failed */
  H2MG_ERR_HIP = 3,           /* a HIP runtime call failed */
  H2MG_ERR_NOT_SPD = 4,       /* p^T A p <= 0 in CG or a Cholesky pivot <= 0 */
  H2MG_ERR_NOT_CONVERGED = 5, /* cycle cap reached; x holds the last iterate */
  H2MG_ERR_NUMERIC = 6,       /* NaN/Inf met during a solve */
  H2MG_ERR_STATE = 7          /* calls in the wrong order */
} h2mg_status;

/* Kernel families (Section 4: exponential eq. a_exp, Gaussian eq. a_gau;
 * Matern-3/2 in addition).  k(0) = 1 for all, and the diagonal of A is
 * k(0) + shift (the paper's 1 + c).
 *   H2MG_KERNEL_EXP:      k(r) = exp(-r / l)
 *   H2MG_KERNEL_GAUSS:    k(r) = exp(-r^2 / (2 l^2))   (paper's sigma = 2 l^2)
 *   H2MG_KERNEL_MATERN32: k(r) = (1 + sqrt(3) r / l) exp(-sqrt(3) r / l) */
typedef enum h2mg_kernel_kind {
  H2MG_KERNEL_EXP = 0,
  H2MG_KERNEL_GAUSS = 1,
  H2MG_KERNEL_MATERN32 = 2,
  H2MG_KERNEL_LAPLACE = 3      /* 1 / (4 pi r), 0 at r = 0 (Section 4.3); no
                                  length scale; use with a per-point diagonal */
} h2mg_kernel_kind;

/* Derivative kernels, for the gradient of L = b^T A^{-1} b (not in the
 * paper; the gradient follows from its problem statement A x = b with
 * A = K(p; l) + s I): the profile dk/dl at fixed r, or g(r) = k'(r) / r,
 * through which grad_{p_i} k(|p_i - p_j|) = g(r_ij) (p_i - p_j).  g is 0 at
 * r = 0 (its self term cancels in the gradient). */
typedef enum h2mg_kernel_derivative {
  H2MG_KERNEL_VALUE = 0,
  H2MG_KERNEL_D_LENGTH = 1,
  H2MG_KERNEL_D_RADIAL = 2
} h2mg_kernel_derivative;

typedef struct h2mg_kernel {
  int32_t kind;          /* h2mg_kernel_kind */
  double length_scale;   /* l > 0 */
  double shift;          /* >= 0, added to the diagonal */
  int32_t derivative;    /* h2mg_kernel_derivative, 0 for the kernel itself */
} h2mg_kernel;

/* Cluster tree and bases (Section 3.1).  Binary tree of uniform depth
 * L = min{L : leaf_size * 2^L >= n}, median split along the longest side of
 * each cluster's tight box; a pair of clusters is far (admissible) when its
 * boxes are apart and max(diam) <= eta * dist; bases are tensor Chebyshev
 * interpolants with cheb_m nodes per axis, rank r = cheb_m^dim.
 * Requires r <= 64 and every leaf to hold at least r points. */
typedef struct h2mg_build_opts {
  int32_t leaf_size;     /* >= 1 */
  double eta;            /* > 0 */
  int32_t cheb_m;        /* >= 1 */
} h2mg_build_opts;

typedef enum h2mg_precision {
  H2MG_FP64 = 0,         /* every step in FP64 */
  H2MG_FP32_IR = 1,      /* V-cycle on FP32 operators inside FP64 refinement */
  H2MG_BF16_IR = 2       /* V-cycle on BF16 operators inside FP64 refinement */
} h2mg_precision;

/* Smoothers (Iter in Algorithm 1).  H2MG_SMOOTHER_CG: plain CG, the paper's
 * choice (Section 3.3).  H2MG_SMOOTHER_BLOCK_JACOBI: CG preconditioned by the
 * inverse diagonal blocks of each level's operator -- the leaf blocks
 * K_ss + shift*I on the finest level (requires leaves of at most 128
 * points), the projected diagonal blocks on coarser levels. */
typedef enum h2mg_smoother {
  H2MG_SMOOTHER_CG = 0,
  H2MG_SMOOTHER_BLOCK_JACOBI = 1
} h2mg_smoother;

/* Solver options (Section 3.3, Algorithm 1 and the remark on fine and
 * coarse iterations).  n_fine / n_coarse smoothing steps pre and post on
 * the finest / coarser levels; the solve stops when
 * ||b - A_H2 x||_2 / ||b||_2 < rtol, measured in FP64, or after max_cycles
 * V-cycles (FP64) or refinement steps (mixed forms, one V-cycle each). */
/* Solver method.  V: Algorithm 1 repeated (Section 3.3).  W and F: the
 * other cycles named after Algorithm 1, in their textbook recursive forms
 * (after the first coarse correction of a level, a second one on the
 * remaining coarse residual by a W-cycle, resp. a V-cycle; skipped when the
 * coarse level is the directly solved one).  CG: the comparison solver of
 * the experiments (Section 4), CG on A_H2 alone in FP64 (block-Jacobi PCG
 * with the block smoother), stopped on the recurrence residual; there
 * max_cycles counts CG iterations. */
typedef enum h2mg_method {
  H2MG_METHOD_V_CYCLE = 0,
  H2MG_METHOD_W_CYCLE = 1,
  H2MG_METHOD_F_CYCLE = 2,
  H2MG_METHOD_CG = 3
} h2mg_method;

typedef struct h2mg_solve_opts {
  int32_t n_fine;        /* >= 0, paper default 1 */
  int32_t n_coarse;      /* >= 0, paper default 40 */
  double rtol;           /* > 0, e.g. 1e-8 */
  int32_t max_cycles;    /* >= 0 (CG iterations for H2MG_METHOD_CG) */
  int32_t precision;     /* h2mg_precision (FP64 only for H2MG_METHOD_CG) */
  int32_t use_x0;        /* 1: x holds the initial guess; 0: start from 0 */
  int32_t smoother;      /* h2mg_smoother */
  int32_t method;        /* h2mg_method, default 0 (V-cycles) */
} h2mg_solve_opts;

typedef struct h2mg_solve_info {
  int32_t cycles;        /* cycles (refinement steps, CG iterations) performed */
  int32_t converged;     /* 1 if the residual test passed */
  double rel_residual;   /* final ||b - A_H2 x|| / ||b|| in FP64 */
  double solve_seconds;  /* wall time of the solve on the host clock */
  int32_t history_len;   /* entries available from h2mg_solve_history */
} h2mg_solve_info;

/* ------------------------------------------------------------------ plan
 * Host-side cluster tree and block partition (no device work).  Exposed so
 * the structure can be inspected and tested without a GPU. */
typedef struct h2mg_plan_s* h2mg_plan_t;

typedef struct h2mg_plan_info {
  int64_t n;             /* number of points */
  int32_t dim;
  int32_t depth;         /* leaf depth L */
  int32_t d_top;         /* shallowest depth with a far pair, -1 if none */
  int32_t rank;          /* r = cheb_m^dim */
  int32_t leaf_min;      /* smallest and largest leaf size */
  int32_t leaf_max;
} h2mg_plan_info;

/* Build the tree and partition of `points_host` (n x dim, host, user order).
 * Errors: INVALID_ARG for n < 1, dim not in {1,2,3}, leaf_size < 1,
 * eta <= 0 or non-finite, cheb_m < 1, r > 64, non-finite coordinates, or a
 * leaf with fewer than r points; OOM.  *out must be freed with
 * h2mg_plan_destroy. */
h2mg_status h2mg_plan_create(const double* points_host, int64_t n, int32_t dim,
                             const h2mg_build_opts* opts, h2mg_plan_t* out);
h2mg_status h2mg_plan_query(h2mg_plan_t plan, h2mg_plan_info* info);
/* perm_host[k] = user index at tree position k (n entries). */
h2mg_status h2mg_plan_perm(h2mg_plan_t plan, int64_t* perm_host);
/* offsets_host[j] = first tree position of cluster j at `depth`
 * (2^depth + 1 entries). */
h2mg_status h2mg_plan_offsets(h2mg_plan_t plan, int32_t depth, int64_t* offsets_host);
/* Number of near (which = 0) or far (which = 1) cluster pairs at `depth`,
 * counting both (s, t) and (t, s). */
h2mg_status h2mg_plan_pair_count(h2mg_plan_t plan, int32_t depth, int32_t which,
                                 int64_t* count);
/* The pairs themselves, sorted by (s, t): pairs_host[2i] = s, [2i+1] = t. */
h2mg_status h2mg_plan_pairs(h2mg_plan_t plan, int32_t depth, int32_t which,
                            int64_t* pairs_host);
void h2mg_plan_destroy(h2mg_plan_t plan);

/* ------------------------------------------------------------------ H2 */
typedef struct h2mg_h2_s* h2mg_h2_t;

/* Build A_H2 from `points_dev` (device, n x dim FP64, user order) and the
 * kernel (Section 3.1): tree and partition on the host, then on the device
 * the orthonormal nested bases (leaf bases Q, transfers E), and the
 * orthogonalised far couplings S of every depth.  Near leaf blocks are
 * evaluated on the fly in every product unless h2mg_store_near stores them.
 * Errors as h2mg_plan_create, plus INVALID_ARG for a null pointer or a bad
 * kernel, OOM, HIP.  Blocks until
 * the build is complete. */
h2mg_status h2mg_build(const double* points_dev, int64_t n, int32_t dim,
                       const h2mg_kernel* kernel, const h2mg_build_opts* opts,
                       hipStream_t stream, h2mg_h2_t* out);

/* As h2mg_build, for the scaled form diag(s) K diag(s) + diag(d): scale_dev
 * (s > 0) and diag_dev (d, replacing the kernel's constant shift) are
 * device arrays of n doubles in user order, either may be null (s = 1,
 * d = shift).  s multiplies the rows of the leaf bases before their
 * orthonormalisation, so the restricted operators of the hierarchy are those
 * of the scaled matrix.  This is the symmetric W^(1/2) G W^(1/2) form of the
 * boundary-element matrix of Section 4.3 (see h2mg_bem_panels).  Errors as
 * h2mg_build, plus INVALID_ARG for s <= 0 or a non-finite s or d. */
h2mg_status h2mg_build_scaled(const double* points_dev, int64_t n, int32_t dim,
                              const h2mg_kernel* kernel, const h2mg_build_opts* opts,
                              const double* scale_dev, const double* diag_dev,
                              hipStream_t stream, h2mg_h2_t* out);

/* Boundary elements of the Laplace single layer (Section 4.3), for a flat
 * triangle mesh: vertices_dev (nv x 3 doubles), triangles_dev (nt x 3
 * int64 vertex indices), both device.  Writes, per triangle i, the centroid
 * (collocation point) to centroids_dev (nt x 3), s_i = sqrt(area_i) to
 * scale_dev and the diagonal entry d_i = I_i / (4 pi) to diag_dev, where I_i
 * is the integral of 1/|y_i - y| over the triangle (closed form).  The
 * paper's regularised entry area_i / (4 pi R_i) is not used: it leaves the
 * matrix indefinite on curved surfaces.  With these, h2mg_build_scaled
 * with H2MG_KERNEL_LAPLACE builds S = W^(1/2) G W^(1/2), and the density
 * of the paper's system A sigma = f is sigma = W^(-1/2) y for S y =
 * W^(1/2) f.  Indices are not checked beyond nt > 0 and nv > 0. */
h2mg_status h2mg_bem_panels(const double* vertices_dev, int64_t nv, const int64_t* triangles_dev,
                            int64_t nt, double* centroids_dev, double* scale_dev,
                            double* diag_dev, hipStream_t stream);
/* The seven-point near field of the boundary-element benchmark: Radon's
 * rule (exact for polynomials of degree <= 5) on every triangle.  Writes
 * qy_dev (nt x 7 x 3 doubles: the rule's points) and qu_dev (nt x 7:
 * the rule's weights times sqrt(area_i)).  Passed to
 * h2mg_set_near_quadrature, the close entries of the symmetric form become
 * the rule applied on both triangles to the double integral of
 * 1 / (4 pi |x - y|), divided by s_i s_j -- the reading of a 7-point
 * near-field rule that keeps the operator symmetric (Section 4.3 gives only
 * the one-point collocation entry).  Same arguments and errors as
 * h2mg_bem_panels. */
h2mg_status h2mg_bem_quadrature7(const double* vertices_dev, int64_t nv, const int64_t* triangles_dev,
                                 int64_t nt, double* qy_dev, double* qu_dev, hipStream_t stream);
/* rhs_dev[i] = s_i / (4 pi |y_i - x0|): W^(1/2) f for the point source x0
 * (3 host doubles) of Section 4.3; centroids and scale from h2mg_bem_panels. */
h2mg_status h2mg_bem_point_source_rhs(const double* centroids_dev, const double* scale_dev,
                                      int64_t n, const double* x0_host, double* rhs_dev,
                                      hipStream_t stream);
/* rhs_dev[i] = s_i * sum_k c_k h_k(y_i): W^(1/2) f for a right-hand side
 * given by a harmonic polynomial (the Dirichlet data of a harmonic
 * function, as in the boundary-element benchmark), with the harmonic basis
 * of degree <= 2 in 3D, h = (1, x, y, z, xy, yz, zx, x^2 - y^2,
 * x^2 + y^2 - 2 z^2) and coeffs_host = (c_0 .. c_8) (9 host doubles).
 * Errors: INVALID_ARG (null, n < 1, a non-finite coefficient). */
h2mg_status h2mg_bem_harmonic_rhs(const double* centroids_dev, const double* scale_dev, int64_t n,
                                  const double* coeffs_host, double* rhs_dev, hipStream_t stream);
/* sigma_dev[i] = y_dev[i] / s_i: the density of the paper's system from the
 * solution of the symmetric one. */
h2mg_status h2mg_bem_density(const double* y_dev, const double* scale_dev, int64_t n,
                             double* sigma_dev, hipStream_t stream);

/* y = A_H2 x (Section 3.1 matvec: upsweep x_i = V_i x_{i-1}, couplings,
 * downsweep y_{i-1} = D_i x_{i-1} + U_i y_i, near field y = D x + U_1 y_1).
 * x_dev, y_dev: device, length n, user order; they must not overlap. */
/* Close entries by quadrature (Section 3.1's close blocks D, evaluated with
 * a quadrature rule instead of point values): point i carries nq
 * sub-points qy_dev[i] (nq x dim doubles, row-major) with weights
 * qu_dev[i] (nq doubles), both device, user order, copied by the call; the
 * entry between distinct points i, j of a close leaf pair becomes
 * sum_p sum_q qu[i][p] qu[j][q] k(|qy[i][p] - qy[j][q]|), the diagonal
 * keeps d (or the shift), and far blocks keep the point values.  Must be
 * called right after the build (before any product, store or setup); it
 * stores the near field (as h2mg_store_near, which cannot release it
 * afterwards), and every product reads the stored tiles -- FP64, or an FP32
 * copy that h2mg_setup_mg makes for the low precisions.  Errors:
 * INVALID_ARG (null, nq outside 1..64), STATE (called after a product or
 * setup, or twice), OOM, HIP. */
h2mg_status h2mg_set_near_quadrature(h2mg_h2_t h, const double* qy_dev, const double* qu_dev,
                                     int32_t nq, hipStream_t stream);

h2mg_status h2mg_matvec(h2mg_h2_t h, const double* x_dev, double* y_dev,
                        hipStream_t stream);

/* Build the H2 matrix of a derivative kernel (`which` = H2MG_KERNEL_D_LENGTH
 * or H2MG_KERNEL_D_RADIAL, shift 0) on the same points, tree, partition and
 * Chebyshev bases as `h` (same kernel kind and length scale).  *out must be
 * destroyed with h2mg_destroy.  Errors: INVALID_ARG (bad which, null), OOM,
 * HIP.  Blocks until the build is complete. */
h2mg_status h2mg_build_derivative(h2mg_h2_t h, int32_t which, hipStream_t stream,
                                  h2mg_h2_t* out);

/* Loss L = b^T x and its gradient for x = A^{-1} b (x from h2mg_solve on h):
 *   dL/dl = -x^T (dA/dl) x,  dL/ds = -x^T x,
 *   dL/dp_ia = -2 x_i [p_ia (G x)_i - (G (x * p_.a))_i],  dL/db = 2 x,
 * with dA/dl and G = [g(r_ij)] the H2 matrices h_dl and h_g from
 * h2mg_build_derivative on h (A symmetric, so the adjoint solve is the
 * forward solve).  Every gradient output is multiplied by `scale` (the
 * incoming gradient of an autodiff chain; 1 for the plain gradient).
 * b_dev, x_dev: device, length n, user order.  grad_points_dev: device,
 * n x dim row-major, user order, or null to skip the 1 + dim products with
 * G; grad_b_dev: device, length n, or null.  Host outputs may be null; h_dl
 * may be null when grad_length is, h_g when grad_points_dev is.  Errors:
 * INVALID_ARG (null handle or vector, a derivative handle missing, of the
 * wrong kind or built on other points), HIP. */
h2mg_status h2mg_quadratic_gradient(h2mg_h2_t h, h2mg_h2_t h_dl, h2mg_h2_t h_g,
                                    const double* b_dev, const double* x_dev, double scale,
                                    double* loss, double* grad_length, double* grad_shift,
                                    double* grad_points_dev, double* grad_b_dev,
                                    hipStream_t stream);

/* Store the near field (Section 3.1: the dense close leaf blocks D of the
 * matvec y = D x + U_1 y_1).  enable != 0 evaluates every close leaf pair
 * once, as 64 x 64 FP64 tiles between chunks of at most 64 points of a leaf
 * (upper triangle of the symmetric operator; at n = 2^20 with leaf 128 this
 * is 126 GB), and every later FP64 fine-level product (h2mg_matvec,
 * level 1 of h2mg_level_apply, the FP64 residuals and smoothing of
 * h2mg_solve) streams those tiles instead of evaluating the kernel.  FP32 and
 * BF16 products keep evaluating the near field.  enable == 0 releases the
 * tiles.  Results agree with the evaluated near field up to rounding order.
 * Errors: OOM (nothing is kept; the evaluated near field stays in use), HIP.
 * Blocks until the tiles are complete. */
h2mg_status h2mg_store_near(h2mg_h2_t h, int32_t enable, hipStream_t stream);

/* Y = A_H2 X for a block of 1 <= nrhs <= 16 vectors (the Section 3.1 matvec
 * applied column by column, computed for all columns at once): x_dev and
 * y_dev are device, row-major n x ldx and n x ldy (entry (i, k) of user row
 * i at i * ld + k), ld >= nrhs.  FP64.  The r x r and near-field tile
 * products run 16 columns at a time on the matrix cores; each stored tile is
 * read at most twice per product (once for its block row, once for its
 * block column, transposed), so the product streams at most twice the bytes
 * of a single matvec for up to 16 of them.  The near-field tiles are the
 * stored ones after h2mg_store_near, else they are evaluated from the points
 * inside the product (64 x 64 tiles between chunks of at most 64 points of a
 * leaf; no near-field storage).  Requires 9 <= r <= 64.  Results equal 16
 * single products up to rounding order.  Errors: INVALID_ARG (null, nrhs or
 * ld out of range, rank out of range), OOM (about 1 GB of block buffers per
 * 2^20 points, plus 8 KB per tile task, allocated on first use and kept),
 * HIP. */
h2mg_status h2mg_matvec_multi(h2mg_h2_t h, int32_t nrhs, const double* x_dev, int32_t ldx,
                              double* y_dev, int32_t ldy, hipStream_t stream);

/* Solve A_H2 X = B for a block of 1 <= nrhs <= 16 right-hand sides: every
 * step of the cycles of h2mg_solve (Algorithm 1, Section 3.3: smoother,
 * restriction, prolongation, coarse Cholesky solve; FP64, or FP64 iterative
 * refinement around an FP32 or BF16 cycle) applied to all columns at once,
 * with the CG scalars of the smoother and the stopping test kept per column
 * (cycles run until every column's FP64 relative residual is below rtol).
 * b_dev, x_dev: device, row-major n x ldb and n x ldx, user order.  Stored
 * tiles are multiplied 16 columns at a time on the matrix cores.  The
 * near-field tiles of the FP64 products are the stored ones after
 * h2mg_store_near, else evaluated from the points inside each product; the
 * FP32 and BF16 cycles always evaluate them, in FP32 (BF16 rounding of the
 * close blocks, which hold the diagonal, can make the operator indefinite).
 * opts->method: V, W or F cycles.  info: cycles run, converged (all
 * columns), the largest column residual, time.  col_residuals: host, nrhs
 * entries (final relative residual of each column), or null.  Requires
 * 9 <= r <= 64; runs h2mg_setup_mg itself when needed.  Errors: as
 * h2mg_solve, plus INVALID_ARG (nrhs, ld or rank out of range, method
 * CG). */
h2mg_status h2mg_solve_multi(h2mg_h2_t h, int32_t nrhs, const double* b_dev, int32_t ldb,
                             double* x_dev, int32_t ldx, const h2mg_solve_opts* opts,
                             h2mg_solve_info* info, double* col_residuals, hipStream_t stream);

/* Independent problems solved together (many right-hand sides of many
 * problems of uneven size): problem i is h2mg_solve_multi on handle hs[i]
 * with nrhs[i] columns b_dev[i] / x_dev[i] (leading dimensions ldb[i],
 * ldx[i]), all with the same opts.  The problems are spread over nstreams
 * streams of their own (0: 4), and each problem's next cycle is enqueued as
 * soon as its own residual has been read, so small and large problems keep
 * the device busy together; with h2mg_set_graphs on a handle its cycles are
 * graph launches.  Every stream first waits for the work already enqueued
 * on `stream`; the call returns when every problem has finished.  Handles
 * must be distinct.  infos, statuses: host arrays of nprob entries (each
 * problem's info and status), or null.  Returns the status of the first
 * failing problem (the others still run to their end); errors as
 * h2mg_solve_multi. */
h2mg_status h2mg_solve_batch(int32_t nprob, const h2mg_h2_t* hs, const int32_t* nrhs,
                             const double* const* b_dev, const int32_t* ldb, double* const* x_dev,
                             const int32_t* ldx, const h2mg_solve_opts* opts,
                             h2mg_solve_info* infos, h2mg_status* statuses, int32_t nstreams,
                             hipStream_t stream);

/* The problems of h2mg_solve_batch solved in one sequence of launches on
 * `stream` (Algorithm 1 for every problem, batched over problems): the
 * problems advance cycle by cycle together, and each tile product of a
 * cycle step -- the couplings, the restricted operators of each level, the
 * near-field tiles -- is one kernel launch over the task lists of every
 * active problem (up to 16 per launch; problems whose level does not exist
 * at that step are left out, and a problem's coarsest level is solved
 * directly when the others go deeper).  Vector steps stay per problem, on
 * up to four lane streams that fork from and join back into `stream`
 * around each group launch.  A problem's arithmetic is the same, in the
 * same order, as in its own h2mg_solve_multi, so results are bitwise equal.
 * With h2mg_set_graphs on every handle, the first cycle of each set of
 * active problems runs kernel by kernel; the set's cycle is captured as one
 * graph when it repeats, and only if that first cycle was launch-bound (its
 * enqueue took at least twice its GPU time).  Arguments, ownership and
 * errors as h2mg_solve_batch. */
h2mg_status h2mg_solve_group(int32_t nprob, const h2mg_h2_t* hs, const int32_t* nrhs,
                             const double* const* b_dev, const int32_t* ldb, double* const* x_dev,
                             const int32_t* ldx, const h2mg_solve_opts* opts,
                             h2mg_solve_info* infos, h2mg_status* statuses, hipStream_t stream);

/* Build the H2-MG hierarchy (Section 3.3): restricted operators
 * A_k = U_{k-1}^T A_{k-1} V_{k-1}^T for every level, i.e. the projected close
 * blocks of eq. a2_str at every depth, the dense coarsest operator A_l and
 * its FP64 Cholesky factor.  precision_mask bit 1 (value 2) also prepares
 * FP32 copies of the operators, bit 2 (value 4) BF16 copies; FP64 is always
 * built.  Errors: NOT_SPD if a Cholesky pivot of A_l is <= 0; OOM; HIP.
 * Calling it again only adds missing precisions. */
h2mg_status h2mg_setup_mg(h2mg_h2_t h, int32_t precision_mask, hipStream_t stream);

/* Number of MG levels l (1 when there is no far block: then A_1 is solved
 * directly) and the size N_k of level k (1-based; N_1 = n). */
h2mg_status h2mg_level_count(h2mg_h2_t h, int32_t* levels);
h2mg_status h2mg_level_size(h2mg_h2_t h, int32_t level, int64_t* size);

/* y = A_k x on level k (level 1: x, y in user order, same as h2mg_matvec;
 * level >= 2: coefficient order).  Requires h2mg_setup_mg for level >= 2. */
h2mg_status h2mg_level_apply(h2mg_h2_t h, int32_t level, const double* x_dev,
                             double* y_dev, hipStream_t stream);
/* y = A_k x with the level's operators in the given h2mg_precision, the
 * product the low-precision V-cycles apply (Section 3.3, eq. a2_str, for
 * level >= 2; Section 3.1 for level 1): FP32 or BF16 bases, transfers,
 * couplings and projected blocks, the level-1 near field evaluated in FP32,
 * FP32 vectors and FP32 accumulation.  x and y are FP64 device vectors of
 * N_k elements (user order on level 1, coefficient order above); x is
 * rounded to FP32 on entry and y widened from FP32 on exit.  The handle
 * allocates two FP32 vectors of N_k for the call.  Errors: INVALID_ARG for a
 * bad level or precision, STATE when h2mg_setup_mg has not prepared that
 * precision (level >= 2, or any level for a non-FP64 precision); OOM; HIP. */
h2mg_status h2mg_level_apply_precision(h2mg_h2_t h, int32_t level, int32_t precision,
                                       const double* x_dev, double* y_dev, hipStream_t stream);
/* Restriction r_{k+1} = U_k^T r_k and prolongation e_k = V_k^T e_{k+1} = U_k e_{k+1}
 * between levels k and k+1 (Algorithm 1).  Level 1 vectors in user order. */
h2mg_status h2mg_restrict(h2mg_h2_t h, int32_t level, const double* r_dev,
                          double* r_next_dev, hipStream_t stream);
h2mg_status h2mg_prolong(h2mg_h2_t h, int32_t level, const double* e_next_dev,
                         double* e_dev, hipStream_t stream);

/* The smoother alone, e = Iter(A_k, r, e0) of Algorithm 1 (Section 3.3):
 * nsteps of CG (smoother 0) or block-Jacobi PCG (smoother 1) on level
 * `level` in FP64, from e0 = e_dev on entry when use_e0 != 0, else from 0.
 * Level 1 vectors in user order (length n), coarser levels in coefficient
 * order (h2mg_level_size).  Runs h2mg_setup_mg itself when needed.  Errors:
 * INVALID_ARG (null, level out of range, bad smoother, the block smoother on
 * the coarsest level), NOT_SPD, OOM, HIP. */
h2mg_status h2mg_smooth(h2mg_h2_t h, int32_t level, const double* r_dev, double* e_dev,
                        int32_t nsteps, int32_t smoother, int32_t use_e0, hipStream_t stream);

/* One V-cycle of Algorithm 1 in FP64: x_out = x0 + e_1 for A_H2 x = b
 * (a W- or F-cycle when opts->method says so; H2MG_METHOD_CG is
 * INVALID_ARG here).  All vectors device, length n, user order; x_out may
 * alias x0. */
h2mg_status h2mg_vcycle(h2mg_h2_t h, const double* x0_dev, const double* b_dev,
                        double* x_out_dev, const h2mg_solve_opts* opts,
                        hipStream_t stream);

/* Solve A_H2 x = b by repeated V-cycles (FP64) or FP64 iterative refinement
 * around a low-precision V-cycle (opts->precision).  b_dev, x_dev: device,
 * length n, user order.  Runs h2mg_setup_mg itself when needed.  Errors:
 * NOT_CONVERGED (x holds the last iterate, info filled), NOT_SPD, NUMERIC,
 * INVALID_ARG (null, bad options, non-finite b).  info may be null. */
h2mg_status h2mg_solve(h2mg_h2_t h, const double* b_dev, double* x_dev,
                       const h2mg_solve_opts* opts, h2mg_solve_info* info,
                       hipStream_t stream);

/* Bytes of the fixed device scratch region of h2mg_solve_noalloc. */
#define H2MG_SOLVE_SCRATCH_BYTES (256ull * 1024ull * 1024ull)

/* h2mg_solve for callers that cannot allocate device memory (tight serving
 * loops, code that must not call hipMalloc): the same solve, arguments and
 * results, with no device allocation or free in the call.  Its vectors (the
 * per-level residuals and corrections, the CG temporaries, tree-ordered b
 * and x) are carved from a fixed region of H2MG_SOLVE_SCRATCH_BYTES in
 * device memory that the library holds on every GPU it runs on until the
 * process ends; cycles are launched kernel by kernel (no graphs).  The
 * region needs about 8 (2 sum_k N_k + 7 n) bytes in FP64 plus half that
 * again for a mixed precision (N = 2^20: about 130 MB); a larger problem is
 * INVALID_ARG, with the bytes it needs in the message.  Everything a solve
 * builds on first use must already exist: h2mg_setup_mg with the
 * precision's bit, and for the block smoother its inverses (built by one
 * h2mg_solve with that smoother and precision); otherwise STATE.  Every
 * call on one GPU uses the same region, which keeps the previous call's
 * contents (no vector is read before the solve writes it): calls that
 * overlap on one GPU, from any handle or stream, race and must be
 * serialised by the caller.  Other errors as h2mg_solve. */
h2mg_status h2mg_solve_noalloc(h2mg_h2_t h, const double* b_dev, double* x_dev,
                               const h2mg_solve_opts* opts, h2mg_solve_info* info,
                               hipStream_t stream);
/* Relative residual before each cycle of the last solve, then at exit
 * (host array of at least `capacity` doubles; copies min(capacity, len)). */
h2mg_status h2mg_solve_history(h2mg_h2_t h, double* history_host, int32_t capacity);

/* Cycle graphs.  When enabled, h2mg_solve records the launches of one cycle
 * (V/W/F-cycle and the update of x, not the FP64 residual and its norm) into
 * a HIP graph on a private stream the first time and then launches that
 * graph once per cycle into the caller's stream; the arithmetic is the same
 * launch for launch, so results are bitwise those of the direct launches.
 * Ignored while kernel timing is enabled and by H2MG_METHOD_CG.  Off by
 * default. */
h2mg_status h2mg_set_graphs(h2mg_h2_t h, int32_t enabled);

/* Tile-run tuning of the 16-column products (h2mg_matvec_multi,
 * h2mg_solve_multi, h2mg_solve_batch).  Their tile products run as tasks of
 * consecutive tiles of one block row (or column); a longer run means fewer
 * partial results to reduce, a shorter one more parallel tasks.  With tuning
 * on, every task set (the couplings of the fine level, the near-field
 * chunk tiles, the restricted operator of every depth) is built for each
 * run length in {2, 4, 8, 16, 32}, its product plus reduce is timed with HIP
 * events on this device, and the fastest is kept.  Off by default (run 8).
 * Changing the setting drops the block buffers, which are rebuilt (and, if
 * on, tuned) at the next 16-column call. */
h2mg_status h2mg_set_autotune(h2mg_h2_t h, int32_t enabled);
/* The run length in use for a task set (which = -2: near field, -1: fine-level
 * couplings, d >= 0: restricted operator of depth d), its measured time in
 * ms per product + reduce (0 when not tuned) and the tiles one product reads
 * (every tile once for its block row, the off-diagonal ones again for their
 * block column); run = 0 when that set has not been built yet.  Errors:
 * INVALID_ARG (null, which out of range). */
h2mg_status h2mg_block_tuning(h2mg_h2_t h, int32_t which, int32_t* run, double* ms, int64_t* tiles_read);

/* Kernel timing, for measurement harnesses.  While enabled, every launch of
 * the block GEMV and of the near-field kernel is bracketed by HIP events on
 * the handle's stream (a small per-launch overhead).  h2mg_set_timing
 * resets the counters.  h2mg_kernel_stats synchronises the stream and
 * returns, for kind 0/1/2 (block GEMV with FP64/FP32/BF16 blocks), the
 * number of launches, their summed duration in ms and the algorithmic bytes
 * they streamed (stored block words x element size); for kind 3/4 (near
 * field evaluated in FP64/FP32) the summed kernel evaluations instead of
 * bytes; for kind 5 (block GEMV over the stored FP64 near-field tiles) the
 * bytes of the tiles it streamed; for kind 6 (both passes of the FP64
 * 16-column tile product over the near-field tiles) the bytes of the tiles
 * read by the two passes. */
h2mg_status h2mg_set_timing(h2mg_h2_t h, int32_t enabled);
h2mg_status h2mg_kernel_stats(h2mg_h2_t h, int32_t kind, int64_t* launches, double* total_ms,
                              double* total_work);

/* The block-GEMV launch of one product, for reading profiles: level 1 is
 * the fine matvec's couplings of every depth, level k >= 2 the restricted
 * operator of depth L - k + 2 (Section 3.3, eq. a2_str).  tasks: waves of
 * the launch (one 64-lane wave per task, four per 256-thread block);
 * blocks: stored r x r blocks it streams.  Level >= 2 needs
 * h2mg_setup_mg.  Errors: INVALID_ARG for a bad level, STATE. */
h2mg_status h2mg_gemv_launch_info(h2mg_h2_t h, int32_t level, int64_t* tasks, int64_t* blocks);

/* Device memory held by the handle, in bytes. */
h2mg_status h2mg_memory_bytes(h2mg_h2_t h, int64_t* bytes);

h2mg_status h2mg_destroy(h2mg_h2_t h);

const char* h2mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* H2MG_H_ */
