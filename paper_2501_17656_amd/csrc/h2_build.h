// Construction, hierarchy setup, products and the solver of an H2 handle.
#pragma once
#include "h2_impl.h"

namespace h2mg {

// scale_dev, diag_dev: optional per-point scale and diagonal (device, user
// order) of the scaled form diag(s) K diag(s) + diag(d).
h2mg_status build_h2(const double* points_dev, int64_t n, int dim, const h2mg_kernel* kernel,
                     const h2mg_build_opts* opts, hipStream_t stream, H2** out,
                     const double* scale_dev = nullptr, const double* diag_dev = nullptr);
h2mg_status setup_mg(H2& h, int precision_mask);
// Close entries by quadrature (user order: nq x dim sub-points and nq
// weights per point); stores the near field, which every later product
// reads (FP64, and an FP32 copy made by setup_mg for low precisions).
h2mg_status set_near_quadrature(H2& h, const double* qy_user, const double* qu_user, int nq);
// enable != 0: evaluate the close leaf blocks once and store them (FP64
// tiles) for every later FP64 fine product; enable == 0: release them and
// go back to evaluating the near field in every product.
h2mg_status store_near(H2& h, int enable);
// Buffers and task sets of the 16-column products and cycles (rebuilt on
// next use).
void release_block_work(H2& h);
// The chunk plan of the near field alone (chunks, tile lists, tasks; no
// tiles), for products that evaluate the near-field tiles from the points.
// Throws on failure.
void plan_near(H2& h);
// y = A_H2 x for a block of nrhs <= 16 vectors (device, user order, row-major
// n x ld), FP64; needs 9 <= r <= 64.
h2mg_status matvec_multi(H2& h, int nrhs, const double* x, int ldx, double* y, int ldy);
// H2 matrix of dk/dl (which 1) or g = k'(r)/r (which 2) on the points and
// tree of h (shift 0).
h2mg_status build_derivative(H2& h, int which, H2** out);
// L = b^T x and scale * (dL/dl, dL/ds, dL/dp, dL/db) for x = A^{-1} b
// (user order; null outputs are skipped; hl is needed for dL/dl, hg for
// dL/dp).
h2mg_status quadratic_gradient(H2& h, H2* hl, H2* hg, const double* b, const double* x, double scale,
                               double* loss, double* grad_l, double* grad_s, double* grad_p,
                               double* grad_b);

// Products in precision p (vectors double for P64, float otherwise).
// Fine level, tree order: out = alpha * A_H2 x + beta * add (add may be null).
void apply_fine(H2& h, int p, const void* xt, void* out, double alpha, const void* add,
                double beta);
// Level k >= 2 (depth L - k + 2), coefficient order: y = A_k x.
void apply_coarse(H2& h, int p, int k, const void* x, void* y);
void apply_level(H2& h, int p, int k, const void* x, void* y);
// r_next = U_k^T r (level k to k+1); level-1 vectors in tree order.
void restrict_level(H2& h, int p, int k, const void* r, void* r_next);
// e = alpha * U_k e_next + beta * add.
void prolong_level(H2& h, int p, int k, const void* e_next, void* e, const void* add, double beta);

struct SolveParams {
  int n_fine = 1, n_coarse = 40;
  double rtol = 1e-8;
  int max_cycles = 500;
  int precision = 0;
  bool use_x0 = false;
  int smoother = 0;      // 0: CG, 1: block-Jacobi preconditioned CG
  int method = 0;        // 0: V-cycles, 1: W-cycles, 2: F-cycles, 3: CG on A_H2 alone
};
// Solve A_H2 x = b; b, x device, user order.  Fills info.
h2mg_status solve(H2& h, const double* b, double* x, const SolveParams& sp, h2mg_solve_info* info);
// The same solve with every vector carved from the fixed device scratch
// region (no allocation, no graphs); STATE unless the hierarchy, the
// precision's operators and, for the block smoother, its inverses exist.
h2mg_status solve_noalloc(H2& h, const double* b, double* x, const SolveParams& sp,
                          h2mg_solve_info* info);
// Device address of the current device's fixed scratch region and its size
// in bytes (noalloc.hip; throws if the address cannot be obtained).
void* solve_scratch(size_t* bytes);
// e = Iter(A_level, r, e0): nsteps of the smoother in FP64 (level 1 in user
// order, coarser levels in coefficient order); e0 = e on entry when use_e0.
h2mg_status smooth_once(H2& h, int level, const double* r, double* e, int nsteps, int smoother,
                        bool use_e0);
// One FP64 cycle (V, W or F by sp.method) from x0 (user order).
h2mg_status vcycle_once(H2& h, const double* x0, const double* b, double* x_out, const SolveParams& sp);
// Inverse diagonal blocks of the block-Jacobi smoother (FP64, plus FP32
// copies when p != P64).
h2mg_status ensure_block_jacobi(H2& h, int p);

// Blocks of up to 16 right-hand sides (device, user order, row-major n x ld).
// Solve A_H2 X = B column by column, all columns per cycle; col_rel (host,
// nrhs entries, may be null) receives each column's final relative residual.
h2mg_status solve_multi(H2& h, int nrhs, const double* b, int ldb, double* x, int ldx,
                        const SolveParams& sp, h2mg_solve_info* info, double* col_rel);
// Independent problems solved together: problem i on handle hs[i] (distinct
// handles), with its cycles on one of nstreams streams; every stream first
// waits for the work enqueued so far on `user`.  Returns the first failing
// problem's status (the others still run to their end); statuses (may be
// null) receives every problem's.
h2mg_status solve_batch(int nprob, H2* const* hs, const int* nrhs, const double* const* b, const int* ldb,
                        double* const* x, const int* ldx, const SolveParams& sp, h2mg_solve_info* infos,
                        h2mg_status* statuses, int nstreams, hipStream_t user);
// The same problems advancing cycle by cycle together on `user`: every tile
// product of a cycle step is one launch over all active problems.
h2mg_status solve_group(int nprob, H2* const* hs, const int* nrhs, const double* const* b, const int* ldb,
                        double* const* x, const int* ldx, const SolveParams& sp, h2mg_solve_info* infos,
                        h2mg_status* statuses, hipStream_t user);

}  // namespace h2mg
