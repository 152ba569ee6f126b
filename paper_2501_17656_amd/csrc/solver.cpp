// The H2-MG solver: Algorithm 1 (Section 3.3) with CG smoothing, repeated
// V-cycles, and FP64 iterative refinement around a low-precision V-cycle.
// Also the W- and F-cycles named after Algorithm 1 (textbook recursive
// forms: the coarse correction of a level is repeated once on the remaining
// residual, with a W- or a V-cycle), and the comparison solver of the
// experiments, CG on A_H2 alone.
//
// Every step runs on the device; the host only enqueues kernels and reads
// the FP64 residual norm (a few hundred partial sums) once per cycle to
// decide whether to stop.  CG scalars stay on the device as fixed-order
// partial sums (kernels_solve.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <stdexcept>
#include <vector>

#include "graph.h"
#include "h2_build.h"

namespace h2mg {

namespace {

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

inline int vprec(int p) { return p == P64 ? P64 : P32; }   // vector type of an operator precision
inline size_t vbytes(int p) { return p == P64 ? 8 : 4; }

// Per-precision cycle vectors: r_k and e~_k per level, the first coarse
// correction of W/F-cycles (ec), CG temporaries.
struct Work {
  std::vector<void*> r, et, ec;
  void *s = nullptr, *pv = nullptr, *q = nullptr, *tmp = nullptr, *z = nullptr;
  int smoother = 0;
  double* gpart[2] = {nullptr, nullptr};
  double* dpart = nullptr;
};

// Where a solve's vectors come from: the handle's allocator, consecutive
// 256-byte aligned pieces of a fixed device region (the entry point that
// allocates nothing), or nowhere (COUNT: only the bytes are added up).
struct VecSource {
  enum Mode { ARENA, CARVE, COUNT } mode = ARENA;
  H2* h = nullptr;
  char* region = nullptr;
  size_t cap = 0, used = 0;
  void* get(size_t bytes) {
    if (mode == ARENA) return h->arena.alloc(bytes);
    const size_t off = (used + 255) & ~size_t(255);
    used = off + bytes;
    if (mode == COUNT) return nullptr;
    if (used > cap) throw std::length_error("solve scratch exhausted");
    return region + off;
  }
  void put(void* p) {
    if (mode == ARENA && p) h->arena.release(p);
  }
};

Work make_work(H2& h, int p, bool second_corrections, VecSource& src) {
  Work w;
  const size_t vb = vbytes(p);
  w.r.resize(h.levels + 1);
  w.et.resize(h.levels + 1);
  w.ec.assign(h.levels + 1, nullptr);
  for (int k = 1; k <= h.levels; ++k) {
    w.r[k] = src.get(size_t(h.level_size(k)) * vb);
    w.et[k] = src.get(size_t(h.level_size(k)) * vb);
    if (second_corrections && k >= 2 && k < h.levels)
      w.ec[k] = src.get(size_t(h.level_size(k)) * vb);
  }
  w.s = src.get(size_t(h.n) * vb);
  w.pv = src.get(size_t(h.n) * vb);
  w.q = src.get(size_t(h.n) * vb);
  w.tmp = src.get(size_t(h.n) * vb);
  w.z = src.get(size_t(h.n) * vb);
  w.gpart[0] = h.dot_part + 512;
  w.gpart[1] = h.dot_part + 1024;
  w.dpart = h.dot_part + 1536;
  return w;
}

Work make_work(H2& h, int p, bool second_corrections = false) {
  VecSource src;
  src.h = &h;
  return make_work(h, p, second_corrections, src);
}

void release_work(H2& h, Work& w, VecSource& src) {
  for (int k = 1; k <= h.levels; ++k) {
    src.put(w.r[k]);
    src.put(w.et[k]);
    src.put(w.ec[k]);
  }
  src.put(w.s);
  src.put(w.pv);
  src.put(w.q);
  src.put(w.tmp);
  src.put(w.z);
}

void release_work(H2& h, Work& w) {
  VecSource src;
  src.h = &h;
  release_work(h, w, src);
}

void zero(H2& h, void* v, int64_t n, int p) { launch_zero(h, p, v, n); }

void read_flags(H2& h, int* f) {
  hip_check(hipMemcpyAsync(f, h.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, h.stream), "flags");
  hip_check(hipStreamSynchronize(h.stream), "sync");
}

// e = Iter(A_k, rhs, e0): n CG steps (plain, or preconditioned by the
// block-Jacobi inverses when w.smoother == 1); e holds e0 on entry unless
// e0_zero.
void cg(H2& h, int p, int k, Work& w, const void* rhs, void* e, bool e0_zero, int nsteps) {
  const int vp = vprec(p);
  const int64_t N = h.level_size(k);
  const bool pre = w.smoother == 1;
  if (e0_zero) zero(h, e, N, vp);
  if (nsteps <= 0) return;
  if (e0_zero) {
    launch_copy(h, vp, rhs, w.s, N);
  } else {
    apply_level(h, p, k, e, w.q);
    launch_copy(h, vp, rhs, w.s, N);
    launch_axpby(h, vp, N, -1.0, w.q, 1.0, w.s);
  }
  int cur = 0;
  if (pre) {
    launch_bj_apply(h, p, k, w.s, w.z);
    launch_copy(h, vp, w.z, w.pv, N);
    launch_dot(h, vp, N, w.s, w.z, w.gpart[cur]);
  } else {
    launch_copy(h, vp, w.s, w.pv, N);
    launch_dot(h, vp, N, w.s, w.s, w.gpart[cur]);
  }
  double* scratch = h.dot_part + 2048;
  for (int it = 0; it < nsteps; ++it) {
    apply_level(h, p, k, w.pv, w.q);
    launch_dot(h, vp, N, w.pv, w.q, w.dpart);
    if (pre) {
      launch_cg_update(h, vp, N, e, w.pv, w.s, w.q, w.gpart[cur], w.dpart, scratch);
      launch_bj_apply(h, p, k, w.s, w.z);
      launch_dot(h, vp, N, w.s, w.z, w.gpart[1 - cur]);
      if (it + 1 < nsteps) launch_cg_pupdate(h, vp, N, w.pv, w.z, w.gpart[cur], w.gpart[1 - cur]);
    } else {
      launch_cg_update(h, vp, N, e, w.pv, w.s, w.q, w.gpart[cur], w.dpart, w.gpart[1 - cur]);
      if (it + 1 < nsteps) launch_cg_pupdate(h, vp, N, w.pv, w.s, w.gpart[cur], w.gpart[1 - cur]);
    }
    cur = 1 - cur;
  }
}

// Direct solve on the coarsest level (FP64 Cholesky factor): e = A_l^{-1} r.
void coarse_solve(H2& h, int p, const void* r, void* e) {
  const int vp = vprec(p);
  if (vp == P64) {
    launch_copy(h, P64, r, e, h.Nl);
    launch_chol_solve(h, h.chol, h.Nl, static_cast<double*>(e));
  } else {
    launch_cast(h, P64, h.vtree2, P32, r, h.Nl);
    launch_chol_solve(h, h.chol, h.Nl, h.vtree2);
    launch_cast(h, P32, e, P64, h.vtree2, h.Nl);
  }
}

enum Cycle { CYCLE_V = 0, CYCLE_W = 1, CYCLE_F = 2 };

// One cycle on level k for A_k e_k = r_k (w.r[k] holds r_k); the result e_k
// is left in w.et[k].  With kind V this is Algorithm 1 from level k down.
void mg(H2& h, int p, Work& w, int k, int kind, int n_f, int n_c) {
  const int vp = vprec(p);
  const int l = h.levels;
  if (k == l) {
    coarse_solve(h, p, w.r[l], w.et[l]);
    return;
  }
  const int nk = k == 1 ? n_f : n_c;
  const int64_t N = h.level_size(k);
  cg(h, p, k, w, w.r[k], w.et[k], true, nk);
  // restriction of the residual: r_{k+1} = U_k^T (r_k - A_k e~_k)
  apply_level(h, p, k, w.et[k], w.tmp);
  launch_axpby(h, vp, N, 1.0, w.r[k], -1.0, w.tmp);
  restrict_level(h, p, k, w.tmp, w.r[k + 1]);
  mg(h, p, w, k + 1, kind, n_f, n_c);
  if (kind != CYCLE_V && k + 1 < l) {
    // second coarse correction on r_{k+1} - A_{k+1} e_{k+1}
    const int64_t N1 = h.level_size(k + 1);
    launch_copy(h, vp, w.et[k + 1], w.ec[k + 1], N1);
    apply_level(h, p, k + 1, w.et[k + 1], w.tmp);
    launch_axpby(h, vp, N1, -1.0, w.tmp, 1.0, w.r[k + 1]);
    mg(h, p, w, k + 1, kind == CYCLE_F ? CYCLE_V : CYCLE_W, n_f, n_c);
    launch_axpby(h, vp, N1, 1.0, w.ec[k + 1], 1.0, w.et[k + 1]);
  }
  prolong_level(h, p, k, w.et[k + 1], w.et[k], w.et[k], 1.0);   // e~_k += U_k e_{k+1}
  cg(h, p, k, w, w.r[k], w.et[k], false, nk);
}

// One cycle on the correction equation A e_1 = r_1 (w.r[1] holds r_1,
// tree order); the result e_1 is left in w.et[1].
void vcycle(H2& h, int p, Work& w, int kind, int n_f, int n_c) { mg(h, p, w, 1, kind, n_f, n_c); }

double host_norm(H2& h, const double* v, int64_t n) {
  const int np = dot_parts(n);
  launch_dot(h, P64, n, v, v, h.dot_part);
  std::vector<double> part(np);
  hip_check(hipMemcpyAsync(part.data(), h.dot_part, np * sizeof(double), hipMemcpyDeviceToHost, h.stream),
            "norm readback");
  hip_check(hipStreamSynchronize(h.stream), "sync");
  double s = 0.0;
  for (int i = 0; i < np; ++i) s += part[i];
  return std::sqrt(s);
}


double sum_parts(H2& h, const double* part, int np) {
  std::vector<double> v(np);
  hip_check(hipMemcpyAsync(v.data(), part, np * sizeof(double), hipMemcpyDeviceToHost, h.stream),
            "readback");
  hip_check(hipStreamSynchronize(h.stream), "sync");
  double s = 0.0;
  for (int i = 0; i < np; ++i) s += v[i];
  return s;
}

// The comparison solver: CG (block-Jacobi PCG with smoother 1) on A_H2 x = b
// in FP64, tree order, from x = 0 or the given x.  The stopping test reads
// the recurrence residual ||s|| / ||b|| (the sum of s.s partials) once per
// iteration; iterations are counted in `cycles`.
h2mg_status plain_cg(H2& h, Work& w, const double* bt, double* xt, double nb, const SolveParams& sp,
                     int* iters, bool* converged) {
  const int64_t n = h.n;
  const int np = dot_parts(n);
  const bool pre = w.smoother == 1;
  double* s = static_cast<double*>(w.s);
  double* z = static_cast<double*>(w.z);
  double* pv = static_cast<double*>(w.pv);
  double* q = static_cast<double*>(w.q);
  double* ss = h.dot_part + 2048;
  // s = b - A x
  apply_fine(h, P64, xt, s, -1.0, bt, 1.0);
  int cur = 0;
  if (pre) {
    launch_bj_apply(h, P64, 1, s, z);
    launch_copy(h, P64, z, pv, n);
    launch_dot(h, P64, n, s, z, w.gpart[cur]);
    launch_dot(h, P64, n, s, s, ss);
  } else {
    launch_copy(h, P64, s, pv, n);
    launch_dot(h, P64, n, s, s, w.gpart[cur]);
  }
  int f[4];
  for (int it = 0;; ++it) {
    const double rn = std::sqrt(sum_parts(h, pre ? ss : w.gpart[cur], np));
    read_flags(h, f);
    const double rel = rn / nb;
    h.history.push_back(rel);
    *iters = it;
    if (f[0]) return fail(H2MG_ERR_NOT_SPD, "CG met p^T A p <= 0 (operator not SPD)");
    if (!std::isfinite(rel)) return fail(H2MG_ERR_NUMERIC, "non-finite residual after %d iterations", it);
    if (rel < sp.rtol) {
      *converged = true;
      return H2MG_OK;
    }
    if (it >= sp.max_cycles)
      return fail(H2MG_ERR_NOT_CONVERGED, "CG: no convergence in %d iterations (rel. residual %.3e)",
                  sp.max_cycles, rel);
    apply_fine(h, P64, pv, q, 1.0, nullptr, 0.0);
    launch_dot(h, P64, n, pv, q, w.dpart);
    if (pre) {
      launch_cg_update(h, P64, n, xt, pv, s, q, w.gpart[cur], w.dpart, ss);
      launch_bj_apply(h, P64, 1, s, z);
      launch_dot(h, P64, n, s, z, w.gpart[1 - cur]);
      launch_cg_pupdate(h, P64, n, pv, z, w.gpart[cur], w.gpart[1 - cur]);
    } else {
      launch_cg_update(h, P64, n, xt, pv, s, q, w.gpart[cur], w.dpart, w.gpart[1 - cur]);
      launch_cg_pupdate(h, P64, n, pv, s, w.gpart[cur], w.gpart[1 - cur]);
    }
    cur = 1 - cur;
  }
}

}  // namespace

// Inverse diagonal blocks for the block-Jacobi smoother (built once per
// handle; FP32 copies for the low-precision forms).
h2mg_status ensure_block_jacobi(H2& h, int p) {
  if (!h.bj_built[P64]) {
    if (h.leaf_max > 128)
      return fail(H2MG_ERR_INVALID_ARG,
                  "the block smoother needs leaves of at most 128 points (largest has %d)",
                  h.leaf_max);
    h.bj_ld = h.leaf_max;
    double* fine = h.arena.make<double>(size_t(h.nleaf) * h.bj_ld * h.bj_ld);
    double* coarse = h.arena.make<double>(size_t(h.ngid) * h.r * h.r);
    hip_check(hipMemsetAsync(h.flags, 0, 4 * sizeof(int), h.stream), "memset");
    launch_bj_inverse_fine(h, fine, h.bj_ld);
    for (int d = h.d_top + 1; d <= h.L && h.d_top >= 0; ++d) {
      std::vector<int> diag;
      for (int b = h.p_first[d]; b < h.p_first[d] + h.p_count[d]; ++b)
        if (h.blk_row_h[b] == h.blk_col_h[b]) diag.push_back(b);
      if (int(diag.size()) != (1 << d)) return fail(H2MG_ERR_STATE, "missing diagonal block at depth %d", d);
      int* dd = h.arena.make<int>(diag.size());
      hip_check(hipMemcpyAsync(dd, diag.data(), diag.size() * sizeof(int), hipMemcpyHostToDevice, h.stream),
                "upload");
      launch_bj_inverse_coarse(h, d, dd, coarse);
      hip_check(hipStreamSynchronize(h.stream), "bj");
      h.arena.release(dd);
    }
    int f[4];
    read_flags(h, f);
    if (f[0]) {
      h.arena.release(fine);
      h.arena.release(coarse);
      return fail(H2MG_ERR_NOT_SPD, "a diagonal block of the block smoother is not positive definite");
    }
    h.bj_fine[P64] = fine;
    h.bj_coarse[P64] = coarse;
    h.bj_built[P64] = true;
  }
  if (p != P64 && !h.bj_built[P32]) {
    const int64_t nf = int64_t(h.nleaf) * h.bj_ld * h.bj_ld, nc = int64_t(h.ngid) * h.r * h.r;
    h.bj_fine[P32] = h.arena.alloc(size_t(nf) * 4);
    h.bj_coarse[P32] = h.arena.alloc(size_t(nc) * 4);
    launch_cast(h, P32, h.bj_fine[P32], P64, h.bj_fine[P64], nf);
    launch_cast(h, P32, h.bj_coarse[P32], P64, h.bj_coarse[P64], nc);
    hip_check(hipStreamSynchronize(h.stream), "bj cast");
    h.bj_built[P32] = true;
  }
  return H2MG_OK;
}

namespace {

// The solve of `solve` (arena vectors, optional graphs) and of `solve_noalloc`
// (vectors carved from the device scratch region, no graphs, nothing built
// on demand).
h2mg_status solve_impl(H2& h, const double* b, double* x, const SolveParams& sp, h2mg_solve_info* info,
                       bool noalloc) {
  const auto t0 = std::chrono::steady_clock::now();
  h.history.clear();
  const int p = sp.precision == 0 ? P64 : sp.precision == 1 ? P32 : P16;
  const bool plain = sp.method == 3;
  if (plain && p != P64) return fail(H2MG_ERR_INVALID_ARG, "CG on A_H2 alone runs in FP64 only");
  const bool need_mg = !(plain && sp.smoother == 0);
  if (noalloc) {
    // everything a solve would otherwise build on its first call must exist
    if (need_mg && (!h.mg_built || (p != P64 && !h.prec[p].ready)))
      return fail(H2MG_ERR_STATE, "the solve that allocates nothing needs h2mg_setup_mg with the %s "
                  "precision bit first", p == P64 ? "FP64" : p == P32 ? "FP32" : "BF16");
    if (sp.smoother == 1 && (!h.bj_built[P64] || (p != P64 && !h.bj_built[P32])))
      return fail(H2MG_ERR_STATE, "the solve that allocates nothing needs the block smoother's "
                  "inverses: run one h2mg_solve with this smoother and precision first");
  }
  // plain CG needs the hierarchy only for the block-Jacobi inverses, which
  // are formed for all levels together
  h2mg_status st = need_mg ? setup_mg(h, p == P64 ? 0 : (1 << p)) : H2MG_OK;
  if (st != H2MG_OK) return st;
  if (sp.smoother == 1) {
    try {
      st = ensure_block_jacobi(h, p);
    } catch (const std::bad_alloc&) {
      return fail(H2MG_ERR_OOM, "device allocation failed for the block smoother");
    } catch (const std::exception& ex) {
      return fail(H2MG_ERR_HIP, "%s", ex.what());
    }
    if (st != H2MG_OK) return st;
  }
  const bool second = sp.method == CYCLE_W || sp.method == CYCLE_F;
  const int64_t n = h.n;
  VecSource src;
  src.h = &h;
  if (noalloc) {
    // bytes of every vector below, then the fixed region they are carved from
    VecSource cnt;
    cnt.mode = VecSource::COUNT;
    make_work(h, P64, second && p == P64, cnt);
    if (p != P64) make_work(h, p, second, cnt);
    cnt.get(size_t(n) * 8);
    cnt.get(size_t(n) * 8);
    size_t cap = 0;
    void* region = nullptr;
    try {
      region = solve_scratch(&cap);
    } catch (const std::exception& ex) {
      return fail(H2MG_ERR_HIP, "%s", ex.what());
    }
    if (cnt.used > cap)
      return fail(H2MG_ERR_INVALID_ARG, "this solve needs %zu bytes of scratch; the fixed region "
                  "holds %zu (H2MG_SOLVE_SCRATCH_BYTES)", cnt.used, cap);
    src.mode = VecSource::CARVE;
    src.region = static_cast<char*>(region);
    src.cap = cap;
  }
  Work w64, wlp;
  bool have_lp = false;
  h2mg_status result = H2MG_OK;
  int cycles = 0;
  bool converged = false;
  double rel = 0.0;
  try {
    w64 = make_work(h, P64, second && p == P64, src);
    w64.smoother = sp.smoother;
    if (p != P64) {
      wlp = make_work(h, p, second, src);
      wlp.smoother = sp.smoother;
      have_lp = true;
    }
    double* bt = static_cast<double*>(src.get(size_t(n) * 8));
    double* xt = static_cast<double*>(src.get(size_t(n) * 8));
    double* res = static_cast<double*>(w64.r[1]);
    auto release_all = [&]() {
      src.put(bt);
      src.put(xt);
      release_work(h, w64, src);
      if (have_lp) release_work(h, wlp, src);
    };
    launch_gather(h, b, bt);
    if (sp.use_x0) launch_gather(h, x, xt);
    else zero(h, xt, n, P64);
    hip_check(hipMemsetAsync(h.flags, 0, 4 * sizeof(int), h.stream), "memset");
    launch_check_finite(h, P64, n, bt);
    int f[4];
    read_flags(h, f);
    if (f[1]) {
      release_all();
      return fail(H2MG_ERR_INVALID_ARG, "b contains a non-finite value");
    }
    const double nb = host_norm(h, bt, n);
    if (nb == 0.0) {
      zero(h, xt, n, P64);
      h.history.push_back(0.0);
      converged = true;
    } else if (sp.method == 3) {
      result = plain_cg(h, w64, bt, xt, nb, sp, &cycles, &converged);
      // report the true FP64 residual of the final iterate
      apply_fine(h, P64, xt, res, -1.0, bt, 1.0);
      rel = host_norm(h, res, n) / nb;
      if (!h.history.empty()) h.history.back() = rel;
    } else {
      // event timing records events between launches, so it runs the cycle
      // launch by launch; the entry point that allocates nothing does too
      // (instantiating a graph allocates)
      const bool use_graph = h.graphs && !h.timing && !noalloc;
      CycleGraph cg_graph;
      for (int cyc = 0;; ++cyc) {
        // res = b - A_H2 x (FP64)
        apply_fine(h, P64, xt, res, -1.0, bt, 1.0);
        const double rn = host_norm(h, res, n);
        read_flags(h, f);
        rel = rn / nb;
        h.history.push_back(rel);
        cycles = cyc;
        if (f[0]) { result = fail(H2MG_ERR_NOT_SPD, "CG met p^T A p <= 0 (operator not SPD)"); break; }
        if (!std::isfinite(rel)) { result = fail(H2MG_ERR_NUMERIC, "non-finite residual after %d cycles", cyc); break; }
        if (rel < sp.rtol) { converged = true; break; }
        if (cyc >= sp.max_cycles) {
          result = fail(H2MG_ERR_NOT_CONVERGED, "no convergence in %d cycles (rel. residual %.3e)",
                        sp.max_cycles, rel);
          break;
        }
        auto body = [&]() {
          if (p == P64) {
            vcycle(h, P64, w64, sp.method, sp.n_fine, sp.n_coarse);
            launch_axpby(h, P64, n, 1.0, w64.et[1], 1.0, xt);
          } else {
            launch_cast(h, P32, wlp.r[1], P64, res, n);
            vcycle(h, p, wlp, sp.method, sp.n_fine, sp.n_coarse);
            launch_cast(h, P64, h.vtree, P32, wlp.et[1], n);
            launch_axpby(h, P64, n, 1.0, h.vtree, 1.0, xt);
          }
        };
        if (use_graph) {
          if (!cg_graph.exec) capture(h, cg_graph, body);
          hip_check(hipGraphLaunch(cg_graph.exec, h.stream), "graph launch");
        } else {
          body();
        }
      }
    }
    launch_scatter(h, xt, x);
    hip_check(hipStreamSynchronize(h.stream), "solve");
    release_all();
  } catch (const std::bad_alloc&) {
    return fail(H2MG_ERR_OOM, "device allocation failed in the solve");
  } catch (const std::exception& ex) {
    return fail(H2MG_ERR_HIP, "%s", ex.what());
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) {
    info->cycles = cycles;
    info->converged = converged ? 1 : 0;
    info->rel_residual = h.history.empty() ? 0.0 : h.history.back();
    info->solve_seconds = secs;
    info->history_len = int(h.history.size());
  }
  return result;
}

}  // namespace

h2mg_status solve(H2& h, const double* b, double* x, const SolveParams& sp, h2mg_solve_info* info) {
  return solve_impl(h, b, x, sp, info, false);
}

h2mg_status solve_noalloc(H2& h, const double* b, double* x, const SolveParams& sp,
                          h2mg_solve_info* info) {
  return solve_impl(h, b, x, sp, info, true);
}

h2mg_status smooth_once(H2& h, int level, const double* r, double* e, int nsteps, int smoother,
                        bool use_e0) {
  h2mg_status st = setup_mg(h, 0);
  if (st != H2MG_OK) return st;
  if (level < 1 || level > h.levels)
    return fail(H2MG_ERR_INVALID_ARG, "level %d out of range 1..%d", level, h.levels);
  if (smoother == 1 && level == h.levels && level > 1)
    return fail(H2MG_ERR_INVALID_ARG, "the block smoother has no blocks on the coarsest level");
  try {
    if (smoother == 1) {
      st = ensure_block_jacobi(h, P64);
      if (st != H2MG_OK) return st;
    }
    Work w = make_work(h, P64);
    w.smoother = smoother;
    const int64_t N = h.level_size(level);
    if (level == 1) {
      launch_gather(h, r, static_cast<double*>(w.r[1]));
      if (use_e0) launch_gather(h, e, static_cast<double*>(w.et[1]));
    } else {
      launch_copy(h, P64, r, w.r[level], N);
      if (use_e0) launch_copy(h, P64, e, w.et[level], N);
    }
    hip_check(hipMemsetAsync(h.flags, 0, 4 * sizeof(int), h.stream), "memset");
    cg(h, P64, level, w, w.r[level], w.et[level], !use_e0, nsteps);
    if (level == 1) launch_scatter(h, static_cast<const double*>(w.et[1]), e);
    else launch_copy(h, P64, w.et[level], e, N);
    int f[4];
    read_flags(h, f);
    release_work(h, w);
    if (f[0]) return fail(H2MG_ERR_NOT_SPD, "CG met p^T A p <= 0 (operator not SPD)");
  } catch (const std::bad_alloc&) {
    return fail(H2MG_ERR_OOM, "device allocation failed in the smoother");
  } catch (const std::exception& ex) {
    return fail(H2MG_ERR_HIP, "%s", ex.what());
  }
  return H2MG_OK;
}

h2mg_status vcycle_once(H2& h, const double* x0, const double* b, double* x_out, const SolveParams& sp) {
  if (sp.method > CYCLE_F) return fail(H2MG_ERR_INVALID_ARG, "one cycle needs method V, W or F");
  h2mg_status st = setup_mg(h, 0);
  if (st != H2MG_OK) return st;
  try {
    if (sp.smoother == 1) {
      st = ensure_block_jacobi(h, P64);
      if (st != H2MG_OK) return st;
    }
    Work w = make_work(h, P64, sp.method != CYCLE_V);
    w.smoother = sp.smoother;
    const int64_t n = h.n;
    double* bt = static_cast<double*>(h.arena.alloc(size_t(n) * 8));
    double* xt = static_cast<double*>(h.arena.alloc(size_t(n) * 8));
    launch_gather(h, b, bt);
    launch_gather(h, x0, xt);
    hip_check(hipMemsetAsync(h.flags, 0, 4 * sizeof(int), h.stream), "memset");
    apply_fine(h, P64, xt, w.r[1], -1.0, bt, 1.0);   // r_1 = b - A x_0
    vcycle(h, P64, w, sp.method, sp.n_fine, sp.n_coarse);
    launch_axpby(h, P64, n, 1.0, w.et[1], 1.0, xt);  // x* = x_0 + e_1
    launch_scatter(h, xt, x_out);
    int f[4];
    read_flags(h, f);
    h.arena.release(bt);
    h.arena.release(xt);
    release_work(h, w);
    if (f[0]) return fail(H2MG_ERR_NOT_SPD, "CG met p^T A p <= 0 (operator not SPD)");
  } catch (const std::bad_alloc&) {
    return fail(H2MG_ERR_OOM, "device allocation failed in the V-cycle");
  } catch (const std::exception& ex) {
    return fail(H2MG_ERR_HIP, "%s", ex.what());
  }
  return H2MG_OK;
}

}  // namespace h2mg
