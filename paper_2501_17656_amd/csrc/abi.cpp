// extern "C" entry points declared in include/h2mg.h.  Every call returns a
// status; exceptions never cross this boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>
#include <cstring>
#include <new>
#include <stdexcept>

#include "h2_build.h"

using namespace h2mg;

struct h2mg_plan_s {
  Plan plan;
};

struct h2mg_h2_s {
  H2* h;
};

namespace {

template <typename F>
h2mg_status guarded(F&& f) {
  clear_error();
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(H2MG_ERR_OOM, "allocation failed");
  } catch (const std::exception& e) {
    return fail(H2MG_ERR_HIP, "%s", e.what());
  } catch (...) {
    return fail(H2MG_ERR_HIP, "unknown error");
  }
}

h2mg_status check_stream_err(hipStream_t s) {
  (void)s;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(H2MG_ERR_HIP, "%s", hipGetErrorString(e));
  return H2MG_OK;
}

bool valid_solve_opts(const h2mg_solve_opts* o) {
  return o && o->n_fine >= 0 && o->n_coarse >= 0 && o->rtol > 0.0 && std::isfinite(o->rtol) &&
         o->max_cycles >= 0 && o->precision >= 0 && o->precision <= 2 && o->smoother >= 0 &&
         o->smoother <= 1 && o->method >= 0 && o->method <= 3;
}

SolveParams to_params(const h2mg_solve_opts* o) {
  SolveParams sp;
  sp.n_fine = o->n_fine;
  sp.n_coarse = o->n_coarse;
  sp.rtol = o->rtol;
  sp.max_cycles = o->max_cycles;
  sp.precision = o->precision;
  sp.use_x0 = o->use_x0 != 0;
  sp.smoother = o->smoother;
  sp.method = o->method;
  return sp;
}

}  // namespace

extern "C" {

const char* h2mg_last_error(void) { return last_error_cstr(); }

h2mg_status h2mg_plan_create(const double* points_host, int64_t n, int32_t dim,
                             const h2mg_build_opts* opts, h2mg_plan_t* out) {
  return guarded([&] {
    if (!out) return fail(H2MG_ERR_INVALID_ARG, "null output handle");
    *out = nullptr;
    auto* p = new h2mg_plan_s();
    h2mg_status st = build_plan(points_host, n, dim, opts, &p->plan);
    if (st != H2MG_OK) {
      delete p;
      return st;
    }
    *out = p;
    return H2MG_OK;
  });
}

h2mg_status h2mg_plan_query(h2mg_plan_t plan, h2mg_plan_info* info) {
  return guarded([&] {
    if (!plan || !info) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    const Plan& P = plan->plan;
    info->n = P.n;
    info->dim = P.dim;
    info->depth = P.L;
    info->d_top = P.d_top;
    info->rank = P.r;
    info->leaf_min = P.leaf_min;
    info->leaf_max = P.leaf_max;
    return H2MG_OK;
  });
}

h2mg_status h2mg_plan_perm(h2mg_plan_t plan, int64_t* perm_host) {
  return guarded([&] {
    if (!plan || !perm_host) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    std::memcpy(perm_host, plan->plan.perm.data(), plan->plan.perm.size() * sizeof(int64_t));
    return H2MG_OK;
  });
}

h2mg_status h2mg_plan_offsets(h2mg_plan_t plan, int32_t depth, int64_t* off) {
  return guarded([&] {
    if (!plan || !off) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    if (depth < 0 || depth > plan->plan.L) return fail(H2MG_ERR_INVALID_ARG, "depth out of range");
    const auto& o = plan->plan.offsets[depth];
    std::memcpy(off, o.data(), o.size() * sizeof(int64_t));
    return H2MG_OK;
  });
}

h2mg_status h2mg_plan_pair_count(h2mg_plan_t plan, int32_t depth, int32_t which, int64_t* count) {
  return guarded([&] {
    if (!plan || !count) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    if (depth < 0 || depth > plan->plan.L || which < 0 || which > 1)
      return fail(H2MG_ERR_INVALID_ARG, "depth or kind out of range");
    const auto& v = which == 0 ? plan->plan.near[depth] : plan->plan.far[depth];
    *count = int64_t(v.size() / 2);
    return H2MG_OK;
  });
}

h2mg_status h2mg_plan_pairs(h2mg_plan_t plan, int32_t depth, int32_t which, int64_t* pairs) {
  return guarded([&] {
    if (!plan || !pairs) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    if (depth < 0 || depth > plan->plan.L || which < 0 || which > 1)
      return fail(H2MG_ERR_INVALID_ARG, "depth or kind out of range");
    const auto& v = which == 0 ? plan->plan.near[depth] : plan->plan.far[depth];
    for (size_t i = 0; i < v.size(); ++i) pairs[i] = v[i];
    return H2MG_OK;
  });
}

void h2mg_plan_destroy(h2mg_plan_t plan) { delete plan; }

h2mg_status h2mg_build(const double* points_dev, int64_t n, int32_t dim, const h2mg_kernel* kernel,
                       const h2mg_build_opts* opts, hipStream_t stream, h2mg_h2_t* out) {
  return guarded([&] {
    if (!out) return fail(H2MG_ERR_INVALID_ARG, "null output handle");
    *out = nullptr;
    H2* h = nullptr;
    h2mg_status st = build_h2(points_dev, n, dim, kernel, opts, stream, &h);
    if (st != H2MG_OK) return st;
    *out = new h2mg_h2_s{h};
    return H2MG_OK;
  });
}

h2mg_status h2mg_build_scaled(const double* points_dev, int64_t n, int32_t dim,
                              const h2mg_kernel* kernel, const h2mg_build_opts* opts,
                              const double* scale_dev, const double* diag_dev, hipStream_t stream,
                              h2mg_h2_t* out) {
  return guarded([&] {
    if (!out) return fail(H2MG_ERR_INVALID_ARG, "null output handle");
    *out = nullptr;
    H2* h = nullptr;
    h2mg_status st = build_h2(points_dev, n, dim, kernel, opts, stream, &h, scale_dev, diag_dev);
    if (st != H2MG_OK) return st;
    *out = new h2mg_h2_s{h};
    return H2MG_OK;
  });
}

h2mg_status h2mg_bem_panels(const double* V, int64_t nv, const int64_t* T, int64_t nt, double* y,
                            double* s, double* d, hipStream_t stream) {
  return guarded([&] {
    if (!V || !T || !y || !s || !d) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    if (nv < 3 || nt < 1) return fail(H2MG_ERR_INVALID_ARG, "need at least 3 vertices and 1 triangle");
    launch_bem_panels(stream, nt, V, T, y, s, d);
    return check_stream_err(stream);
  });
}

h2mg_status h2mg_bem_quadrature7(const double* V, int64_t nv, const int64_t* T, int64_t nt, double* qy,
                                 double* qu, hipStream_t stream) {
  return guarded([&] {
    if (!V || !T || !qy || !qu) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    if (nv < 3 || nt < 1) return fail(H2MG_ERR_INVALID_ARG, "need at least 3 vertices and 1 triangle");
    launch_bem_quadrature7(stream, nt, V, T, qy, qu);
    return check_stream_err(stream);
  });
}

h2mg_status h2mg_set_near_quadrature(h2mg_h2_t hh, const double* qy, const double* qu, int32_t nq,
                                     hipStream_t stream) {
  return guarded([&] {
    if (!hh || !qy || !qu) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    hh->h->stream = stream;
    return set_near_quadrature(*hh->h, qy, qu, nq);
  });
}

h2mg_status h2mg_bem_point_source_rhs(const double* y, const double* s, int64_t n, const double* x0,
                                      double* f, hipStream_t stream) {
  return guarded([&] {
    if (!y || !s || !x0 || !f || n < 1) return fail(H2MG_ERR_INVALID_ARG, "null argument or n < 1");
    launch_bem_rhs(stream, n, y, x0, s, f);
    return check_stream_err(stream);
  });
}

h2mg_status h2mg_bem_harmonic_rhs(const double* y, const double* s, int64_t n, const double* coeffs,
                                  double* f, hipStream_t stream) {
  return guarded([&] {
    if (!y || !s || !coeffs || !f || n < 1) return fail(H2MG_ERR_INVALID_ARG, "null argument or n < 1");
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(coeffs[k])) return fail(H2MG_ERR_INVALID_ARG, "coefficients must be finite");
    launch_bem_harmonic(stream, n, y, coeffs, s, f);
    return check_stream_err(stream);
  });
}

h2mg_status h2mg_bem_density(const double* yv, const double* s, int64_t n, double* sigma,
                             hipStream_t stream) {
  return guarded([&] {
    if (!yv || !s || !sigma || n < 1) return fail(H2MG_ERR_INVALID_ARG, "null argument or n < 1");
    launch_div(stream, n, yv, s, sigma);
    return check_stream_err(stream);
  });
}

h2mg_status h2mg_matvec(h2mg_h2_t hh, const double* x, double* y, hipStream_t stream) {
  return guarded([&] {
    if (!hh || !x || !y) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    H2& h = *hh->h;
    h.stream = stream;
    launch_gather(h, x, h.vtree);
    apply_fine(h, P64, h.vtree, h.vtree2, 1.0, nullptr, 0.0);
    launch_scatter(h, h.vtree2, y);
    return check_stream_err(stream);
  });
}

h2mg_status h2mg_setup_mg(h2mg_h2_t hh, int32_t mask, hipStream_t stream) {
  return guarded([&] {
    if (!hh) return fail(H2MG_ERR_INVALID_ARG, "null handle");
    hh->h->stream = stream;
    return setup_mg(*hh->h, mask);
  });
}

h2mg_status h2mg_level_count(h2mg_h2_t hh, int32_t* levels) {
  return guarded([&] {
    if (!hh || !levels) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    const H2& h = *hh->h;
    *levels = h.d_top < 0 ? 1 : h.L - h.d_top + 2;
    return H2MG_OK;
  });
}

h2mg_status h2mg_level_size(h2mg_h2_t hh, int32_t level, int64_t* size) {
  return guarded([&] {
    if (!hh || !size) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    const H2& h = *hh->h;
    const int l = h.d_top < 0 ? 1 : h.L - h.d_top + 2;
    if (level < 1 || level > l) return fail(H2MG_ERR_INVALID_ARG, "level out of range");
    *size = h.level_size(level);
    return H2MG_OK;
  });
}

h2mg_status h2mg_level_apply(h2mg_h2_t hh, int32_t level, const double* x, double* y,
                             hipStream_t stream) {
  return guarded([&] {
    if (!hh || !x || !y) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    H2& h = *hh->h;
    h.stream = stream;
    if (level == 1) {
      launch_gather(h, x, h.vtree);
      apply_fine(h, P64, h.vtree, h.vtree2, 1.0, nullptr, 0.0);
      launch_scatter(h, h.vtree2, y);
      return check_stream_err(stream);
    }
    if (!h.mg_built) return fail(H2MG_ERR_STATE, "call h2mg_setup_mg before applying level %d", level);
    if (level < 2 || level > h.levels) return fail(H2MG_ERR_INVALID_ARG, "level out of range");
    apply_coarse(h, P64, level, x, y);
    return check_stream_err(stream);
  });
}

h2mg_status h2mg_level_apply_precision(h2mg_h2_t hh, int32_t level, int32_t precision,
                                       const double* x, double* y, hipStream_t stream) {
  return guarded([&] {
    if (!hh || !x || !y) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    if (precision < H2MG_FP64 || precision > H2MG_BF16_IR)
      return fail(H2MG_ERR_INVALID_ARG, "unknown precision %d", precision);
    if (precision == H2MG_FP64) return h2mg_level_apply(hh, level, x, y, stream);
    H2& h = *hh->h;
    h.stream = stream;
    const int p = precision == H2MG_FP32_IR ? P32 : P16;
    if (level < 1 || level > h.levels) return fail(H2MG_ERR_INVALID_ARG, "level out of range");
    if (!h.mg_built || !h.prec[p].ready)
      return fail(H2MG_ERR_STATE, "call h2mg_setup_mg with the %s precision bit first",
                  p == P32 ? "FP32" : "BF16");
    const int64_t nk = h.level_size(level);
    float* x32 = h.arena.make<float>(size_t(nk));
    float* y32 = h.arena.make<float>(size_t(nk));
    if (level == 1) {
      launch_gather(h, x, h.vtree);
      launch_cast(h, P32, x32, P64, h.vtree, nk);
      apply_fine(h, p, x32, y32, 1.0, nullptr, 0.0);
      launch_cast(h, P64, h.vtree2, P32, y32, nk);
      launch_scatter(h, h.vtree2, y);
    } else {
      launch_cast(h, P32, x32, P64, x, nk);
      apply_coarse(h, p, level, x32, y32);
      launch_cast(h, P64, y, P32, y32, nk);
    }
    const h2mg_status st = check_stream_err(stream);
    (void)hipStreamSynchronize(stream);
    h.arena.release(x32);
    h.arena.release(y32);
    return st;
  });
}

h2mg_status h2mg_restrict(h2mg_h2_t hh, int32_t level, const double* r, double* r_next,
                          hipStream_t stream) {
  return guarded([&] {
    if (!hh || !r || !r_next) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    H2& h = *hh->h;
    h.stream = stream;
    const int l = h.d_top < 0 ? 1 : h.L - h.d_top + 2;
    if (level < 1 || level >= l) return fail(H2MG_ERR_INVALID_ARG, "level out of range");
    if (level == 1) {
      launch_gather(h, r, h.vtree);
      restrict_level(h, P64, 1, h.vtree, r_next);
    } else {
      restrict_level(h, P64, level, r, r_next);
    }
    return check_stream_err(stream);
  });
}

h2mg_status h2mg_prolong(h2mg_h2_t hh, int32_t level, const double* e_next, double* e,
                         hipStream_t stream) {
  return guarded([&] {
    if (!hh || !e_next || !e) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    H2& h = *hh->h;
    h.stream = stream;
    const int l = h.d_top < 0 ? 1 : h.L - h.d_top + 2;
    if (level < 1 || level >= l) return fail(H2MG_ERR_INVALID_ARG, "level out of range");
    if (level == 1) {
      prolong_level(h, P64, 1, e_next, h.vtree, nullptr, 0.0);
      launch_scatter(h, h.vtree, e);
    } else {
      prolong_level(h, P64, level, e_next, e, nullptr, 0.0);
    }
    return check_stream_err(stream);
  });
}

h2mg_status h2mg_smooth(h2mg_h2_t hh, int32_t level, const double* r, double* e, int32_t nsteps,
                        int32_t smoother, int32_t use_e0, hipStream_t stream) {
  return guarded([&] {
    if (!hh || !r || !e) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    if (nsteps < 0 || smoother < 0 || smoother > 1) return fail(H2MG_ERR_INVALID_ARG, "bad smoother options");
    hh->h->stream = stream;
    return smooth_once(*hh->h, level, r, e, nsteps, smoother, use_e0 != 0);
  });
}

h2mg_status h2mg_vcycle(h2mg_h2_t hh, const double* x0, const double* b, double* x_out,
                        const h2mg_solve_opts* opts, hipStream_t stream) {
  return guarded([&] {
    if (!hh || !x0 || !b || !x_out) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    if (!valid_solve_opts(opts)) return fail(H2MG_ERR_INVALID_ARG, "invalid solve options");
    hh->h->stream = stream;
    return vcycle_once(*hh->h, x0, b, x_out, to_params(opts));
  });
}

h2mg_status h2mg_solve(h2mg_h2_t hh, const double* b, double* x, const h2mg_solve_opts* opts,
                       h2mg_solve_info* info, hipStream_t stream) {
  return guarded([&] {
    if (!hh || !b || !x) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    if (!valid_solve_opts(opts)) return fail(H2MG_ERR_INVALID_ARG, "invalid solve options");
    hh->h->stream = stream;
    return solve(*hh->h, b, x, to_params(opts), info);
  });
}

h2mg_status h2mg_solve_noalloc(h2mg_h2_t hh, const double* b, double* x, const h2mg_solve_opts* opts,
                               h2mg_solve_info* info, hipStream_t stream) {
  return guarded([&] {
    if (!hh || !b || !x) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    if (!valid_solve_opts(opts)) return fail(H2MG_ERR_INVALID_ARG, "invalid solve options");
    hh->h->stream = stream;
    return solve_noalloc(*hh->h, b, x, to_params(opts), info);
  });
}

h2mg_status h2mg_solve_history(h2mg_h2_t hh, double* hist, int32_t cap) {
  return guarded([&] {
    if (!hh || (!hist && cap > 0)) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    const auto& v = hh->h->history;
    for (int i = 0; i < cap && i < int(v.size()); ++i) hist[i] = v[i];
    return H2MG_OK;
  });
}

h2mg_status h2mg_memory_bytes(h2mg_h2_t hh, int64_t* bytes) {
  return guarded([&] {
    if (!hh || !bytes) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    *bytes = int64_t(hh->h->arena.bytes);
    return H2MG_OK;
  });
}

h2mg_status h2mg_build_derivative(h2mg_h2_t hh, int32_t which, hipStream_t stream, h2mg_h2_t* out) {
  return guarded([&] {
    if (!hh || !out) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    hh->h->stream = stream;
    H2* d = nullptr;
    h2mg_status st = build_derivative(*hh->h, which, &d);
    if (st != H2MG_OK) return st;
    *out = new h2mg_h2_s{d};
    return H2MG_OK;
  });
}

h2mg_status h2mg_quadratic_gradient(h2mg_h2_t hh, h2mg_h2_t hl, h2mg_h2_t hg, const double* b,
                                    const double* x, double scale, double* loss, double* grad_l,
                                    double* grad_s, double* grad_p, double* grad_b,
                                    hipStream_t stream) {
  return guarded([&] {
    if (!hh || !b || !x) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    if (!std::isfinite(scale)) return fail(H2MG_ERR_INVALID_ARG, "scale must be finite");
    hh->h->stream = stream;
    return quadratic_gradient(*hh->h, hl ? hl->h : nullptr, hg ? hg->h : nullptr, b, x, scale, loss,
                              grad_l, grad_s, grad_p, grad_b);
  });
}

h2mg_status h2mg_matvec_multi(h2mg_h2_t hh, int32_t nrhs, const double* x, int32_t ldx, double* y,
                              int32_t ldy, hipStream_t stream) {
  return guarded([&] {
    if (!hh || !x || !y) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    hh->h->stream = stream;
    h2mg_status st = matvec_multi(*hh->h, nrhs, x, ldx, y, ldy);
    if (st != H2MG_OK) return st;
    return check_stream_err(stream);
  });
}

h2mg_status h2mg_solve_multi(h2mg_h2_t hh, int32_t nrhs, const double* b, int32_t ldb, double* x,
                             int32_t ldx, const h2mg_solve_opts* opts, h2mg_solve_info* info,
                             double* col_residuals, hipStream_t stream) {
  return guarded([&] {
    if (!hh || !b || !x) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    if (!valid_solve_opts(opts)) return fail(H2MG_ERR_INVALID_ARG, "invalid solve options");
    hh->h->stream = stream;
    return solve_multi(*hh->h, nrhs, b, ldb, x, ldx, to_params(opts), info, col_residuals);
  });
}

h2mg_status h2mg_solve_batch(int32_t nprob, const h2mg_h2_t* hs, const int32_t* nrhs,
                             const double* const* b, const int32_t* ldb, double* const* x,
                             const int32_t* ldx, const h2mg_solve_opts* opts, h2mg_solve_info* infos,
                             h2mg_status* statuses, int32_t nstreams, hipStream_t stream) {
  return guarded([&] {
    if (nprob < 1 || !hs || !nrhs || !b || !ldb || !x || !ldx)
      return fail(H2MG_ERR_INVALID_ARG, "null argument or empty batch");
    if (!valid_solve_opts(opts)) return fail(H2MG_ERR_INVALID_ARG, "invalid solve options");
    if (nstreams < 0) return fail(H2MG_ERR_INVALID_ARG, "nstreams must be >= 0");
    std::vector<H2*> hv(nprob);
    for (int i = 0; i < nprob; ++i) {
      if (!hs[i]) return fail(H2MG_ERR_INVALID_ARG, "null handle in problem %d", i);
      hv[i] = hs[i]->h;
    }
    return solve_batch(nprob, hv.data(), nrhs, b, ldb, x, ldx, to_params(opts), infos, statuses, nstreams,
                       stream);
  });
}

h2mg_status h2mg_solve_group(int32_t nprob, const h2mg_h2_t* hs, const int32_t* nrhs,
                             const double* const* b, const int32_t* ldb, double* const* x,
                             const int32_t* ldx, const h2mg_solve_opts* opts, h2mg_solve_info* infos,
                             h2mg_status* statuses, hipStream_t stream) {
  return guarded([&] {
    if (nprob < 1 || !hs || !nrhs || !b || !ldb || !x || !ldx)
      return fail(H2MG_ERR_INVALID_ARG, "null argument or empty group");
    if (!valid_solve_opts(opts)) return fail(H2MG_ERR_INVALID_ARG, "invalid solve options");
    std::vector<H2*> hv(nprob);
    for (int i = 0; i < nprob; ++i) {
      if (!hs[i]) return fail(H2MG_ERR_INVALID_ARG, "null handle in problem %d", i);
      hv[i] = hs[i]->h;
    }
    return solve_group(nprob, hv.data(), nrhs, b, ldb, x, ldx, to_params(opts), infos, statuses, stream);
  });
}

h2mg_status h2mg_store_near(h2mg_h2_t hh, int32_t enable, hipStream_t stream) {
  return guarded([&] {
    if (!hh) return fail(H2MG_ERR_INVALID_ARG, "null handle");
    hh->h->stream = stream;
    return store_near(*hh->h, enable);
  });
}

h2mg_status h2mg_set_autotune(h2mg_h2_t hh, int32_t enabled) {
  return guarded([&] {
    if (!hh) return fail(H2MG_ERR_INVALID_ARG, "null handle");
    H2& h = *hh->h;
    if (h.autotune != (enabled != 0)) {
      (void)hipStreamSynchronize(h.stream);
      release_block_work(h);
      h.autotune = enabled != 0;
    }
    return H2MG_OK;
  });
}

h2mg_status h2mg_block_tuning(h2mg_h2_t hh, int32_t which, int32_t* run, double* ms, int64_t* tiles_read) {
  return guarded([&] {
    if (!hh || !run || !ms || !tiles_read) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    const H2& h = *hh->h;
    const BlockWork& w = h.blk16;
    const TileSet* ts = nullptr;
    if (which == -2) ts = w.near_ready ? &w.near : nullptr;
    else if (which == -1) ts = w.ready ? &w.fine : nullptr;
    else if (which >= 0 && which < int(w.coarse.size())) ts = &w.coarse[which];
    else if (which < -2 || which > h.L) return fail(H2MG_ERR_INVALID_ARG, "which must be -2, -1 or a depth");
    *run = ts ? ts->run : 0;
    *ms = ts ? ts->tuned_ms : 0.0;
    *tiles_read = ts ? ts->ntiles + ts->nctiles : 0;
    return H2MG_OK;
  });
}

h2mg_status h2mg_set_graphs(h2mg_h2_t hh, int32_t enabled) {
  return guarded([&] {
    if (!hh) return fail(H2MG_ERR_INVALID_ARG, "null handle");
    hh->h->graphs = enabled != 0;
    return H2MG_OK;
  });
}

h2mg_status h2mg_set_timing(h2mg_h2_t hh, int32_t enabled) {
  return guarded([&] {
    if (!hh) return fail(H2MG_ERR_INVALID_ARG, "null handle");
    H2& h = *hh->h;
    h.flush_timing();
    for (auto& k : h.kstat) k = KStat();
    h.timing = enabled != 0;
    return H2MG_OK;
  });
}

h2mg_status h2mg_kernel_stats(h2mg_h2_t hh, int32_t kind, int64_t* launches, double* total_ms,
                              double* total_work) {
  return guarded([&] {
    if (!hh || !launches || !total_ms || !total_work) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    if (kind < 0 || kind >= KS_COUNT) return fail(H2MG_ERR_INVALID_ARG, "unknown kernel kind");
    H2& h = *hh->h;
    h.flush_timing();
    *launches = h.kstat[kind].launches;
    *total_ms = h.kstat[kind].ms;
    *total_work = h.kstat[kind].bytes;
    return H2MG_OK;
  });
}

h2mg_status h2mg_gemv_launch_info(h2mg_h2_t hh, int32_t level, int64_t* tasks, int64_t* blocks) {
  return guarded([&] {
    if (!hh || !tasks || !blocks) return fail(H2MG_ERR_INVALID_ARG, "null argument");
    H2& h = *hh->h;
    if (level < 1 || level > h.levels) return fail(H2MG_ERR_INVALID_ARG, "level out of range");
    if (level == 1) {
      *tasks = h.fine_launch.ntasks;
      *blocks = h.fine_launch.nblocks;
      return H2MG_OK;
    }
    if (!h.mg_built) return fail(H2MG_ERR_STATE, "call h2mg_setup_mg first");
    const Launch& l = h.coarse_launch[h.level_depth(level)];
    *tasks = l.ntasks;
    *blocks = l.nblocks;
    return H2MG_OK;
  });
}

h2mg_status h2mg_destroy(h2mg_h2_t hh) {
  return guarded([&] {
    if (!hh) return H2MG_OK;
    (void)hipStreamSynchronize(hh->h->stream);
    delete hh->h;
    delete hh;
    return H2MG_OK;
  });
}

}  // extern "C"
