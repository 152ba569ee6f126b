// Building an H2 handle: host index structures, device allocations, and the
// order of the setup kernels (Section 3.1 for the H2 pieces, Section 3.3 for
// the restricted operators and the coarsest Cholesky factor).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <stdexcept>

#include "h2_build.h"

namespace h2mg {

void* Arena::alloc(size_t nbytes) {
  if (nbytes == 0) nbytes = 8;
  void* p = nullptr;
  if (hipMalloc(&p, nbytes) != hipSuccess || p == nullptr) {
    (void)hipGetLastError();
    throw std::bad_alloc();
  }
  ptrs.emplace_back(p, nbytes);
  bytes += nbytes;
  return p;
}

void Arena::release(void* p) {
  for (size_t i = 0; i < ptrs.size(); ++i)
    if (ptrs[i].first == p) {
      (void)hipFree(p);
      bytes -= ptrs[i].second;
      ptrs.erase(ptrs.begin() + i);
      return;
    }
}

Arena::~Arena() {
  for (auto& pr : ptrs) (void)hipFree(pr.first);
}

H2::~H2() {
  for (hipEvent_t e : events) (void)hipEventDestroy(e);
  if (capture_stream) (void)hipStreamDestroy(capture_stream);
}

int H2::take_event() {
  if (next_event == int(events.size())) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) throw std::runtime_error("hipEventCreate failed");
    events.push_back(e);
  }
  return next_event++;
}

void H2::time_begin(int& ev) {
  ev = -1;
  if (!timing) return;
  ev = take_event();
  (void)hipEventRecord(events[ev], stream);
}

void H2::time_end(int kind, int ev, double bytes) {
  if (ev < 0) return;
  const int e2 = take_event();
  (void)hipEventRecord(events[e2], stream);
  kstat[kind].pending.emplace_back(ev, e2);
  kstat[kind].pending_bytes.push_back(bytes);
  if (next_event > 4096) flush_timing();
}

void H2::flush_timing() {
  if (next_event == 0) return;
  (void)hipStreamSynchronize(stream);
  for (auto& k : kstat) {
    for (size_t i = 0; i < k.pending.size(); ++i) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, events[k.pending[i].first], events[k.pending[i].second]);
      k.ms += ms;
      k.bytes += k.pending_bytes[i];
      k.launches += 1;
    }
    k.pending.clear();
    k.pending_bytes.clear();
  }
  next_event = 0;
}

namespace {

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
T* upload(H2& h, const std::vector<T>& v) {
  T* d = h.arena.make<T>(std::max<size_t>(v.size(), 1));
  if (!v.empty())
    hip_check(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, h.stream),
              "upload");
  return d;
}

constexpr int CHUNK = 16;      // stored blocks per GEMV task
constexpr int NEAR_CHUNK = 4;  // close leaf pairs per near-field task

// Tasks and column lists of the stored blocks [first, first + count) of one
// depth (sorted by row gid, then column gid).
View make_view(H2& h, int d, int first, int count) {
  View v;
  v.depth = d;
  const int nrows = 1 << d;
  const int gid0 = nrows - 1;
  std::vector<int> rtp(nrows + 1, 0);
  for (int b = first; b < first + count;) {
    const int row = h.blk_row_h[b];
    int e = b;
    while (e < first + count && h.blk_row_h[e] == row) ++e;
    for (int c = b; c < e; c += CHUNK) {
      v.task.push_back(row);
      v.task.push_back(c);
      v.task.push_back(std::min(e, c + CHUNK));
      rtp[row - gid0 + 1]++;
    }
    b = e;
  }
  for (int i = 0; i < nrows; ++i) rtp[i + 1] += rtp[i];
  v.ntasks = int(v.task.size() / 3);
  std::vector<int> cptr(nrows + 1, 0), cblk;
  for (int b = first; b < first + count; ++b)
    if (h.blk_col_h[b] != h.blk_row_h[b]) cptr[h.blk_col_h[b] - gid0 + 1]++;
  for (int i = 0; i < nrows; ++i) cptr[i + 1] += cptr[i];
  cblk.resize(cptr[nrows]);
  std::vector<int> fill(cptr.begin(), cptr.end() - 1);
  for (int b = first; b < first + count; ++b)
    if (h.blk_col_h[b] != h.blk_row_h[b]) cblk[fill[h.blk_col_h[b] - gid0]++] = b;
  v.slot_base = h.nslot;
  for (size_t c = 0; c < cblk.size(); ++c) h.blk_slot_h[cblk[c]] = h.nslot + int(c);
  h.nslot += int(cblk.size());
  v.row_task_ptr = upload(h, rtp);
  v.col_ptr = upload(h, cptr);
  v.col_blk = upload(h, cblk);
  return v;
}

Launch make_launch(H2& h, const std::vector<const View*>& views) {
  Launch l;
  std::vector<int> all;
  for (const View* v : views) {
    l.base.push_back(int(all.size() / 3));
    all.insert(all.end(), v->task.begin(), v->task.end());
    for (size_t i = 0; i < v->task.size(); i += 3) l.nblocks += v->task[i + 2] - v->task[i + 1];
  }
  l.ntasks = int(all.size() / 3);
  l.task = upload(h, all);
  h.max_tasks = std::max(h.max_tasks, l.ntasks);
  return l;
}

}  // namespace

h2mg_status build_h2(const double* points_dev, int64_t n, int dim, const h2mg_kernel* kernel,
                     const h2mg_build_opts* opts, hipStream_t stream, H2** out,
                     const double* scale_dev, const double* diag_dev) {
  if (!points_dev || !kernel || !opts || !out) return fail(H2MG_ERR_INVALID_ARG, "null argument");
  if (kernel->kind < 0 || kernel->kind > 3) return fail(H2MG_ERR_INVALID_ARG, "unknown kernel kind %d", kernel->kind);
  if (kernel->derivative < 0 || kernel->derivative > 2)
    return fail(H2MG_ERR_INVALID_ARG, "unknown kernel derivative %d", kernel->derivative);
  if (kernel->kind == KER_LAPLACE && kernel->derivative != 0)
    return fail(H2MG_ERR_INVALID_ARG, "the Laplace kernel has no derivative kernels");
  if (!(kernel->length_scale > 0.0) || !std::isfinite(kernel->length_scale))
    return fail(H2MG_ERR_INVALID_ARG, "length_scale must be finite and > 0");
  if (!(kernel->shift >= 0.0) || !std::isfinite(kernel->shift))
    return fail(H2MG_ERR_INVALID_ARG, "shift must be finite and >= 0");
  if (n < 1 || dim < 1 || dim > 3) return fail(H2MG_ERR_INVALID_ARG, "bad n or dim");
  if (opts->leaf_size > 256)
    return fail(H2MG_ERR_INVALID_ARG, "leaf_size must be <= 256 (got %d)", opts->leaf_size);

  std::vector<double> pts_h(size_t(n) * dim), scale_h, diag_h;
  hipError_t e = hipMemcpyAsync(pts_h.data(), points_dev, pts_h.size() * sizeof(double),
                                hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && scale_dev) {
    scale_h.resize(n);
    e = hipMemcpyAsync(scale_h.data(), scale_dev, n * sizeof(double), hipMemcpyDeviceToHost, stream);
  }
  if (e == hipSuccess && diag_dev) {
    diag_h.resize(n);
    e = hipMemcpyAsync(diag_h.data(), diag_dev, n * sizeof(double), hipMemcpyDeviceToHost, stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return fail(H2MG_ERR_HIP, "copying points to the host: %s", hipGetErrorString(e));
  for (double v : scale_h)
    if (!(v > 0.0) || !std::isfinite(v)) return fail(H2MG_ERR_INVALID_ARG, "scale must be finite and > 0");
  for (double v : diag_h)
    if (!std::isfinite(v)) return fail(H2MG_ERR_INVALID_ARG, "diag must be finite");

  H2* hp = new (std::nothrow) H2();
  if (!hp) return fail(H2MG_ERR_OOM, "host allocation failed");
  H2& h = *hp;
  h2mg_status st = build_plan(pts_h.data(), n, dim, opts, &h.plan);
  if (st != H2MG_OK) {
    delete hp;
    return st;
  }
  try {
    const Plan& P = h.plan;
    h.stream = stream;
    h.n = int(n);
    h.dim = dim;
    h.r = P.r;
    h.m = P.m;
    h.L = P.L;
    h.d_top = P.d_top;
    h.T = tile_T(h.r);
    h.nleaf = 1 << h.L;
    h.leaf_max = P.leaf_max;
    h.ngid = (1 << (h.L + 1)) - 1;
    h.kernel = *kernel;
    h.opts = *opts;
    h.kp.kind = kernel->kind;
    h.kp.deriv = kernel->derivative;
    h.kp.inv_l = 1.0 / kernel->length_scale;
    h.kp.inv_2l2 = 1.0 / (2.0 * kernel->length_scale * kernel->length_scale);
    h.kp.shift = kernel->shift;

    // ---- geometry
    std::vector<double> ptree(size_t(n) * dim);
    for (int64_t i = 0; i < n; ++i)
      for (int a = 0; a < dim; ++a) ptree[i * dim + a] = pts_h[P.perm[i] * dim + a];
    h.pts = upload(h, ptree);
    h.perm = upload(h, P.perm);
    auto tree_order = [&](const std::vector<double>& v) {
      std::vector<double> t(v.size());
      for (int64_t i = 0; i < n; ++i) t[i] = v[P.perm[i]];
      return t;
    };
    if (!scale_h.empty()) h.scale = upload(h, tree_order(scale_h));
    if (!diag_h.empty()) h.diag = upload(h, tree_order(diag_h));
    std::vector<int> loff(h.nleaf + 1);
    for (int j = 0; j <= h.nleaf; ++j) loff[j] = int(P.offsets[h.L][j]);
    h.leaf_off = upload(h, loff);
    double Hmax = 0.0;
    for (int a = 0; a < dim; ++a) Hmax = std::max(Hmax, 0.5 * (P.hi[0][a] - P.lo[0][a]));
    const double floor_h = 1e-9 * Hmax;
    std::vector<double> cb(size_t(h.ngid) * dim), hb(size_t(h.ngid) * dim);
    for (int d = 0; d <= h.L; ++d)
      for (int j = 0; j < (1 << d); ++j) {
        const int g = (1 << d) - 1 + j;
        for (int a = 0; a < dim; ++a) {
          const double lo = P.lo[d][j * dim + a], hi = P.hi[d][j * dim + a];
          cb[size_t(g) * dim + a] = 0.5 * (lo + hi);
          hb[size_t(g) * dim + a] = std::max(0.5 * (hi - lo), floor_h);
        }
      }
    h.cbox = upload(h, cb);
    h.hbox = upload(h, hb);
    std::vector<double> t(h.m);
    for (int k = 0; k < h.m; ++k) t[k] = std::cos((2.0 * k + 1.0) * M_PI / (2.0 * h.m));
    h.nodes1d = upload(h, t);

    // ---- stored blocks (upper triangle): S of depths d_top..L, then Pi
    h.s_first.assign(h.L + 1, 0);
    h.s_count.assign(h.L + 1, 0);
    h.p_first.assign(h.L + 1, 0);
    h.p_count.assign(h.L + 1, 0);
    const int dlo = h.d_top < 0 ? h.L + 1 : h.d_top;
    for (int pass = 0; pass < 2; ++pass)
      for (int d = dlo; d <= h.L; ++d) {
        const auto& lst = pass == 0 ? P.far[d] : P.near[d];
        const int gid0 = (1 << d) - 1;
        (pass == 0 ? h.s_first : h.p_first)[d] = int(h.blk_row_h.size());
        for (size_t i = 0; i < lst.size(); i += 2)
          if (lst[i] <= lst[i + 1]) {
            h.blk_row_h.push_back(gid0 + lst[i]);
            h.blk_col_h.push_back(gid0 + lst[i + 1]);
          }
        (pass == 0 ? h.s_count : h.p_count)[d] =
            int(h.blk_row_h.size()) - (pass == 0 ? h.s_first : h.p_first)[d];
      }
    h.nblk = int(h.blk_row_h.size());
    h.blk_row = upload(h, h.blk_row_h);
    h.blk_col = upload(h, h.blk_col_h);
    h.blk_slot_h.assign(h.nblk, -1);
    h.sview.resize(h.L + 1);
    h.pview.resize(h.L + 1);
    h.coarse_launch.resize(h.L + 1);
    if (h.d_top >= 0) {
      for (int d = h.d_top; d <= h.L; ++d) {
        h.sview[d] = make_view(h, d, h.s_first[d], h.s_count[d]);
        h.pview[d] = make_view(h, d, h.p_first[d], h.p_count[d]);
      }
      h.blk_slot = upload(h, h.blk_slot_h);
      std::vector<const View*> vs;
      for (int d = h.d_top; d <= h.L; ++d) vs.push_back(&h.sview[d]);
      h.fine_launch = make_launch(h, vs);
      for (int d = h.d_top; d <= h.L; ++d) {
        std::vector<const View*> cv;
        for (int q = h.d_top; q < d; ++q) cv.push_back(&h.sview[q]);
        cv.push_back(&h.pview[d]);
        cv.push_back(&h.sview[d]);
        h.coarse_launch[d] = make_launch(h, cv);
      }
    }

    // ---- close leaf pairs for the near field
    {
      const auto& lst = P.near[h.L];
      std::vector<int> prow, pcol;
      for (size_t i = 0; i < lst.size(); i += 2)
        if (lst[i] <= lst[i + 1]) {
          prow.push_back(lst[i]);
          pcol.push_back(lst[i + 1]);
        }
      NearField& nf = h.near;
      nf.npairs = int(prow.size());
      std::vector<int> task, rtp(h.nleaf + 1, 0), cptr(h.nleaf + 1, 0), cpair;
      for (int p = 0; p < nf.npairs;) {
        int e2 = p;
        while (e2 < nf.npairs && prow[e2] == prow[p]) ++e2;
        for (int c = p; c < e2; c += NEAR_CHUNK) {
          task.push_back(prow[p]);
          task.push_back(c);
          task.push_back(std::min(e2, c + NEAR_CHUNK));
          rtp[prow[p] + 1]++;
        }
        p = e2;
      }
      for (int i = 0; i < h.nleaf; ++i) rtp[i + 1] += rtp[i];
      for (int p = 0; p < nf.npairs; ++p)
        if (pcol[p] != prow[p]) cptr[pcol[p] + 1]++;
      for (int i = 0; i < h.nleaf; ++i) cptr[i + 1] += cptr[i];
      cpair.resize(cptr[h.nleaf]);
      std::vector<int> fill(cptr.begin(), cptr.end() - 1);
      for (int p = 0; p < nf.npairs; ++p)
        if (pcol[p] != prow[p]) cpair[fill[pcol[p]]++] = p;
      nf.ntasks = int(task.size() / 3);
      nf.task = upload(h, task);
      nf.pair_col = upload(h, pcol);
      nf.row_task_ptr = upload(h, rtp);
      nf.col_ptr = upload(h, cptr);
      nf.col_pair = upload(h, cpair);
      nf.ld = (h.leaf_max + 7) / 8 * 8;
      for (int p = 0; p < nf.npairs; ++p)
        h.near_evals += int64_t(loff[prow[p] + 1] - loff[prow[p]]) * (loff[pcol[p] + 1] - loff[pcol[p]]);
    }

    // ---- workspace
    const size_t rr = size_t(h.r);
    h.xall = h.arena.make<double>(size_t(h.ngid) * rr);
    h.yall = h.arena.make<double>(size_t(h.ngid) * rr);
    h.partial = h.arena.make<double>(size_t(std::max(h.max_tasks, 1)) * rr);
    h.colpart = h.arena.make<double>(size_t(std::max(h.nslot, 1)) * rr);
    h.near_partial = h.arena.make<double>(size_t(std::max(h.near.ntasks, 1)) * h.near.ld);
    h.near_colpart = h.arena.make<double>(size_t(std::max(h.near.npairs, 1)) * h.near.ld);
    h.vtree = h.arena.make<double>(h.n);
    h.vtree2 = h.arena.make<double>(h.n);
    h.flags = h.arena.make<int>(4);
    h.dot_part = h.arena.make<double>(8 * 512);
    hip_check(hipMemsetAsync(h.flags, 0, 4 * sizeof(int), h.stream), "memset");
    hip_check(hipMemsetAsync(h.yall, 0, size_t(h.ngid) * rr * sizeof(double), h.stream), "memset");

    // ---- FP64 operator storage
    const int64_t te = tile_elems(h.T);
    PrecData& p64 = h.prec[P64];
    p64.Qr = h.arena.make<double>(size_t(h.n) * rr);
    p64.Qc = h.arena.make<double>(size_t(h.n) * rr);
    p64.E = h.arena.make<double>(size_t(h.ngid) * te);
    p64.blk = h.arena.make<double>(size_t(std::max(h.nblk, 1)) * te);
    hip_check(hipMemsetAsync(p64.E, 0, size_t(h.ngid) * te * sizeof(double), h.stream), "memset");
    hip_check(hipMemsetAsync(p64.blk, 0, size_t(std::max(h.nblk, 1)) * te * sizeof(double), h.stream),
              "memset");
    h.R = h.arena.make<double>(size_t(h.ngid) * rr * rr);

    // ---- setup kernels
    launch_leaf_basis_qr(h);
    if (h.d_top >= 0) {
      for (int d = h.L - 1; d >= h.d_top; --d) launch_transfer_qr(h, d);
      for (int d = h.d_top; d <= h.L; ++d) launch_couplings(h, d);
    }
    hip_check(hipStreamSynchronize(h.stream), "build");
    h.arena.release(h.R);
    h.R = nullptr;
    p64.ready = true;
  } catch (const std::bad_alloc&) {
    delete hp;
    return fail(H2MG_ERR_OOM, "device allocation failed while building the H2 matrix");
  } catch (const std::exception& ex) {
    delete hp;
    return fail(H2MG_ERR_HIP, "%s", ex.what());
  }
  *out = hp;
  return H2MG_OK;
}

h2mg_status build_derivative(H2& h, int which, H2** out) {
  if (which != 1 && which != 2) return fail(H2MG_ERR_INVALID_ARG, "derivative must be 1 or 2 (got %d)", which);
  if (h.kp.kind == KER_LAPLACE || h.scale || h.diag || h.nq > 0)
    return fail(H2MG_ERR_INVALID_ARG, "derivative kernels exist for the exp, Gauss and Matern kernels "
                                      "without per-point scale or diagonal");
  double* user = nullptr;
  try {
    user = h.arena.make<double>(size_t(h.n) * h.dim);
    launch_scatter_rows(h, h.pts, user);
    hip_check(hipStreamSynchronize(h.stream), "scatter points");
  } catch (const std::bad_alloc&) {
    return fail(H2MG_ERR_OOM, "device allocation failed");
  } catch (const std::exception& ex) {
    return fail(H2MG_ERR_HIP, "%s", ex.what());
  }
  h2mg_kernel k = h.kernel;
  k.derivative = which;
  k.shift = 0.0;
  const h2mg_status st = build_h2(user, h.n, h.dim, &k, &h.opts, h.stream, out);
  h.arena.release(user);
  if (st == H2MG_OK && (*out)->plan.perm != h.plan.perm) {
    delete *out;
    *out = nullptr;
    return fail(H2MG_ERR_HIP, "derivative build produced a different tree");
  }
  return st;
}

h2mg_status quadratic_gradient(H2& h, H2* hl, H2* hg, const double* b, const double* x, double scale,
                               double* loss, double* grad_l, double* grad_s, double* grad_p,
                               double* grad_b) {
  auto same_points = [&](const H2* d) {
    return d->n == h.n && d->dim == h.dim && d->plan.perm == h.plan.perm;
  };
  if (grad_l && (!hl || !same_points(hl) || hl->kp.deriv != DER_LENGTH))
    return fail(H2MG_ERR_INVALID_ARG, "dL/dl needs h_dl, the length-scale derivative on the same points");
  if (grad_p && (!hg || !same_points(hg) || hg->kp.deriv != DER_RADIAL))
    return fail(H2MG_ERR_INVALID_ARG, "dL/dp needs h_g, the radial derivative on the same points");
  const int64_t n = h.n;
  const int np = dot_parts(n);
  auto host_sum = [&](const double* part) {
    std::vector<double> v(np);
    hip_check(hipMemcpyAsync(v.data(), part, np * sizeof(double), hipMemcpyDeviceToHost, h.stream),
              "readback");
    hip_check(hipStreamSynchronize(h.stream), "sync");
    double acc = 0.0;
    for (double t : v) acc += t;
    return acc;
  };
  double* u = nullptr;
  double* w = nullptr;
  try {
    // L = b^T x, dL/ds = -x^T x (user order)
    launch_dot(h, P64, n, b, x, h.dot_part);
    const double L = host_sum(h.dot_part);
    launch_dot(h, P64, n, x, x, h.dot_part);
    const double xx = host_sum(h.dot_part);
    if (loss) *loss = L;
    if (grad_s) *grad_s = -scale * xx;
    // dL/dl = -x^T (dA/dl) x (tree order)
    if (grad_l) {
      H2& dl = *hl;
      dl.stream = h.stream;
      launch_gather(dl, x, dl.vtree);
      apply_fine(dl, P64, dl.vtree, dl.vtree2, 1.0, nullptr, 0.0);
      launch_dot(dl, P64, n, dl.vtree, dl.vtree2, h.dot_part);
      *grad_l = -scale * host_sum(h.dot_part);
    }
    // dL/dp_ia = -2 x_i [p_ia (G x)_i - (G (x * p_.a))_i]
    if (grad_p) {
      H2& g = *hg;
      g.stream = h.stream;
      u = g.arena.make<double>(n);
      w = g.arena.make<double>(n);
      launch_gather(g, x, g.vtree);
      apply_fine(g, P64, g.vtree, g.vtree2, 1.0, nullptr, 0.0);
      for (int a = 0; a < h.dim; ++a) {
        launch_coord_mul(g, a, g.vtree, w);
        apply_fine(g, P64, w, u, 1.0, nullptr, 0.0);
        launch_coord_grad(g, a, scale, g.vtree, g.vtree2, u, grad_p);
      }
    }
    if (grad_b) launch_axpby(h, P64, n, 2.0 * scale, x, 0.0, grad_b);
    hip_check(hipStreamSynchronize(h.stream), "gradient");
  } catch (const std::bad_alloc&) {
    if (u) hg->arena.release(u);
    if (w) hg->arena.release(w);
    return fail(H2MG_ERR_OOM, "device allocation failed in the gradient");
  } catch (const std::exception& ex) {
    (void)hipStreamSynchronize(h.stream);
    if (u) hg->arena.release(u);
    if (w) hg->arena.release(w);
    return fail(H2MG_ERR_HIP, "%s", ex.what());
  }
  if (u) hg->arena.release(u);
  if (w) hg->arena.release(w);
  return H2MG_OK;
}

void release_block_work(H2& h) {
  for (void* p : h.blk16.owned) h.arena.release(p);
  h.blk16 = BlockWork();
}

namespace {

void release_stored_near(H2& h) {
  release_block_work(h);               // its near-field task lists refer to the tiles
  for (void* p : h.snear.owned) h.arena.release(p);
  h.snear = StoredNear();
}

}  // namespace

void plan_near(H2& h) {
  StoredNear& sn = h.snear;
  if (sn.planned) return;
  auto own = [&](auto* p) {
    sn.owned.push_back(static_cast<void*>(p));
    return p;
  };
  const Plan& P = h.plan;
  const auto& off = P.offsets[h.L];
  // chunks of at most 64 points per leaf
  std::vector<int> cbase(h.nleaf + 1, 0), cstart, cn;
  sn.identity = true;
  for (int s = 0; s < h.nleaf; ++s) {
    const int s0 = int(off[s]), ns = int(off[s + 1] - off[s]);
    const int k = (ns + 63) / 64;
    if (ns % 64 != 0) sn.identity = false;
    for (int q = 0; q < k; ++q) {
      cstart.push_back(s0 + 64 * q);
      cn.push_back(std::min(64, ns - 64 * q));
    }
    cbase[s + 1] = cbase[s] + k;
  }
  sn.nchunk = cbase[h.nleaf];
  // tiles sorted by (row chunk, column chunk): row leaf, its row chunk,
  // then the leaf's close partners t >= s in order, then their chunks
  const auto& lst = P.near[h.L];
  std::vector<int> brow, bcol;
  for (size_t p = 0; p < lst.size();) {
    const int64_t s = lst[p];
    size_t e = p;
    while (e < lst.size() && lst[e] == s) e += 2;
    const int ks = cbase[s + 1] - cbase[s];
    for (int i = 0; i < ks; ++i)
      for (size_t q = p; q < e; q += 2) {
        const int64_t t = lst[q + 1];
        if (t < s) continue;
        for (int j = (t == s ? i : 0); j < cbase[t + 1] - cbase[t]; ++j) {
          brow.push_back(cbase[s] + i);
          bcol.push_back(cbase[t] + j);
        }
      }
    p = e;
  }
  sn.nblocks = int64_t(brow.size());
  // tasks of at most CHUNK tiles of one row chunk; column slots by column
  std::vector<int> task, rtp(sn.nchunk + 1, 0), cptr(sn.nchunk + 1, 0), slot(brow.size(), -1);
  for (size_t b = 0; b < brow.size();) {
    size_t e = b;
    while (e < brow.size() && brow[e] == brow[b]) ++e;
    for (size_t c = b; c < e; c += CHUNK) {
      task.push_back(brow[b]);
      task.push_back(int(c));
      task.push_back(int(std::min(e, c + CHUNK)));
      rtp[brow[b] + 1]++;
    }
    b = e;
  }
  for (int i = 0; i < sn.nchunk; ++i) rtp[i + 1] += rtp[i];
  for (size_t b = 0; b < brow.size(); ++b)
    if (bcol[b] != brow[b]) cptr[bcol[b] + 1]++;
  for (int i = 0; i < sn.nchunk; ++i) cptr[i + 1] += cptr[i];
  std::vector<int> fill(cptr.begin(), cptr.end() - 1);
  for (size_t b = 0; b < brow.size(); ++b)
    if (bcol[b] != brow[b]) slot[b] = fill[bcol[b]]++;
  sn.nslot = cptr[sn.nchunk];
  sn.ntasks = int(task.size() / 3);

  sn.brow_h = brow;
  sn.bcol_h = bcol;
  sn.chunk_base = own(upload(h, cbase));
  sn.chunk_start = own(upload(h, cstart));
  sn.chunk_n = own(upload(h, cn));
  sn.blk_row = own(upload(h, brow));
  sn.blk_col = own(upload(h, bcol));
  sn.blk_slot = own(upload(h, slot));
  sn.task = own(upload(h, task));
  sn.row_task_ptr = own(upload(h, rtp));
  sn.col_ptr = own(upload(h, cptr));
  hip_check(hipStreamSynchronize(h.stream), "near plan");
  sn.planned = true;
}

h2mg_status store_near(H2& h, int enable) {
  if (!enable && h.nq > 0)
    return fail(H2MG_ERR_STATE, "close entries given by quadrature are applied from the stored tiles only");
  if (!enable) {
    hip_check(hipStreamSynchronize(h.stream), "store_near");
    release_stored_near(h);
    return H2MG_OK;
  }
  if (h.snear.ready) return H2MG_OK;
  StoredNear& sn = h.snear;
  auto own = [&](auto* p) {
    sn.owned.push_back(static_cast<void*>(p));
    return p;
  };
  try {
    plan_near(h);
    const size_t nvec = size_t(sn.nchunk) * 64;
    sn.partial = own(h.arena.make<double>(size_t(std::max(sn.ntasks, 1)) * 64));
    sn.colpart = own(h.arena.make<double>(size_t(std::max(sn.nslot, 1)) * 64));
    sn.yc = own(h.arena.make<double>(nvec));
    if (!sn.identity) {
      sn.xc = own(h.arena.make<double>(nvec));
      hip_check(hipMemsetAsync(sn.xc, 0, nvec * sizeof(double), h.stream), "memset");
    }
    sn.tiles = own(h.arena.make<double>(size_t(std::max<int64_t>(sn.nblocks, 1)) * tile_elems(8)));
    launch_near_tiles(h);
    hip_check(hipStreamSynchronize(h.stream), "near_tiles");
    sn.ready = true;
  } catch (const std::bad_alloc&) {
    (void)hipStreamSynchronize(h.stream);
    release_stored_near(h);
    return fail(H2MG_ERR_OOM, "device allocation failed while storing the near field");
  } catch (const std::exception& ex) {
    (void)hipStreamSynchronize(h.stream);
    release_stored_near(h);
    return fail(H2MG_ERR_HIP, "%s", ex.what());
  }
  return H2MG_OK;
}

h2mg_status set_near_quadrature(H2& h, const double* qy_user, const double* qu_user, int nq) {
  if (nq < 1 || nq > 64) return fail(H2MG_ERR_INVALID_ARG, "quadrature points per point must be 1..64 (got %d)", nq);
  if (h.nq > 0) return fail(H2MG_ERR_STATE, "the close entries already have a quadrature");
  if (h.mg_built || h.snear.ready || h.bj_built[P64] || h.blk16.ready)
    return fail(H2MG_ERR_STATE, "set the quadrature of the close entries right after the build");
  try {
    h.qy = h.arena.make<double>(size_t(h.n) * nq * h.dim);
    h.qu = h.arena.make<double>(size_t(h.n) * nq);
    launch_gather_rows(h, nq * h.dim, qy_user, h.qy);
    launch_gather_rows(h, nq, qu_user, h.qu);
    hip_check(hipStreamSynchronize(h.stream), "quadrature");
  } catch (const std::bad_alloc&) {
    return fail(H2MG_ERR_OOM, "device allocation failed for the quadrature");
  } catch (const std::exception& ex) {
    return fail(H2MG_ERR_HIP, "%s", ex.what());
  }
  h.nq = nq;
  const h2mg_status st = store_near(h, 1);
  if (st != H2MG_OK) {
    h.arena.release(h.qy);
    h.arena.release(h.qu);
    h.qy = h.qu = nullptr;
    h.nq = 0;
  }
  return st;
}

h2mg_status setup_mg(H2& h, int precision_mask) {
  try {
    if (!h.mg_built) {
      if (h.d_top >= 0) {
        launch_pi_leaf(h);
        // child block lookup: (row gid, col gid) -> block id.  The coupling
        // and close blocks of a depth are each sorted by (row, column) (the
        // plan sorts its pair lists), so a binary search finds a child.
        auto key = [](int a, int b) { return (int64_t(a) << 32) | uint32_t(b); };
        auto find_block = [&](int first, int count, int64_t k) {
          int lo = first, hi = first + count;
          while (lo < hi) {
            const int mid = lo + (hi - lo) / 2;
            if (key(h.blk_row_h[mid], h.blk_col_h[mid]) < k) lo = mid + 1;
            else hi = mid;
          }
          return lo < first + count && key(h.blk_row_h[lo], h.blk_col_h[lo]) == k ? lo : -1;
        };
        // all maps first (host work that may throw), then the launches
        std::vector<std::vector<int>> host_maps;   // alive until the copies are done
        for (int d = h.L - 1; d >= h.d_top; --d) {
          auto child = [&](int cs, int ct) {
            const int64_t k = key(cs, ct);
            int b = find_block(h.s_first[d + 1], h.s_count[d + 1], k);
            if (b < 0) b = find_block(h.p_first[d + 1], h.p_count[d + 1], k);
            if (b < 0) throw std::runtime_error("child block not found");
            return b;
          };
          host_maps.emplace_back();
          std::vector<int>& cmap = host_maps.back();
          cmap.reserve(size_t(h.p_count[d]) * 4);
          for (int b = h.p_first[d]; b < h.p_first[d] + h.p_count[d]; ++b) {
            const int gs = h.blk_row_h[b], gt = h.blk_col_h[b];
            for (int a = 0; a < 2; ++a)
              for (int bb = 0; bb < 2; ++bb) {
                const int cs = 2 * gs + 1 + a, ct = 2 * gt + 1 + bb;
                cmap.push_back(cs <= ct ? child(cs, ct) : -child(ct, cs) - 1);
              }
          }
        }
        std::vector<int*> maps;
        for (int d = h.L - 1, k = 0; d >= h.d_top; --d, ++k) {
          maps.push_back(upload(h, host_maps[k]));
          // stream order: depth d reads the blocks depth d + 1 wrote
          launch_pi_upper(h, d, maps.back());
        }
        hip_check(hipStreamSynchronize(h.stream), "pi_upper");
        for (int* m : maps) h.arena.release(m);
        h.Nl = int64_t(1 << h.d_top) * h.r;
        h.levels = h.L - h.d_top + 2;
      } else {
        if (h.n > 32768)
          return fail(H2MG_ERR_INVALID_ARG,
                      "no far blocks: the dense direct solve is limited to n <= 32768");
        h.Nl = h.n;
        h.levels = 1;
      }
      h.chol = h.arena.make<double>(size_t(h.Nl) * h.Nl);
      hip_check(hipMemsetAsync(h.chol, 0, size_t(h.Nl) * h.Nl * sizeof(double), h.stream), "memset");
      if (h.d_top >= 0) launch_assemble_dense(h, h.chol, h.Nl);
      else launch_assemble_kernel_dense(h, h.chol, h.Nl);
      hip_check(hipMemsetAsync(h.flags, 0, 4 * sizeof(int), h.stream), "memset");
      launch_potrf(h, h.chol, h.Nl);
      int flags[4];
      hip_check(hipMemcpyAsync(flags, h.flags, sizeof(flags), hipMemcpyDeviceToHost, h.stream), "flags");
      hip_check(hipStreamSynchronize(h.stream), "setup_mg");
      if (flags[0]) {
        h.arena.release(h.chol);
        h.chol = nullptr;
        return fail(H2MG_ERR_NOT_SPD, "the coarsest operator (order %lld) is not positive definite",
                    (long long)h.Nl);
      }
      h.mg_built = true;
    }
    for (int p = P32; p <= P16; ++p) {
      if (!(precision_mask & (1 << p)) || h.prec[p].ready) continue;
      const size_t eb = elem_bytes(p);
      const int64_t te = tile_elems(h.T);
      PrecData& pd = h.prec[p];
      pd.Qr = h.arena.alloc(size_t(h.n) * h.r * eb);
      pd.Qc = h.arena.alloc(size_t(h.n) * h.r * eb);
      pd.E = h.arena.alloc(size_t(h.ngid) * te * eb);
      pd.blk = h.arena.alloc(size_t(std::max(h.nblk, 1)) * te * eb);
      hip_check(hipMemsetAsync(pd.E, 0, size_t(h.ngid) * te * eb, h.stream), "memset");
      hip_check(hipMemsetAsync(pd.blk, 0, size_t(std::max(h.nblk, 1)) * te * eb, h.stream), "memset");
      launch_cast_precision(h, p);
      hip_check(hipStreamSynchronize(h.stream), "cast");
      pd.ready = true;
    }
    // close entries by quadrature cannot be evaluated in the low-precision
    // products: they read an FP32 copy of the stored tiles
    if ((precision_mask & ((1 << P32) | (1 << P16))) && h.nq > 0 && h.snear.ready && !h.snear.tiles32) {
      StoredNear& sn = h.snear;
      sn.tiles32 = h.arena.make<float>(size_t(std::max<int64_t>(sn.nblocks, 1)) * tile_elems(8));
      sn.owned.push_back(sn.tiles32);
      if (!sn.identity) {
        // the padding must stay zero (a padded tile column times a non-finite
        // leftover would not vanish)
        const size_t nvec = size_t(sn.nchunk) * 64;
        sn.xc32 = h.arena.make<float>(nvec);
        sn.owned.push_back(sn.xc32);
        hip_check(hipMemsetAsync(sn.xc32, 0, nvec * sizeof(float), h.stream), "memset");
      }
      launch_cast_near_tiles(h);
      hip_check(hipStreamSynchronize(h.stream), "cast near tiles");
    }
  } catch (const std::bad_alloc&) {
    return fail(H2MG_ERR_OOM, "device allocation failed while building the hierarchy");
  } catch (const std::exception& ex) {
    return fail(H2MG_ERR_HIP, "%s", ex.what());
  }
  return H2MG_OK;
}

}  // namespace h2mg
