// Host-side cluster tree and block partition (Section 3.1).
//
// The paper partitions the index set into M leaf blocks, groups p of them
// per coarser block, and separates close (full-rank) from far (low-rank)
// blocks under strong admissibility without giving the construction.  This
// file builds a binary tree of uniform depth by median bisection and the
// close/far lists by a level-by-level dual traversal.  Compiled without
// floating-point contraction so the box tests round exactly like plain
// IEEE arithmetic, operation by operation.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>

namespace h2mg {

static thread_local std::string g_last_error;

h2mg_status fail(h2mg_status st, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

const char* last_error_cstr() { return g_last_error.c_str(); }
void clear_error() { g_last_error.clear(); }

namespace {

void tight_box(const double* pts, int dim, const int64_t* idx, int64_t cnt,
               double* lo, double* hi) {
  for (int a = 0; a < dim; ++a) {
    lo[a] = INFINITY;
    hi[a] = -INFINITY;
  }
  for (int64_t k = 0; k < cnt; ++k) {
    const double* p = pts + idx[k] * dim;
    for (int a = 0; a < dim; ++a) {
      lo[a] = std::min(lo[a], p[a]);
      hi[a] = std::max(hi[a], p[a]);
    }
  }
}

// Sum of squares over axes in increasing axis order.
inline double sq_sum(const double* v, int dim) {
  double s = v[0] * v[0];
  for (int a = 1; a < dim; ++a) s = s + v[a] * v[a];
  return s;
}

bool admissible(const double* lo_s, const double* hi_s, const double* lo_t,
                const double* hi_t, int dim, double eta2) {
  double ws[3], wt[3], gap[3];
  for (int a = 0; a < dim; ++a) {
    ws[a] = hi_s[a] - lo_s[a];
    wt[a] = hi_t[a] - lo_t[a];
    double g = std::max(lo_t[a] - hi_s[a], lo_s[a] - hi_t[a]);
    gap[a] = std::max(g, 0.0);
  }
  const double ds = sq_sum(ws, dim), dt = sq_sum(wt, dim);
  const double dist2 = sq_sum(gap, dim);
  return dist2 > 0.0 && std::max(ds, dt) <= eta2 * dist2;
}

void sort_pairs(std::vector<int32_t>& v) {
  const size_t k = v.size() / 2;
  std::vector<int64_t> keys(k);
  for (size_t i = 0; i < k; ++i)
    keys[i] = (int64_t(v[2 * i]) << 32) | uint32_t(v[2 * i + 1]);
  std::sort(keys.begin(), keys.end());
  for (size_t i = 0; i < k; ++i) {
    v[2 * i] = int32_t(keys[i] >> 32);
    v[2 * i + 1] = int32_t(keys[i] & 0xffffffff);
  }
}

}  // namespace

h2mg_status build_plan(const double* points, int64_t n, int dim,
                       const h2mg_build_opts* o, Plan* out) {
  if (!points || !o || !out) return fail(H2MG_ERR_INVALID_ARG, "null argument");
  if (n < 1) return fail(H2MG_ERR_INVALID_ARG, "n must be >= 1 (got %lld)", (long long)n);
  if (n >= (int64_t(1) << 31))
    return fail(H2MG_ERR_INVALID_ARG, "n must be < 2^31 (got %lld)", (long long)n);
  if (dim < 1 || dim > 3) return fail(H2MG_ERR_INVALID_ARG, "dim must be 1, 2 or 3 (got %d)", dim);
  if (o->leaf_size < 1) return fail(H2MG_ERR_INVALID_ARG, "leaf_size must be >= 1");
  if (!(o->eta > 0.0) || !std::isfinite(o->eta))
    return fail(H2MG_ERR_INVALID_ARG, "eta must be finite and > 0");
  if (o->cheb_m < 1) return fail(H2MG_ERR_INVALID_ARG, "cheb_m must be >= 1");
  int64_t r = 1;
  for (int a = 0; a < dim; ++a) r *= o->cheb_m;
  if (r > 64) return fail(H2MG_ERR_INVALID_ARG, "rank cheb_m^dim = %lld exceeds 64", (long long)r);
  for (int64_t i = 0; i < n * dim; ++i)
    if (!std::isfinite(points[i]))
      return fail(H2MG_ERR_INVALID_ARG, "non-finite coordinate at point %lld", (long long)(i / dim));

  try {
    Plan& P = *out;
    P = Plan();
    P.n = n;
    P.dim = dim;
    P.m = o->cheb_m;
    P.r = int(r);
    P.eta = o->eta;
    int L = 0;
    while (int64_t(o->leaf_size) * (int64_t(1) << L) < n) ++L;
    P.L = L;
    P.perm.resize(n);
    for (int64_t i = 0; i < n; ++i) P.perm[i] = i;
    P.offsets.assign(L + 1, {});
    P.offsets[0] = {0, n};
    std::vector<double> lo(dim), hi(dim);
    for (int d = 0; d < L; ++d) {
      const auto& off = P.offsets[d];
      auto& nxt = P.offsets[d + 1];
      nxt.assign(1, 0);
      for (int64_t j = 0; j < (int64_t(1) << d); ++j) {
        const int64_t s = off[j], e = off[j + 1];
        int axis = 0;
        if (e > s) {
          tight_box(points, dim, P.perm.data() + s, e - s, lo.data(), hi.data());
          double best = hi[0] - lo[0];
          for (int a = 1; a < dim; ++a) {
            const double ext = hi[a] - lo[a];
            if (ext > best) { best = ext; axis = a; }
          }
        }
        std::stable_sort(P.perm.begin() + s, P.perm.begin() + e,
                         [&](int64_t u, int64_t v) {
                           return points[u * dim + axis] < points[v * dim + axis];
                         });
        const int64_t nl = (e - s + 1) / 2;
        nxt.push_back(s + nl);
        nxt.push_back(e);
      }
    }
    P.lo.assign(L + 1, {});
    P.hi.assign(L + 1, {});
    for (int d = 0; d <= L; ++d) {
      const int64_t nc = int64_t(1) << d;
      P.lo[d].resize(nc * dim);
      P.hi[d].resize(nc * dim);
      for (int64_t j = 0; j < nc; ++j)
        tight_box(points, dim, P.perm.data() + P.offsets[d][j],
                  P.offsets[d][j + 1] - P.offsets[d][j], &P.lo[d][j * dim], &P.hi[d][j * dim]);
    }
    const auto& lo_off = P.offsets[L];
    P.leaf_min = INT32_MAX;
    P.leaf_max = 0;
    for (int64_t j = 0; j < (int64_t(1) << L); ++j) {
      const int sz = int(lo_off[j + 1] - lo_off[j]);
      P.leaf_min = std::min(P.leaf_min, sz);
      P.leaf_max = std::max(P.leaf_max, sz);
    }
    if (P.leaf_min < P.r)
      return fail(H2MG_ERR_INVALID_ARG,
                  "smallest leaf holds %d points, fewer than the rank %d", P.leaf_min, P.r);

    // Dual traversal, one depth at a time.
    const double eta2 = o->eta * o->eta;
    P.near.assign(L + 1, {});
    P.far.assign(L + 1, {});
    std::vector<int32_t> cur = {0, 0};
    for (int d = 0; d <= L; ++d) {
      const double* LO = P.lo[d].data();
      const double* HI = P.hi[d].data();
      std::vector<int32_t>& nr = P.near[d];
      std::vector<int32_t>& fr = P.far[d];
      for (size_t i = 0; i < cur.size(); i += 2) {
        const int32_t s = cur[i], t = cur[i + 1];
        if (admissible(LO + s * dim, HI + s * dim, LO + t * dim, HI + t * dim, dim, eta2)) {
          fr.push_back(s);
          fr.push_back(t);
        } else {
          nr.push_back(s);
          nr.push_back(t);
        }
      }
      sort_pairs(nr);
      sort_pairs(fr);
      if (!fr.empty() && P.d_top < 0) P.d_top = d;
      if (d < L) {
        std::vector<int32_t> nxt;
        nxt.reserve(nr.size() * 4);
        for (size_t i = 0; i < nr.size(); i += 2)
          for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
              nxt.push_back(2 * nr[i] + a);
              nxt.push_back(2 * nr[i + 1] + b);
            }
        cur.swap(nxt);
      }
    }
  } catch (const std::bad_alloc&) {
    return fail(H2MG_ERR_OOM, "host allocation failed while building the cluster tree");
  }
  return H2MG_OK;
}

}  // namespace h2mg
