// Products with the H2 matrix (Section 3.1, matvec recursion after eq. h2)
// and with the restricted operators (Section 3.3, eq. a2_str), and the level
// transfers of Algorithm 1.
#include <hip/hip_runtime.h>

#include <stdexcept>

#include "h2_build.h"

namespace h2mg {

namespace {

inline size_t vbytes(int p) { return p == P64 ? 8 : 4; }

// Pointer to the coefficients of depth d inside a gid-indexed buffer.
inline void* at_depth(void* base, int p, int d, int r) {
  return static_cast<char*>(base) + size_t((1 << d) - 1) * r * vbytes(p);
}
inline const void* at_depth(const void* base, int p, int d, int r) {
  return static_cast<const char*>(base) + size_t((1 << d) - 1) * r * vbytes(p);
}

}  // namespace

void apply_fine(H2& h, int p, const void* xt, void* out, double alpha, const void* add, double beta) {
  void* xall = h.xall;
  void* yall = h.yall;
  const int r = h.r;
  if (h.d_top >= 0) {
    // upsweep: x_L = Q^T x, then x_d = E^T x_{d+1}
    launch_leaf_up(h, p, xt, at_depth(xall, p, h.L, r));
    for (int d = h.L - 1; d >= h.d_top; --d)
      launch_transfer_up(h, p, d, at_depth(xall, p, d + 1, r), at_depth(xall, p, d, r));
    // couplings of every depth in one launch
    launch_gemv(h, p, h.fine_launch, xall);
    // downsweep: y_d = S_d x_d + E y_{d-1}
    for (int d = h.d_top; d <= h.L; ++d) {
      const void* addend = nullptr;
      if (d > h.d_top) {
        launch_transfer_down(h, p, d - 1, at_depth(yall, p, d - 1, r), at_depth(yall, p, d, r), nullptr);
        addend = at_depth(yall, p, d, r);
      }
      launch_reduce(h, p, d, &h.sview[d], h.fine_launch.base[d - h.d_top], nullptr, 0, addend,
                    at_depth(yall, p, d, r));
    }
  }
  // near field and leaf downsweep: y = D x + Q y_L
  launch_near(h, p, xt);
  launch_fine_reduce(h, p, at_depth(yall, p, h.L, r), out, false, alpha, add, beta);
}

void apply_coarse(H2& h, int p, int k, const void* x, void* y) {
  const int d = h.level_depth(k);
  const int r = h.r;
  void* xall = h.xall;
  void* yall = h.yall;
  launch_copy(h, p, x, at_depth(xall, p, d, r), int64_t(1 << d) * r);
  for (int q = d - 1; q >= h.d_top; --q)
    launch_transfer_up(h, p, q, at_depth(xall, p, q + 1, r), at_depth(xall, p, q, r));
  const Launch& l = h.coarse_launch[d];
  launch_gemv(h, p, l, xall);
  for (int q = h.d_top; q <= d; ++q) {
    const void* addend = nullptr;
    if (q > h.d_top) {
      launch_transfer_down(h, p, q - 1, at_depth(yall, p, q - 1, r), at_depth(yall, p, q, r), nullptr);
      addend = at_depth(yall, p, q, r);
    }
    if (q < d) {
      launch_reduce(h, p, q, &h.sview[q], l.base[q - h.d_top], nullptr, 0, addend,
                    at_depth(yall, p, q, r));
    } else {
      const int nv = d - h.d_top;   // views before Pi_d
      launch_reduce(h, p, d, &h.pview[d], l.base[nv], &h.sview[d], l.base[nv + 1], addend, y);
    }
  }
}

void apply_level(H2& h, int p, int k, const void* x, void* y) {
  if (k == 1) apply_fine(h, p, x, y, 1.0, nullptr, 0.0);
  else apply_coarse(h, p, k, x, y);
}

void restrict_level(H2& h, int p, int k, const void* r, void* r_next) {
  if (k == 1) launch_leaf_up(h, p, r, r_next);
  else launch_transfer_up(h, p, h.level_depth(k) - 1, r, r_next);
}

void prolong_level(H2& h, int p, int k, const void* e_next, void* e, const void* add, double beta) {
  if (k == 1) launch_leaf_down(h, p, e_next, e, 1.0, add, beta);
  else {
    if (add && beta != 1.0) throw std::runtime_error("prolongation supports beta = 1 only");
    launch_transfer_down(h, p, h.level_depth(k) - 1, e_next, e, add);
  }
}

}  // namespace h2mg
