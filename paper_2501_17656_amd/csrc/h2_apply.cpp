// Products with the H2 matrix (Section 3.1, matvec recursion after eq. h2)
// and with the restricted operators (Section 3.3, eq. a2_str), and the level
// transfers of Algorithm 1.
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <vector>

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
    // couplings of every depth in one launch, then one reduce for all depths
    launch_gemv(h, p, h.fine_launch, xall);
    std::vector<const View*> vs;
    std::vector<int> bs;
    for (int d = h.d_top; d <= h.L; ++d) {
      vs.push_back(&h.sview[d]);
      bs.push_back(h.fine_launch.base[d - h.d_top]);
    }
    launch_reduce(h, p, h.d_top, h.L, vs.data(), bs.data(), nullptr, nullptr, yall, nullptr);
    // downsweep: y_d += E y_{d-1}
    for (int d = h.d_top + 1; d <= h.L; ++d)
      launch_transfer_down(h, p, d - 1, at_depth(yall, p, d - 1, r), at_depth(yall, p, d, r),
                           at_depth(yall, p, d, r));
  }
  // near field and leaf downsweep: y = D x + Q y_L
  if (near_stored_for(h, p)) launch_near_stored(h, p, xt);
  else launch_near(h, p, xt);
  launch_fine_reduce(h, p, at_depth(yall, p, h.L, r), out, false, alpha, add, beta, xt);
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
  // partial sums of every depth: S_q for q < d, Pi_d and S_d at depth d
  std::vector<const View*> v0, v1;
  std::vector<int> b0, b1;
  for (int q = h.d_top; q < d; ++q) {
    v0.push_back(&h.sview[q]);
    b0.push_back(l.base[q - h.d_top]);
    v1.push_back(nullptr);
    b1.push_back(0);
  }
  const int nv = d - h.d_top;
  v0.push_back(&h.pview[d]);
  b0.push_back(l.base[nv]);
  v1.push_back(&h.sview[d]);
  b1.push_back(l.base[nv + 1]);
  launch_reduce(h, p, h.d_top, d, v0.data(), b0.data(), v1.data(), b1.data(), yall,
                d == h.d_top ? y : nullptr);
  // downsweep, the last step writing the output
  for (int q = h.d_top + 1; q <= d; ++q)
    launch_transfer_down(h, p, q - 1, at_depth(yall, p, q - 1, r), q == d ? y : at_depth(yall, p, q, r),
                         at_depth(yall, p, q, r));
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
