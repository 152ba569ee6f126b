// Host-side cluster tree and block partition (Section 3.1).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "h2mg.h"

namespace h2mg {

// Record a message for h2mg_last_error() and return the status.
h2mg_status fail(h2mg_status st, const char* fmt, ...);

struct Plan {
  int64_t n = 0;
  int dim = 0;
  int L = 0;          // leaf depth
  int d_top = -1;     // shallowest depth with a far pair (-1: none)
  int m = 0;          // Chebyshev nodes per axis
  int r = 0;          // rank m^dim
  int leaf_min = 0, leaf_max = 0;
  double eta = 0.0;
  std::vector<int64_t> perm;                  // tree position -> user index
  std::vector<std::vector<int64_t>> offsets;  // [d][j], 2^d + 1 entries
  std::vector<std::vector<double>> lo, hi;    // [d][j * dim + a], tight boxes
  // Pairs (s, t) at depth d, both orders, sorted by (s, t), flattened.
  std::vector<std::vector<int32_t>> near, far;
};

// Tree: uniform depth L = min{L : leaf * 2^L >= n}; each cluster split at
// the median (first ceil(n/2) after a stable sort) along the longest side of
// its tight box (ties: lowest axis).  Partition: dual traversal from the
// root pair; admissible iff dist > 0 and max(diam^2) <= eta^2 dist^2.
h2mg_status build_plan(const double* points, int64_t n, int dim,
                       const h2mg_build_opts* opts, Plan* out);

}  // namespace h2mg
