// Host driver for the cluster tree and block partition (Section 3.1), built
// with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitize.py.  It builds plans for ordinary and degenerate
// point sets and checks their structural invariants:
//   * the permutation is a bijection of 0 .. n-1;
//   * each depth's offsets start at 0, end at n and do not decrease, and every
//     leaf holds at most leaf_size points;
//   * each depth's pair lists are sorted by (s, t), symmetric, in range, and
//     every diagonal pair (s, s) of the leaf depth is close;
//   * invalid arguments (a bad dimension, n, eta, a NaN coordinate, a leaf
//     with fewer points than the rank) are refused with INVALID_ARG.
// Exit status 0 when every check holds.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <set>
#include <utility>
#include <vector>

#include "plan.h"

namespace {

int failures = 0;

void check(bool ok, const char* what, int64_t n, int dim) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s (n=%lld dim=%d)\n", what, static_cast<long long>(n), dim);
    ++failures;
  }
}

// Points from a 64-bit linear congruential generator (Knuth's MMIX
// constants), mapped to [0, 1).
std::vector<double> points(int64_t n, int dim, uint64_t seed) {
  std::vector<double> p(size_t(n) * dim);
  uint64_t s = seed;
  for (double& v : p) {
    s = s * 6364136223846793005ULL + 1442695040888963407ULL;
    v = double(s >> 11) * (1.0 / 9007199254740992.0);
  }
  return p;
}

void check_plan(const std::vector<double>& p, int64_t n, int dim, int leaf, double eta, int m) {
  h2mg_build_opts o{};
  o.leaf_size = leaf;
  o.eta = eta;
  o.cheb_m = m;
  h2mg::Plan P;
  const h2mg_status st = h2mg::build_plan(p.data(), n, dim, &o, &P);
  if (st != H2MG_OK) {
    std::fprintf(stderr, "build_plan refused n=%lld dim=%d leaf=%d: %d\n", static_cast<long long>(n), dim,
                 leaf, int(st));
    ++failures;
    return;
  }
  std::vector<int64_t> q = P.perm;
  std::sort(q.begin(), q.end());
  bool bij = int64_t(q.size()) == n;
  for (int64_t i = 0; bij && i < n; ++i) bij = q[size_t(i)] == i;
  check(bij, "permutation is a bijection", n, dim);
  check(int(P.offsets.size()) == P.L + 1, "one offset list per depth", n, dim);
  for (int d = 0; d <= P.L && d < int(P.offsets.size()); ++d) {
    const std::vector<int64_t>& off = P.offsets[size_t(d)];
    check(off.size() == (size_t(1) << d) + 1, "2^d + 1 offsets", n, dim);
    check(off.front() == 0 && off.back() == n, "offsets span 0 .. n", n, dim);
    for (size_t j = 1; j < off.size(); ++j) {
      check(off[j] >= off[j - 1], "offsets do not decrease", n, dim);
      if (d == P.L) check(off[j] - off[j - 1] <= leaf, "leaf size bound", n, dim);
    }
  }
  for (int d = 0; d <= P.L && d < int(P.near.size()); ++d) {
    const int64_t nc = int64_t(1) << d;
    for (int kind = 0; kind < 2; ++kind) {
      const std::vector<int32_t>& v = kind == 0 ? P.near[size_t(d)] : P.far[size_t(d)];
      check(v.size() % 2 == 0, "pairs come in (s, t)", n, dim);
      std::set<std::pair<int32_t, int32_t>> set;
      for (size_t i = 0; i + 1 < v.size(); i += 2) {
        check(v[i] >= 0 && v[i] < nc && v[i + 1] >= 0 && v[i + 1] < nc, "pair in range", n, dim);
        if (i >= 2) {
          const bool sorted = v[i - 2] < v[i] || (v[i - 2] == v[i] && v[i - 1] < v[i + 1]);
          check(sorted, "pairs sorted by (s, t)", n, dim);
        }
        set.insert({v[i], v[i + 1]});
      }
      for (const auto& pr : set) check(set.count({pr.second, pr.first}) == 1, "pair list symmetric", n, dim);
      if (kind == 0 && d == P.L)
        for (int32_t s = 0; s < nc; ++s)
          if (P.offsets[size_t(d)][size_t(s) + 1] > P.offsets[size_t(d)][size_t(s)])
            check(set.count({s, s}) == 1, "diagonal leaf pair is close", n, dim);
    }
  }
}

}  // namespace

int main() {
  // ordinary shapes: 1-3 dimensions, ragged leaves, several ranks
  const struct { int64_t n; int dim; int leaf; double eta; int m; } shapes[] = {
      {1, 1, 1, 0.7, 1},  {7, 1, 2, 0.7, 1},    {1000, 1, 16, 0.7, 4}, {4096, 2, 64, 0.7, 4},
      {1500, 2, 40, 0.5, 3}, {3000, 3, 64, 0.7, 3}, {9000, 3, 128, 1.0, 4}, {513, 3, 8, 0.7, 1},
  };
  uint64_t seed = 1;
  for (const auto& s : shapes) check_plan(points(s.n, s.dim, seed++), s.n, s.dim, s.leaf, s.eta, s.m);
  // degenerate point sets: all points equal, points on a line in 3D, two clusters of duplicates
  {
    const int64_t n = 300;
    std::vector<double> same(size_t(n) * 3, 0.25);
    check_plan(same, n, 3, 16, 0.7, 1);
    std::vector<double> line(size_t(n) * 3);
    for (int64_t i = 0; i < n; ++i) {
      line[size_t(i) * 3] = double(i) / double(n);
      line[size_t(i) * 3 + 1] = 0.5;
      line[size_t(i) * 3 + 2] = 0.5;
    }
    check_plan(line, n, 3, 16, 0.7, 2);
    std::vector<double> two(size_t(n) * 2);
    for (int64_t i = 0; i < n; ++i) {
      two[size_t(i) * 2] = i < n / 2 ? 0.0 : 1.0;
      two[size_t(i) * 2 + 1] = i < n / 2 ? 0.0 : 1.0;
    }
    check_plan(two, n, 2, 16, 0.7, 2);
  }
  // refused arguments
  {
    const std::vector<double> p = points(100, 2, 99);
    h2mg_build_opts o{};
    o.leaf_size = 16;
    o.eta = 0.7;
    o.cheb_m = 2;
    h2mg::Plan P;
    check(h2mg::build_plan(p.data(), 100, 4, &o, &P) == H2MG_ERR_INVALID_ARG, "dim 4 refused", 100, 4);
    check(h2mg::build_plan(p.data(), 0, 2, &o, &P) == H2MG_ERR_INVALID_ARG, "n 0 refused", 0, 2);
    o.eta = -1.0;
    check(h2mg::build_plan(p.data(), 100, 2, &o, &P) == H2MG_ERR_INVALID_ARG, "eta < 0 refused", 100, 2);
    o.eta = 0.7;
    std::vector<double> bad = p;
    bad[7] = std::nan("");
    check(h2mg::build_plan(bad.data(), 100, 2, &o, &P) == H2MG_ERR_INVALID_ARG, "NaN refused", 100, 2);
    // ragged leaves of 1 or 2 points cannot carry rank 2
    const std::vector<double> q = points(7, 1, 98);
    o.leaf_size = 2;
    o.cheb_m = 2;
    check(h2mg::build_plan(q.data(), 7, 1, &o, &P) == H2MG_ERR_INVALID_ARG, "leaf below the rank refused", 7, 1);
  }
  if (failures) std::fprintf(stderr, "%d check(s) failed\n", failures);
  else std::printf("plan driver: all checks passed\n");
  return failures ? 1 : 0;
}
