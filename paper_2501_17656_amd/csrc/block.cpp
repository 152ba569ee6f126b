// Products and H2-MG cycles on blocks of up to 16 right-hand sides: the
// matvec of Section 3.1 and the cycle of Algorithm 1 (Section 3.3) applied to
// every column at once, so that each stored tile is streamed once per pass
// for all 16 columns (kernels_block.hip), and independent problems (one
// handle each) solved together on several streams.  Columns never mix: every
// CG scalar of the smoother Iter and every stopping test is per column.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <new>
#include <stdexcept>
#include <vector>

#include "graph.h"
#include "h2_build.h"

namespace h2mg {

namespace {

constexpr int NR = MULTI_NR;
constexpr int RUN = 8;                 // tiles per tile-product task (without tuning)
constexpr int RUNS[] = {32, 16, 8, 4, 2};   // candidates of the tuner, by growing partial-sum memory

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

inline size_t vbytes(int p) { return p == P64 ? 8 : 4; }
inline int vprec(int p) { return p == P64 ? P64 : P32; }

void* alloc_owned(H2& h, size_t bytes) {
  void* d = h.arena.alloc(std::max<size_t>(bytes, 8));
  h.blk16.owned.push_back(d);
  return d;
}

template <typename T>
T* upload_owned(H2& h, const std::vector<T>& v) {
  T* d = static_cast<T*>(alloc_owned(h, v.size() * sizeof(T)));
  if (!v.empty())
    hip_check(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, h.stream), "upload");
  return d;
}

// Task set over the tiles `ids` (rows[b], cols[b]: block row and column of
// tile b; rows and columns index 0 .. nrows_total - 1).  Row-pass tasks cover
// every tile, column-pass tasks the off-diagonal ones; tiles keep their id
// order within a row or column, and a row's (column's) tasks are
// consecutive.
// Read-once form for 64 x 64 tiles (rank 64 and the near-field tiles): a
// tile's transposed product (rr x 16 words, a quarter of the tile at rank 64)
// is written once and reduced once, which moves less than reading the tile a
// second time.  For 32 x 32 and smaller tiles the two passes are faster
// (measured at rank 27, where the transposed product is 42% of the padded
// tile: 13 batched problems solved in 11.3 s with these tiles in two passes,
// 12.3 s with them read once).
bool use_dual(int T, int rr) { return T == 8 && rr * NR * 2 <= (8 * T) * (8 * T); }

TileSet make_set(H2& h, const std::vector<int>& ids, const std::vector<int>& rows, const std::vector<int>& cols,
                 int nrows_total, int row0, int nrows, const int* brow, const int* bcol, int run,
                 bool dual) {
  TileSet ts;
  ts.run = run;
  ts.dual = dual;
  ts.brow = brow;
  ts.bcol = bcol;
  ts.row0 = row0;
  ts.nrows = nrows;
  ts.ntiles = int64_t(ids.size());
  auto build = [&](bool by_col, int runlen, std::vector<int>& order, std::vector<int>& tasks,
                   std::vector<int>& ptr) {
    std::vector<std::pair<int, int>> kb;
    for (int b : ids) {
      if (by_col && rows[b] == cols[b]) continue;
      kb.emplace_back(by_col ? cols[b] : rows[b], b);
    }
    std::stable_sort(kb.begin(), kb.end(), [](const auto& u, const auto& v) { return u.first < v.first; });
    order.resize(kb.size());
    for (size_t i = 0; i < kb.size(); ++i) order[i] = kb[i].second;
    ptr.assign(size_t(nrows_total) + 1, 0);
    for (size_t i = 0; i < kb.size();) {
      size_t e = i;
      while (e < kb.size() && kb[e].first == kb[i].first) ++e;
      for (size_t c = i; c < e; c += size_t(runlen)) {
        tasks.push_back(kb[i].first);
        tasks.push_back(int(c));
        tasks.push_back(int(std::min(e, c + size_t(runlen))));
        ptr[size_t(kb[i].first) + 1]++;
      }
      i = e;
    }
    for (int r = 0; r < nrows_total; ++r) ptr[r + 1] += ptr[r];
    return int64_t(kb.size());
  };
  std::vector<int> ro, rt, rp, co, ct, cp;
  build(false, run, ro, rt, rp);
  // read-once: one column slot per off-diagonal tile (runs of 1), no column tasks
  ts.nctiles = build(true, dual ? 1 : run, co, ct, cp);
  ts.nrt = int(rt.size() / 3);
  ts.nct = dual ? 0 : int(ct.size() / 3);
  ts.rorder = upload_owned(h, ro);
  ts.rtask = upload_owned(h, rt);
  ts.rtp = upload_owned(h, rp);
  ts.corder = upload_owned(h, co);
  ts.ctask = upload_owned(h, ct);
  ts.ctp = upload_owned(h, cp);
  if (dual) {
    std::vector<int> pos(size_t(*std::max_element(ids.begin(), ids.end())) + 1, -1);
    for (size_t i = 0; i < co.size(); ++i) pos[size_t(co[i])] = int(i);
    std::vector<int> slot(ro.size());
    for (size_t i = 0; i < ro.size(); ++i) slot[i] = pos[size_t(ro[i])];
    ts.rslot = upload_owned(h, slot);
  }
  return ts;
}

void ensure_partial(H2& h, int64_t elems) {
  BlockWork& w = h.blk16;
  if (elems <= w.partial_elems) return;
  if (w.partial) {
    hip_check(hipStreamSynchronize(h.stream), "sync");
    h.arena.release(w.partial);
    w.owned.erase(std::find(w.owned.begin(), w.owned.end(), w.partial));
  }
  w.partial = alloc_owned(h, size_t(elems) * sizeof(double));
  w.partial_elems = elems;
}

void free_set(H2& h, TileSet& ts) {
  BlockWork& w = h.blk16;
  for (void* d : {static_cast<void*>(ts.rorder), static_cast<void*>(ts.rtask), static_cast<void*>(ts.rtp),
                  static_cast<void*>(ts.corder), static_cast<void*>(ts.ctask), static_cast<void*>(ts.ctp),
                  static_cast<void*>(ts.rslot)}) {
    auto it = std::find(w.owned.begin(), w.owned.end(), d);
    if (it != w.owned.end()) {
      w.owned.erase(it);
      h.arena.release(d);
    }
  }
  ts = TileSet();
}

// The tile product and reduce of one set, as run inside a product.
void run_set(H2& h, int p, const TileSet& ts, bool near, const void* x, void* out) {
  BlockWork& w = h.blk16;
  const int rr = near ? 64 : h.r;
  if (!near) launch_tgemm(h, p, h.T, ts, h.prec[p].blk, rr, x, w.partial);
  else if (p == P64 && h.snear.ready) launch_tgemm(h, P64, 8, ts, h.snear.tiles, 64, x, w.partial);
  else launch_tgemm_eval(h, p == P64 ? P64 : P32, ts, x, w.partial);
  launch_reduce16(h, p, ts, rr, w.partial, out);
}

// Task set with the run length (tiles per task) that makes this set's tile
// product plus reduce fastest on this device, measured with HIP events over
// two launches per candidate (after one untimed); with tuning off, RUN.
TileSet tuned_set(H2& h, int p, bool near, const void* x, void* out, const std::vector<int>& ids,
                  const std::vector<int>& rows, const std::vector<int>& cols, int nrows_total, int row0,
                  int nrows, const int* brow, const int* bcol) {
  const int rr = near ? 64 : h.r;
  const bool dual = use_dual(near ? 8 : h.T, rr);
  if (!h.autotune || ids.empty())
    return make_set(h, ids, rows, cols, nrows_total, row0, nrows, brow, bcol, RUN, dual);
  hipEvent_t e0, e1;
  hip_check(hipEventCreate(&e0), "event");
  hip_check(hipEventCreate(&e1), "event");
  TileSet best;
  float best_ms = 0.0f;
  try {
    for (int run : RUNS) {
      TileSet ts = make_set(h, ids, rows, cols, nrows_total, row0, nrows, brow, bcol, run, dual);
      const int64_t need = ts.nslots() * rr * NR;
      size_t free_b = 0, total_b = 0;
      hip_check(hipMemGetInfo(&free_b, &total_b), "memory info");
      if (best.rtask && need > h.blk16.partial_elems && size_t(need) * sizeof(double) > free_b / 4) {
        free_set(h, ts);               // its partial sums would take too much of the free memory
        continue;
      }
      ensure_partial(h, need);
      run_set(h, p, ts, near, x, out);
      hip_check(hipEventRecord(e0, h.stream), "event");
      for (int rep = 0; rep < 2; ++rep) run_set(h, p, ts, near, x, out);
      hip_check(hipEventRecord(e1, h.stream), "event");
      hip_check(hipEventSynchronize(e1), "event sync");
      float ms = 0.0f;
      hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
      ts.tuned_ms = 0.5 * ms;
      if (best.rtask == nullptr || ms < best_ms) {
        if (best.rtask) free_set(h, best);
        best = ts;
        best_ms = ms;
      } else {
        free_set(h, ts);
      }
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

// Task sets and buffers: couplings (at first use), near-field chunk plan and
// tasks, restricted operators of every depth (once the hierarchy is built).
// p: the precision the sets are tuned for.
void ensure_block(H2& h, int p) {
  BlockWork& w = h.blk16;
  const int r = h.r;
  if (!w.ready) {
    if (h.T < 2) throw std::invalid_argument("blocks of vectors need a rank of 9 to 64");
    if (h.d_top >= 0) {
      std::vector<int> ids;
      for (int d = h.d_top; d <= h.L; ++d)
        for (int b = h.s_first[d]; b < h.s_first[d] + h.s_count[d]; ++b) ids.push_back(b);
      const int row0 = (1 << h.d_top) - 1;
      w.xall = alloc_owned(h, size_t(h.ngid) * r * NR * sizeof(double));
      w.yall = alloc_owned(h, size_t(h.ngid) * r * NR * sizeof(double));
      hip_check(hipMemsetAsync(w.xall, 0, size_t(h.ngid) * r * NR * sizeof(double), h.stream), "memset");
      w.fine = tuned_set(h, p, false, w.xall, w.yall, ids, h.blk_row_h, h.blk_col_h, h.ngid, row0,
                         h.ngid - row0, h.blk_row, h.blk_col);
      ensure_partial(h, w.fine.nslots() * r * NR);
    }
    w.bx = static_cast<double*>(alloc_owned(h, size_t(h.n) * NR * sizeof(double)));
    w.by = static_cast<double*>(alloc_owned(h, size_t(h.n) * NR * sizeof(double)));
    hip_check(hipMemsetAsync(w.bx, 0, size_t(h.n) * NR * sizeof(double), h.stream), "memset");
    w.ready = true;
  }
  const StoredNear& sn = h.snear;
  if (!w.near_ready) {
    plan_near(h);
    std::vector<int> ids(sn.brow_h.size());
    for (size_t b = 0; b < ids.size(); ++b) ids[b] = int(b);
    const size_t nv = size_t(sn.nchunk) * 64 * NR;
    if (!sn.identity) {
      w.xc64 = static_cast<double*>(alloc_owned(h, nv * sizeof(double)));
      w.xc32 = static_cast<float*>(alloc_owned(h, nv * sizeof(float)));
      hip_check(hipMemsetAsync(w.xc64, 0, nv * sizeof(double), h.stream), "memset");
      hip_check(hipMemsetAsync(w.xc32, 0, nv * sizeof(float), h.stream), "memset");
    }
    w.yc = alloc_owned(h, nv * sizeof(double));
    const void* xn = sn.identity ? static_cast<const void*>(w.bx)
                                 : p == P64 ? static_cast<const void*>(w.xc64) : static_cast<const void*>(w.xc32);
    w.near = tuned_set(h, p, true, xn, w.yc, ids, sn.brow_h, sn.bcol_h, sn.nchunk, 0, sn.nchunk, sn.blk_row,
                       sn.blk_col);
    ensure_partial(h, w.near.nslots() * 64 * NR);
    w.near_ready = true;
  }
  if (h.mg_built && !w.coarse_ready && h.d_top >= 0) {
    w.coarse.assign(size_t(h.L) + 1, TileSet());
    const int row0 = (1 << h.d_top) - 1;
    for (int d = h.d_top; d <= h.L; ++d) {
      std::vector<int> ids;
      for (int q = h.d_top; q <= d; ++q)
        for (int b = h.s_first[q]; b < h.s_first[q] + h.s_count[q]; ++b) ids.push_back(b);
      for (int b = h.p_first[d]; b < h.p_first[d] + h.p_count[d]; ++b) ids.push_back(b);
      w.coarse[d] = tuned_set(h, p, false, w.xall, w.yall, ids, h.blk_row_h, h.blk_col_h, h.ngid, row0,
                              (2 << d) - 1 - row0, h.blk_row, h.blk_col);
      ensure_partial(h, w.coarse[d].nslots() * r * NR);
    }
    w.coarse_ready = true;
  }
  // partial sums for the largest chosen set only (tuning may have grown them)
  int64_t need = 0;
  auto fit = [&](const TileSet& ts, int rr) { need = std::max(need, ts.nslots() * rr * NR); };
  fit(w.fine, r);
  fit(w.near, 64);
  for (const TileSet& ts : w.coarse) fit(ts, r);
  if (need > 0 && need < w.partial_elems) {
    hip_check(hipStreamSynchronize(h.stream), "sync");
    h.arena.release(w.partial);
    w.owned.erase(std::find(w.owned.begin(), w.owned.end(), w.partial));
    w.partial = nullptr;
    w.partial_elems = 0;
    ensure_partial(h, need);
  }
  hip_check(hipStreamSynchronize(h.stream), "block setup");
}

// Coefficients of depth d inside a gid-indexed block buffer.
inline void* at_depth(void* base, int p, int d, int r) {
  return static_cast<char*>(base) + size_t((1 << d) - 1) * r * NR * vbytes(p);
}

// ------------------------------------------------------------ products
// Fine level, tree order: out = alpha * A_H2 X + beta * add.
void apply_fine16(H2& h, int p, const void* X, void* out, double alpha, const void* add, double beta) {
  BlockWork& w = h.blk16;
  const int r = h.r;
  const void* yhat = nullptr;
  if (h.d_top >= 0) {
    launch_leaf_up16(h, p, X, at_depth(w.xall, p, h.L, r));
    for (int d = h.L - 1; d >= h.d_top; --d)
      launch_transfer_up16(h, p, d, at_depth(w.xall, p, d + 1, r), at_depth(w.xall, p, d, r));
    launch_tgemm(h, p, h.T, w.fine, h.prec[p].blk, r, w.xall, w.partial);
    launch_reduce16(h, p, w.fine, r, w.partial, w.yall);
    for (int d = h.d_top + 1; d <= h.L; ++d)
      launch_transfer_down16(h, p, d - 1, at_depth(w.yall, p, d - 1, r), at_depth(w.yall, p, d, r),
                             at_depth(w.yall, p, d, r));
    yhat = at_depth(w.yall, p, h.L, r);
  }
  const StoredNear& sn = h.snear;
  const void* xc = X;
  if (!sn.identity) {
    void* buf = p == P64 ? static_cast<void*>(w.xc64) : static_cast<void*>(w.xc32);
    launch_near_pad16(h, p, X, buf);
    xc = buf;
  }
  if (p == P64 && sn.ready) {
    int ev;
    h.time_begin(ev);
    launch_tgemm(h, P64, 8, w.near, sn.tiles, 64, xc, w.partial);
    h.time_end(KS_NEAR16, ev, double(w.near.ntiles) * 4096.0 * sizeof(double));   // each stored tile once
  } else if (near_stored_for(h, p)) {
    launch_tgemm(h, P32, 8, w.near, sn.tiles32, 64, xc, w.partial);
  } else {
    launch_tgemm_eval(h, vprec(p), w.near, xc, w.partial);
  }
  launch_reduce16(h, p, w.near, 64, w.partial, w.yc);
  launch_leaf_down16(h, p, yhat, w.yc, out, alpha, add, beta);
}

// Level k >= 2 (depth d = L - k + 2), coefficient order: Y = A_k X.
void apply_coarse16(H2& h, int p, int k, const void* X, void* Y) {
  BlockWork& w = h.blk16;
  const int r = h.r, d = h.level_depth(k);
  launch_copy(h, vprec(p), X, at_depth(w.xall, p, d, r), int64_t(1 << d) * r * NR);
  for (int q = d - 1; q >= h.d_top; --q)
    launch_transfer_up16(h, p, q, at_depth(w.xall, p, q + 1, r), at_depth(w.xall, p, q, r));
  launch_tgemm(h, p, h.T, w.coarse[d], h.prec[p].blk, r, w.xall, w.partial);
  launch_reduce16(h, p, w.coarse[d], r, w.partial, w.yall);
  for (int q = h.d_top + 1; q <= d; ++q)
    launch_transfer_down16(h, p, q - 1, at_depth(w.yall, p, q - 1, r), q == d ? Y : at_depth(w.yall, p, q, r),
                           at_depth(w.yall, p, q, r));
  if (d == h.d_top) launch_copy(h, vprec(p), at_depth(w.yall, p, d, r), Y, int64_t(1 << d) * r * NR);
}

void apply16(H2& h, int p, int k, const void* X, void* Y) {
  if (k == 1) apply_fine16(h, p, X, Y, 1.0, nullptr, 0.0);
  else apply_coarse16(h, p, k, X, Y);
}

// ------------------------------------------------------------ cycle
struct Work16 {
  int p = P64;
  int smoother = 0;
  std::vector<void*> r, et, ec;
  void *s = nullptr, *pv = nullptr, *q = nullptr, *tmp = nullptr, *z = nullptr;
  double* part = nullptr;              // 4 slots of 256 x NR partial sums
  double* coarse64 = nullptr;          // Nl x NR, FP64 coarse solve of a low-precision cycle
  std::vector<void*> owned;
  double* gpart(int i) const { return part + size_t(i) * 256 * NR; }
  double* dpart() const { return part + size_t(2) * 256 * NR; }
  double* scratch() const { return part + size_t(3) * 256 * NR; }
};

void make_work16(H2& h, Work16& w, int p, bool second) {
  auto take = [&](size_t bytes) {
    void* d = h.arena.alloc(std::max<size_t>(bytes, 8));
    w.owned.push_back(d);
    return d;
  };
  const size_t vb = vbytes(p) * NR;
  w.p = p;
  w.r.assign(size_t(h.levels) + 1, nullptr);
  w.et.assign(size_t(h.levels) + 1, nullptr);
  w.ec.assign(size_t(h.levels) + 1, nullptr);
  for (int k = 1; k <= h.levels; ++k) {
    w.r[k] = take(size_t(h.level_size(k)) * vb);
    w.et[k] = take(size_t(h.level_size(k)) * vb);
    if (second && k >= 2 && k < h.levels) w.ec[k] = take(size_t(h.level_size(k)) * vb);
  }
  w.s = take(size_t(h.n) * vb);
  w.pv = take(size_t(h.n) * vb);
  w.q = take(size_t(h.n) * vb);
  w.tmp = take(size_t(h.n) * NR * sizeof(double));
  w.z = take(size_t(h.n) * vb);
  w.part = static_cast<double*>(take(size_t(4) * 256 * NR * sizeof(double)));
  if (p != P64) w.coarse64 = static_cast<double*>(take(size_t(h.Nl) * NR * sizeof(double)));
}

void release_work16(H2& h, Work16& w) {
  for (void* d : w.owned) h.arena.release(d);
  w.owned.clear();
}

// e = Iter(A_k, rhs, e0) on every column: nsteps of CG, or of block-Jacobi
// PCG when w.smoother == 1; e holds e0 on entry unless e0_zero.
void cg16(H2& h, Work16& w, int k, const void* rhs, void* e, bool e0_zero, int nsteps) {
  const int p = w.p, vp = vprec(p);
  const int64_t N = h.level_size(k), nf = N * NR;
  const bool pre = w.smoother == 1;
  if (e0_zero) launch_zero(h, vp, e, nf);
  if (nsteps <= 0) return;
  if (e0_zero) {
    launch_copy(h, vp, rhs, w.s, nf);
  } else {
    apply16(h, p, k, e, w.q);
    launch_copy(h, vp, rhs, w.s, nf);
    launch_axpby(h, vp, nf, -1.0, w.q, 1.0, w.s);
  }
  int cur = 0;
  if (pre) {
    launch_bj_apply16(h, p, k, w.s, w.z);
    launch_copy(h, vp, w.z, w.pv, nf);
    launch_dot16(h, vp, N, w.s, w.z, w.gpart(cur));
  } else {
    launch_copy(h, vp, w.s, w.pv, nf);
    launch_dot16(h, vp, N, w.s, w.s, w.gpart(cur));
  }
  for (int it = 0; it < nsteps; ++it) {
    apply16(h, p, k, w.pv, w.q);
    launch_dot16(h, vp, N, w.pv, w.q, w.dpart());
    if (pre) {
      launch_cg_update16(h, vp, N, e, w.pv, w.s, w.q, w.gpart(cur), w.dpart(), w.scratch());
      launch_bj_apply16(h, p, k, w.s, w.z);
      launch_dot16(h, vp, N, w.s, w.z, w.gpart(1 - cur));
      if (it + 1 < nsteps) launch_cg_pupdate16(h, vp, N, w.pv, w.z, w.gpart(cur), w.gpart(1 - cur));
    } else {
      launch_cg_update16(h, vp, N, e, w.pv, w.s, w.q, w.gpart(cur), w.dpart(), w.gpart(1 - cur));
      if (it + 1 < nsteps) launch_cg_pupdate16(h, vp, N, w.pv, w.s, w.gpart(cur), w.gpart(1 - cur));
    }
    cur = 1 - cur;
  }
}

// Direct solve on the coarsest level with the FP64 Cholesky factor.
void coarse_solve16(H2& h, Work16& w, const void* r, void* e) {
  const int64_t nf = h.Nl * NR;
  if (w.p == P64) {
    launch_copy(h, P64, r, e, nf);
    launch_chol_solve16(h, h.chol, h.Nl, static_cast<double*>(e));
  } else {
    launch_cast(h, P64, w.coarse64, P32, r, nf);
    launch_chol_solve16(h, h.chol, h.Nl, w.coarse64);
    launch_cast(h, P32, e, P64, w.coarse64, nf);
  }
}

enum Cycle { CYCLE_V = 0, CYCLE_W = 1, CYCLE_F = 2 };

// One cycle on level k for A_k E_k = R_k (w.r[k]); the result in w.et[k].
void mg16(H2& h, Work16& w, int k, int kind, int n_f, int n_c) {
  const int p = w.p, vp = vprec(p), l = h.levels;
  if (k == l) {
    coarse_solve16(h, w, w.r[l], w.et[l]);
    return;
  }
  const int nk = k == 1 ? n_f : n_c;
  const int64_t nf = h.level_size(k) * NR;
  cg16(h, w, k, w.r[k], w.et[k], true, nk);
  // R_{k+1} = U_k^T (R_k - A_k E~_k)
  apply16(h, p, k, w.et[k], w.tmp);
  launch_axpby(h, vp, nf, 1.0, w.r[k], -1.0, w.tmp);
  if (k == 1) launch_leaf_up16(h, p, w.tmp, w.r[k + 1]);
  else launch_transfer_up16(h, p, h.level_depth(k) - 1, w.tmp, w.r[k + 1]);
  mg16(h, w, k + 1, kind, n_f, n_c);
  if (kind != CYCLE_V && k + 1 < l) {
    const int64_t nf1 = h.level_size(k + 1) * NR;
    launch_copy(h, vp, w.et[k + 1], w.ec[k + 1], nf1);
    apply16(h, p, k + 1, w.et[k + 1], w.tmp);
    launch_axpby(h, vp, nf1, -1.0, w.tmp, 1.0, w.r[k + 1]);
    mg16(h, w, k + 1, kind == CYCLE_F ? CYCLE_V : CYCLE_W, n_f, n_c);
    launch_axpby(h, vp, nf1, 1.0, w.ec[k + 1], 1.0, w.et[k + 1]);
  }
  // E~_k += U_k E_{k+1}
  if (k == 1) launch_leaf_down16(h, p, w.et[k + 1], nullptr, w.et[k], 1.0, w.et[k], 1.0);
  else launch_transfer_down16(h, p, h.level_depth(k) - 1, w.et[k + 1], w.et[k], w.et[k]);
  cg16(h, w, k, w.r[k], w.et[k], false, nk);
}

// ------------------------------------------------------------ several problems per launch
// The same cycle for a group of independent problems advancing in step: every
// tile product of a step (couplings, projected blocks, near-field tiles) is
// one launch over the task sets of all members (launch_tgemm_group), the
// other steps are each member's own launches on the group's stream.  Each
// member's arithmetic, and its order, is exactly that of its own solve, so
// its iterates are bit for bit those of a solve of its own.  A member takes
// part in a level's step only when that level exists for it (problems have
// different depths); on its coarsest level it does the direct solve.
struct GM {
  H2* h;
  Work16* w;
};

// Lanes for the members' own launches: a section of per-member launches is
// bracketed by a fork (every lane stream waits for the group's stream, and
// member i launches on lane i mod L) and a join (the group's stream waits for
// every lane, and the members launch on the group's stream again).  Sections
// of different members then overlap, while each group launch stays ordered
// after every member's preceding work and before its following work.  Under
// stream capture the event record / wait pairs become graph edges.
struct GroupLanes {
  std::vector<hipStream_t> lane;
  std::vector<hipEvent_t> join_ev;
  hipEvent_t fork_ev = nullptr;
  hipStream_t main = nullptr;
  bool open = false;

  void create(int n) {
    for (int l = 0; l < n; ++l) {
      hipStream_t s = nullptr;
      hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "lane stream");
      lane.push_back(s);
      hipEvent_t e = nullptr;
      hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "lane event");
      join_ev.push_back(e);
    }
    hip_check(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming), "lane event");
  }
  void destroy() {
    for (hipStream_t s : lane) (void)hipStreamDestroy(s);
    for (hipEvent_t e : join_ev) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    lane.clear();
    join_ev.clear();
    fork_ev = nullptr;
  }
  void fork(const std::vector<H2*>& hs) {
    main = hs[0]->stream;
    hip_check(hipEventRecord(fork_ev, main), "fork");
    for (hipStream_t s : lane) hip_check(hipStreamWaitEvent(s, fork_ev, 0), "fork");
    for (size_t i = 0; i < hs.size(); ++i) hs[i]->stream = lane[i % lane.size()];
    open = true;
  }
  void join(const std::vector<H2*>& hs) {
    for (size_t l = 0; l < lane.size(); ++l) {
      hip_check(hipEventRecord(join_ev[l], lane[l]), "join");
      hip_check(hipStreamWaitEvent(main, join_ev[l], 0), "join");
    }
    for (H2* h : hs) h->stream = main;
    open = false;
  }
};

// The lanes of the group solve running on this thread (none outside it).
thread_local GroupLanes* t_lanes = nullptr;
constexpr int GROUP_LANES = 4;       // lane streams of a group solve

// A section of per-member launches: forked on construction, joined by end().
class MemberSection {
 public:
  template <typename V, typename F>
  MemberSection(const V& members, F h_of) {
    for (const auto& m : members) hs_.push_back(h_of(m));
    on_ = t_lanes && hs_.size() > 1;
    if (on_) t_lanes->fork(hs_);
  }
  explicit MemberSection(const std::vector<GM>& G) : MemberSection(G, [](const GM& m) { return m.h; }) {}
  void end() {
    if (on_) t_lanes->join(hs_);
    on_ = false;
  }

 private:
  std::vector<H2*> hs_;
  bool on_ = false;
};

// Y_m = A_k X_m for every member (each at its own level k).
void apply16_group(const std::vector<GM>& G, int p, int k, const std::vector<const void*>& X,
                   const std::vector<void*>& Y, double alpha = 1.0, const std::vector<const void*>* add = nullptr,
                   double beta = 0.0) {
  if (G.empty()) return;
  const hipStream_t st = G[0].h->stream;
  const int vp = vprec(p);
  std::vector<GroupTiles> tiles;
  if (k == 1) {
    std::vector<const void*> yhat(G.size(), nullptr);
    MemberSection up(G);
    for (size_t i = 0; i < G.size(); ++i) {
      H2& h = *G[i].h;
      BlockWork& w = h.blk16;
      if (h.d_top < 0) continue;
      launch_leaf_up16(h, p, X[i], at_depth(w.xall, p, h.L, h.r));
      for (int d = h.L - 1; d >= h.d_top; --d)
        launch_transfer_up16(h, p, d, at_depth(w.xall, p, d + 1, h.r), at_depth(w.xall, p, d, h.r));
      tiles.push_back(GroupTiles{h.T, &w.fine, h.prec[p].blk, h.r, w.xall, w.partial});
    }
    up.end();
    launch_tgemm_group(st, p, tiles);
    std::vector<const void*> xc(G.size());
    MemberSection down(G);
    for (size_t i = 0; i < G.size(); ++i) {
      H2& h = *G[i].h;
      BlockWork& w = h.blk16;
      if (h.d_top >= 0) {
        launch_reduce16(h, p, w.fine, h.r, w.partial, w.yall);
        for (int d = h.d_top + 1; d <= h.L; ++d)
          launch_transfer_down16(h, p, d - 1, at_depth(w.yall, p, d - 1, h.r), at_depth(w.yall, p, d, h.r),
                                 at_depth(w.yall, p, d, h.r));
        yhat[i] = at_depth(w.yall, p, h.L, h.r);
      }
      xc[i] = X[i];
      if (!h.snear.identity) {
        void* buf = p == P64 ? static_cast<void*>(w.xc64) : static_cast<void*>(w.xc32);
        launch_near_pad16(h, p, X[i], buf);
        xc[i] = buf;
      }
    }
    down.end();
    tiles.clear();
    std::vector<GroupTiles> tiles32;
    std::vector<GroupEval> evals;
    for (size_t i = 0; i < G.size(); ++i) {
      H2& h = *G[i].h;
      BlockWork& w = h.blk16;
      if (p == P64 && h.snear.ready) tiles.push_back(GroupTiles{8, &w.near, h.snear.tiles, 64, xc[i], w.partial});
      else if (near_stored_for(h, p)) tiles32.push_back(GroupTiles{8, &w.near, h.snear.tiles32, 64, xc[i], w.partial});
      else evals.push_back(GroupEval{&h, &w.near, xc[i], w.partial});
    }
    launch_tgemm_group(st, P64, tiles);
    launch_tgemm_group(st, P32, tiles32);
    launch_tgemm_eval_group(st, vp, evals);
    MemberSection out(G);
    for (size_t i = 0; i < G.size(); ++i) {
      H2& h = *G[i].h;
      BlockWork& w = h.blk16;
      launch_reduce16(h, p, w.near, 64, w.partial, w.yc);
      launch_leaf_down16(h, p, yhat[i], w.yc, Y[i], alpha, add ? (*add)[i] : nullptr, beta);
    }
    out.end();
    return;
  }
  MemberSection up(G);
  for (size_t i = 0; i < G.size(); ++i) {
    H2& h = *G[i].h;
    BlockWork& w = h.blk16;
    const int r = h.r, d = h.level_depth(k);
    launch_copy(h, vp, X[i], at_depth(w.xall, p, d, r), int64_t(1 << d) * r * NR);
    for (int q = d - 1; q >= h.d_top; --q)
      launch_transfer_up16(h, p, q, at_depth(w.xall, p, q + 1, r), at_depth(w.xall, p, q, r));
    tiles.push_back(GroupTiles{h.T, &w.coarse[d], h.prec[p].blk, r, w.xall, w.partial});
  }
  up.end();
  launch_tgemm_group(st, p, tiles);
  MemberSection down(G);
  for (size_t i = 0; i < G.size(); ++i) {
    H2& h = *G[i].h;
    BlockWork& w = h.blk16;
    const int r = h.r, d = h.level_depth(k);
    launch_reduce16(h, p, w.coarse[d], r, w.partial, w.yall);
    for (int q = h.d_top + 1; q <= d; ++q)
      launch_transfer_down16(h, p, q - 1, at_depth(w.yall, p, q - 1, r), q == d ? Y[i] : at_depth(w.yall, p, q, r),
                             at_depth(w.yall, p, q, r));
    if (d == h.d_top) launch_copy(h, vp, at_depth(w.yall, p, d, r), Y[i], int64_t(1 << d) * r * NR);
  }
  down.end();
}

// cg16 for every member: e = Iter(A_k, rhs, e0) on level k.
void cg16_group(const std::vector<GM>& G, int k, bool e0_zero, int nsteps) {
  if (G.empty()) return;
  const int p = G[0].w->p, vp = vprec(p);
  auto N = [&](const GM& m) { return m.h->level_size(k); };
  std::vector<const void*> X(G.size());
  std::vector<void*> Y(G.size());
  if (e0_zero) {
    MemberSection zero(G);
    for (const GM& m : G) launch_zero(*m.h, vp, m.w->et[k], N(m) * NR);
    zero.end();
  }
  if (nsteps <= 0) return;
  if (!e0_zero) {
    for (size_t i = 0; i < G.size(); ++i) {
      X[i] = G[i].w->et[k];
      Y[i] = G[i].w->q;
    }
    apply16_group(G, p, k, X, Y);
  }
  MemberSection init(G);
  for (const GM& m : G) {
    H2& h = *m.h;
    Work16& w = *m.w;
    const int64_t nf = N(m) * NR;
    launch_copy(h, vp, w.r[k], w.s, nf);
    if (!e0_zero) launch_axpby(h, vp, nf, -1.0, w.q, 1.0, w.s);
    if (w.smoother == 1) {
      launch_bj_apply16(h, p, k, w.s, w.z);
      launch_copy(h, vp, w.z, w.pv, nf);
      launch_dot16(h, vp, N(m), w.s, w.z, w.gpart(0));
    } else {
      launch_copy(h, vp, w.s, w.pv, nf);
      launch_dot16(h, vp, N(m), w.s, w.s, w.gpart(0));
    }
  }
  init.end();
  int cur = 0;
  for (int it = 0; it < nsteps; ++it) {
    for (size_t i = 0; i < G.size(); ++i) {
      X[i] = G[i].w->pv;
      Y[i] = G[i].w->q;
    }
    apply16_group(G, p, k, X, Y);
    MemberSection step(G);
    for (const GM& m : G) {
      H2& h = *m.h;
      Work16& w = *m.w;
      const int64_t n = N(m);
      void* e = w.et[k];
      launch_dot16(h, vp, n, w.pv, w.q, w.dpart());
      if (w.smoother == 1) {
        launch_cg_update16(h, vp, n, e, w.pv, w.s, w.q, w.gpart(cur), w.dpart(), w.scratch());
        launch_bj_apply16(h, p, k, w.s, w.z);
        launch_dot16(h, vp, n, w.s, w.z, w.gpart(1 - cur));
        if (it + 1 < nsteps) launch_cg_pupdate16(h, vp, n, w.pv, w.z, w.gpart(cur), w.gpart(1 - cur));
      } else {
        launch_cg_update16(h, vp, n, e, w.pv, w.s, w.q, w.gpart(cur), w.dpart(), w.gpart(1 - cur));
        if (it + 1 < nsteps) launch_cg_pupdate16(h, vp, n, w.pv, w.s, w.gpart(cur), w.gpart(1 - cur));
      }
    }
    step.end();
    cur = 1 - cur;
  }
}

// mg16 for every member, level k down.
void mg16_group(const std::vector<GM>& all, int k, int kind, int n_f, int n_c) {
  std::vector<GM> G, C;
  for (const GM& m : all) {
    if (k == m.h->levels) C.push_back(m);
    else if (k < m.h->levels) G.push_back(m);
  }
  if (!C.empty()) {
    MemberSection coarse(C);
    for (const GM& m : C) coarse_solve16(*m.h, *m.w, m.w->r[k], m.w->et[k]);
    coarse.end();
  }
  if (G.empty()) return;
  const int p = G[0].w->p, vp = vprec(p);
  const int nk = k == 1 ? n_f : n_c;
  cg16_group(G, k, true, nk);
  std::vector<const void*> X(G.size());
  std::vector<void*> Y(G.size());
  for (size_t i = 0; i < G.size(); ++i) {
    X[i] = G[i].w->et[k];
    Y[i] = G[i].w->tmp;
  }
  apply16_group(G, p, k, X, Y);
  MemberSection restrict_(G);
  for (const GM& m : G) {
    H2& h = *m.h;
    Work16& w = *m.w;
    launch_axpby(h, vp, h.level_size(k) * NR, 1.0, w.r[k], -1.0, w.tmp);
    if (k == 1) launch_leaf_up16(h, p, w.tmp, w.r[k + 1]);
    else launch_transfer_up16(h, p, h.level_depth(k) - 1, w.tmp, w.r[k + 1]);
  }
  restrict_.end();
  mg16_group(G, k + 1, kind, n_f, n_c);
  if (kind != CYCLE_V) {
    std::vector<GM> sub;
    for (const GM& m : G)
      if (k + 1 < m.h->levels) sub.push_back(m);
    if (!sub.empty()) {
      std::vector<const void*> X1(sub.size());
      std::vector<void*> Y1(sub.size());
      MemberSection save(sub);
      for (size_t i = 0; i < sub.size(); ++i) {
        H2& h = *sub[i].h;
        Work16& w = *sub[i].w;
        launch_copy(h, vp, w.et[k + 1], w.ec[k + 1], h.level_size(k + 1) * NR);
        X1[i] = w.et[k + 1];
        Y1[i] = w.tmp;
      }
      save.end();
      apply16_group(sub, p, k + 1, X1, Y1);
      MemberSection res(sub);
      for (const GM& m : sub)
        launch_axpby(*m.h, vp, m.h->level_size(k + 1) * NR, -1.0, m.w->tmp, 1.0, m.w->r[k + 1]);
      res.end();
      mg16_group(sub, k + 1, kind == CYCLE_F ? CYCLE_V : CYCLE_W, n_f, n_c);
      MemberSection add(sub);
      for (const GM& m : sub)
        launch_axpby(*m.h, vp, m.h->level_size(k + 1) * NR, 1.0, m.w->ec[k + 1], 1.0, m.w->et[k + 1]);
      add.end();
    }
  }
  MemberSection prolong(G);
  for (const GM& m : G) {
    H2& h = *m.h;
    Work16& w = *m.w;
    if (k == 1) launch_leaf_down16(h, p, w.et[k + 1], nullptr, w.et[k], 1.0, w.et[k], 1.0);
    else launch_transfer_down16(h, p, h.level_depth(k) - 1, w.et[k + 1], w.et[k], w.et[k]);
  }
  prolong.end();
  cg16_group(G, k, false, nk);
}

// ------------------------------------------------------------ solve driver
// One problem's solve as separate steps, so that several problems can be
// interleaved on several streams.
struct BlockSolve {
  H2* h = nullptr;
  SolveParams sp;
  int p = P64, nrhs = 0, np = 0;
  double* xuser = nullptr;
  int ldx = 0;
  Work16 w64, wlp;
  double* bt = nullptr;
  double* xt = nullptr;
  double* npart = nullptr;
  double* host = nullptr;              // pinned: np x NR partial sums, then 4 flag ints
  hipEvent_t ev = nullptr;
  std::vector<double> nb, rel;
  CycleGraph graph;
  int cycles = 0;
  bool converged = false, done = false;
  h2mg_status status = H2MG_OK;
  std::chrono::steady_clock::time_point t0;

  ~BlockSolve() { release(); }
  void release() {
    if (!h) return;
    graph.reset();
    release_work16(*h, w64);
    release_work16(*h, wlp);
    for (double* d : {bt, xt, npart})
      if (d) h->arena.release(d);
    bt = xt = npart = nullptr;
    if (host) (void)hipHostFree(host);
    host = nullptr;
    if (ev) (void)hipEventDestroy(ev);
    ev = nullptr;
    h = nullptr;
  }

  void read_async() {
    H2& H = *h;
    hip_check(hipMemcpyAsync(host, npart, size_t(np) * NR * sizeof(double), hipMemcpyDeviceToHost, H.stream),
              "norm readback");
    hip_check(hipMemcpyAsync(host + size_t(np) * NR, H.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, H.stream),
              "flag readback");
    hip_check(hipEventRecord(ev, H.stream), "event");
  }
  const int* flags() const { return reinterpret_cast<const int*>(host + size_t(np) * NR); }
  double column_sum(int k) const {
    double s = 0.0;
    for (int b = 0; b < np; ++b) s += host[size_t(b) * NR + k];
    return s;
  }

  h2mg_status begin(H2& H, int nrhs_, const double* b, int ldb, double* x, int ldx_, const SolveParams& sp_) {
    t0 = std::chrono::steady_clock::now();
    sp = sp_;
    nrhs = nrhs_;
    xuser = x;
    ldx = ldx_;
    p = sp.precision == 0 ? P64 : sp.precision == 1 ? P32 : P16;
    H.history.clear();
    h2mg_status st = setup_mg(H, p == P64 ? 0 : (1 << p));
    if (st != H2MG_OK) return st;
    if (sp.smoother == 1) {
      st = ensure_block_jacobi(H, p);
      if (st != H2MG_OK) return st;
    }
    ensure_block(H, p);
    h = &H;
    const bool second = sp.method == CYCLE_W || sp.method == CYCLE_F;
    make_work16(H, w64, P64, second && p == P64);
    w64.smoother = sp.smoother;
    if (p != P64) {
      make_work16(H, wlp, p, second);
      wlp.smoother = sp.smoother;
    }
    const int64_t n = H.n;
    np = parts16(n);
    bt = static_cast<double*>(H.arena.alloc(size_t(n) * NR * sizeof(double)));
    xt = static_cast<double*>(H.arena.alloc(size_t(n) * NR * sizeof(double)));
    npart = static_cast<double*>(H.arena.alloc(size_t(np) * NR * sizeof(double)));
    hip_check(hipHostMalloc(reinterpret_cast<void**>(&host), size_t(np) * NR * sizeof(double) + 4 * sizeof(int),
                            hipHostMallocDefault),
              "pinned alloc");
    hip_check(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event create");
    launch_gather16(H, nrhs, b, ldb, bt);
    if (sp.use_x0) launch_gather16(H, nrhs, x, ldx, xt);
    else launch_zero(H, P64, xt, n * NR);
    hip_check(hipMemsetAsync(H.flags, 0, 4 * sizeof(int), H.stream), "memset");
    launch_check_finite(H, P64, n * NR, bt);
    launch_dot16(H, P64, n, bt, bt, npart);
    read_async();
    hip_check(hipEventSynchronize(ev), "sync");
    if (flags()[1]) return fail(H2MG_ERR_INVALID_ARG, "B contains a non-finite value");
    nb.assign(NR, 0.0);
    rel.assign(NR, 0.0);
    bool any = false;
    for (int k = 0; k < nrhs; ++k) {
      nb[k] = std::sqrt(column_sum(k));
      any = any || nb[k] > 0.0;
    }
    if (!any) {
      H.history.push_back(0.0);
      converged = true;
      done = true;
    }
    return H2MG_OK;
  }

  // R = B - A_H2 X (FP64), its column norms and the flags, read back
  // asynchronously (complete once `ev` has fired).
  void enqueue_residual() {
    apply_fine16(*h, P64, xt, w64.r[1], -1.0, bt, 1.0);
    launch_dot16(*h, P64, h->n, w64.r[1], w64.r[1], npart);
    read_async();
  }

  void check() {
    double mx = 0.0;
    for (int k = 0; k < nrhs; ++k) {
      rel[k] = nb[k] > 0.0 ? std::sqrt(column_sum(k)) / nb[k] : 0.0;
      if (!(rel[k] <= mx)) mx = rel[k];
    }
    h->history.push_back(mx);
    if (flags()[0]) {
      status = fail(H2MG_ERR_NOT_SPD, "CG met p^T A p <= 0 (operator not SPD)");
      done = true;
    } else if (!std::isfinite(mx)) {
      status = fail(H2MG_ERR_NUMERIC, "non-finite residual after %d cycles", cycles);
      done = true;
    } else if (mx < sp.rtol) {
      converged = true;
      done = true;
    } else if (cycles >= sp.max_cycles) {
      status = fail(H2MG_ERR_NOT_CONVERGED, "no convergence in %d cycles (rel. residual %.3e)", sp.max_cycles, mx);
      done = true;
    }
  }

  void enqueue_cycle() {
    H2& H = *h;
    const int64_t nf = int64_t(H.n) * NR;
    auto body = [&]() {
      if (p == P64) {
        mg16(H, w64, 1, sp.method, sp.n_fine, sp.n_coarse);
        launch_axpby(H, P64, nf, 1.0, w64.et[1], 1.0, xt);
      } else {
        launch_cast(H, P32, wlp.r[1], P64, w64.r[1], nf);
        mg16(H, wlp, 1, sp.method, sp.n_fine, sp.n_coarse);
        launch_cast(H, P64, w64.tmp, P32, wlp.et[1], nf);
        launch_axpby(H, P64, nf, 1.0, w64.tmp, 1.0, xt);
      }
    };
    if (H.graphs && !H.timing) {
      if (!graph.exec) capture(H, graph, body);
      hip_check(hipGraphLaunch(graph.exec, H.stream), "graph launch");
    } else {
      body();
    }
    ++cycles;
  }

  void finish(h2mg_solve_info* info, double* col_rel) {
    H2& H = *h;
    if (xuser) launch_scatter16(H, nrhs, xt, xuser, ldx);
    hip_check(hipStreamSynchronize(H.stream), "solve");
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) {
      info->cycles = cycles;
      info->converged = converged ? 1 : 0;
      info->rel_residual = H.history.empty() ? 0.0 : H.history.back();
      info->solve_seconds = secs;
      info->history_len = int(H.history.size());
    }
    if (col_rel)
      for (int k = 0; k < nrhs; ++k) col_rel[k] = rel[k];
    release();
  }
};

h2mg_status check_block_args(const H2& h, int nrhs, int ldb, int ldx, const SolveParams& sp) {
  if (nrhs < 1 || nrhs > NR) return fail(H2MG_ERR_INVALID_ARG, "nrhs must be 1..%d (got %d)", NR, nrhs);
  if (ldb < nrhs || ldx < nrhs) return fail(H2MG_ERR_INVALID_ARG, "leading dimensions must be >= nrhs");
  if (h.T < 2) return fail(H2MG_ERR_INVALID_ARG, "blocks of vectors need a rank of 9 to 64 (got %d)", h.r);
  if (sp.method > CYCLE_F) return fail(H2MG_ERR_INVALID_ARG, "blocks of vectors are solved by V-, W- or F-cycles");
  return H2MG_OK;
}

}  // namespace

h2mg_status matvec_multi(H2& h, int nrhs, const double* x, int ldx, double* y, int ldy) {
  if (nrhs < 1 || nrhs > NR) return fail(H2MG_ERR_INVALID_ARG, "nrhs must be 1..%d (got %d)", NR, nrhs);
  if (ldx < nrhs || ldy < nrhs) return fail(H2MG_ERR_INVALID_ARG, "leading dimensions must be >= nrhs");
  if (h.T < 2) return fail(H2MG_ERR_INVALID_ARG, "products with vector blocks need a rank of 9 to 64 (got %d)", h.r);
  try {
    ensure_block(h, P64);
    BlockWork& w = h.blk16;
    launch_gather16(h, nrhs, x, ldx, w.bx);
    apply_fine16(h, P64, w.bx, w.by, 1.0, nullptr, 0.0);
    launch_scatter16(h, nrhs, w.by, y, ldy);
  } catch (const std::bad_alloc&) {
    return fail(H2MG_ERR_OOM, "device allocation failed for the vector-block product");
  } catch (const std::exception& ex) {
    return fail(H2MG_ERR_HIP, "%s", ex.what());
  }
  return H2MG_OK;
}

h2mg_status solve_multi(H2& h, int nrhs, const double* b, int ldb, double* x, int ldx, const SolveParams& sp,
                        h2mg_solve_info* info, double* col_rel) {
  h2mg_status st = check_block_args(h, nrhs, ldb, ldx, sp);
  if (st != H2MG_OK) return st;
  try {
    BlockSolve bs;
    st = bs.begin(h, nrhs, b, ldb, x, ldx, sp);
    if (st != H2MG_OK) return st;
    while (!bs.done) {
      bs.enqueue_residual();
      hip_check(hipEventSynchronize(bs.ev), "sync");
      bs.check();
      if (!bs.done) bs.enqueue_cycle();
    }
    st = bs.status;
    bs.finish(info, col_rel);
  } catch (const std::bad_alloc&) {
    return fail(H2MG_ERR_OOM, "device allocation failed in the block solve");
  } catch (const std::exception& ex) {
    return fail(H2MG_ERR_HIP, "%s", ex.what());
  }
  return st;
}

h2mg_status solve_batch(int nprob, H2* const* hs, const int* nrhs, const double* const* b, const int* ldb,
                        double* const* x, const int* ldx, const SolveParams& sp, h2mg_solve_info* infos,
                        h2mg_status* statuses, int nstreams, hipStream_t user) {
  if (nprob < 1) return fail(H2MG_ERR_INVALID_ARG, "a batch needs at least one problem");
  for (int i = 0; i < nprob; ++i) {
    if (!hs[i] || !b[i] || !x[i]) return fail(H2MG_ERR_INVALID_ARG, "null argument in problem %d", i);
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(H2MG_ERR_INVALID_ARG, "problems %d and %d share a handle", j, i);
    h2mg_status st = check_block_args(*hs[i], nrhs[i], ldb[i], ldx[i], sp);
    if (st != H2MG_OK) return st;
  }
  const int ns = std::max(1, std::min(nstreams > 0 ? nstreams : 4, nprob));
  std::vector<hipStream_t> streams(ns, nullptr);
  std::vector<hipStream_t> saved(nprob);
  for (int i = 0; i < nprob; ++i) saved[i] = hs[i]->stream;
  hipEvent_t start = nullptr;
  std::vector<h2mg_status> result(nprob, H2MG_OK);
  std::vector<std::string> message(nprob);
  std::vector<std::unique_ptr<BlockSolve>> bs(nprob);
  auto record = [&](int i, h2mg_status st) {
    if (st != H2MG_OK && result[i] == H2MG_OK) {
      result[i] = st;
      message[i] = last_error_cstr();
    }
  };
  auto cleanup = [&]() {
    for (auto& s : bs) s.reset();
    for (int i = 0; i < nprob; ++i) hs[i]->stream = saved[i];
    for (hipStream_t s : streams)
      if (s) (void)hipStreamDestroy(s);
    if (start) (void)hipEventDestroy(start);
  };
  h2mg_status err = H2MG_OK;
  try {
    hip_check(hipEventCreateWithFlags(&start, hipEventDisableTiming), "event create");
    hip_check(hipEventRecord(start, user), "event");
    for (int s = 0; s < ns; ++s) {
      hip_check(hipStreamCreateWithFlags(&streams[s], hipStreamNonBlocking), "stream create");
      hip_check(hipStreamWaitEvent(streams[s], start, 0), "stream wait");
    }
    for (int i = 0; i < nprob; ++i) hs[i]->stream = streams[i % ns];
    for (int i = 0; i < nprob; ++i) {
      bs[i].reset(new BlockSolve);
      const h2mg_status st = bs[i]->begin(*hs[i], nrhs[i], b[i], ldb[i], x[i], ldx[i], sp);
      record(i, st);
      if (st != H2MG_OK) bs[i].reset();
      else if (!bs[i]->done) bs[i]->enqueue_residual();
    }
    // Round robin: each problem's residual norms are read as soon as its own
    // stream has produced them, while the other streams keep running.
    for (bool active = true; active;) {
      active = false;
      for (int i = 0; i < nprob; ++i) {
        if (!bs[i]) continue;
        if (!bs[i]->done) {
          hip_check(hipEventSynchronize(bs[i]->ev), "sync");
          bs[i]->check();
          record(i, bs[i]->status);
        }
        if (bs[i]->done) {
          bs[i]->finish(infos ? infos + i : nullptr, nullptr);
          bs[i].reset();
          continue;
        }
        bs[i]->enqueue_cycle();
        bs[i]->enqueue_residual();
        active = true;
      }
    }
  } catch (const std::bad_alloc&) {
    err = H2MG_ERR_OOM;
  } catch (const std::exception& ex) {
    err = H2MG_ERR_HIP;
    message[0] = ex.what();
  }
  if (err != H2MG_OK) {
    (void)hipDeviceSynchronize();
    cleanup();
    return err == H2MG_ERR_OOM ? fail(err, "device allocation failed in the batched solve")
                               : fail(err, "%s", message[0].c_str());
  }
  cleanup();
  if (statuses)
    for (int i = 0; i < nprob; ++i) statuses[i] = result[i];
  for (int i = 0; i < nprob; ++i)
    if (result[i] != H2MG_OK) return fail(result[i], "problem %d: %s", i, message[i].c_str());
  return H2MG_OK;
}

h2mg_status solve_group(int nprob, H2* const* hs, const int* nrhs, const double* const* b, const int* ldb,
                        double* const* x, const int* ldx, const SolveParams& sp, h2mg_solve_info* infos,
                        h2mg_status* statuses, hipStream_t user) {
  if (nprob < 1) return fail(H2MG_ERR_INVALID_ARG, "a group needs at least one problem");
  for (int i = 0; i < nprob; ++i) {
    if (!hs[i] || !b[i] || !x[i]) return fail(H2MG_ERR_INVALID_ARG, "null argument in problem %d", i);
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(H2MG_ERR_INVALID_ARG, "problems %d and %d share a handle", j, i);
    h2mg_status st = check_block_args(*hs[i], nrhs[i], ldb[i], ldx[i], sp);
    if (st != H2MG_OK) return st;
  }
  std::vector<hipStream_t> saved(nprob);
  for (int i = 0; i < nprob; ++i) saved[i] = hs[i]->stream;
  std::vector<h2mg_status> result(nprob, H2MG_OK);
  std::vector<std::string> message(nprob);
  std::vector<std::unique_ptr<BlockSolve>> bs(nprob);
  hipStream_t cap = nullptr;
  CycleGraph graph;
  std::vector<int> graph_set;          // members of the captured cycle
  std::vector<int> eager_set;          // members of the last cycle run kernel by kernel
  hipEvent_t eager_ev[2] = {nullptr, nullptr};
  double eager_host_ms = 0.0;          // host time to enqueue that cycle
  bool eager_pending = false;          // its GPU time not read yet
  bool eager_launch_bound = false;
  GroupLanes lanes;
  auto record = [&](int i, h2mg_status st) {
    if (st != H2MG_OK && result[i] == H2MG_OK) {
      result[i] = st;
      message[i] = last_error_cstr();
    }
  };
  auto cleanup = [&]() {
    t_lanes = nullptr;
    for (hipEvent_t& e : eager_ev)
      if (e) {
        (void)hipEventDestroy(e);
        e = nullptr;
      }
    graph.reset();
    for (auto& q : bs) q.reset();
    for (int i = 0; i < nprob; ++i) hs[i]->stream = saved[i];
    if (cap) (void)hipStreamDestroy(cap);
    lanes.destroy();
  };
  const int p = sp.precision == 0 ? P64 : sp.precision == 1 ? P32 : P16;
  bool graphs = true;
  for (int i = 0; i < nprob; ++i) graphs = graphs && hs[i]->graphs && !hs[i]->timing;
  h2mg_status err = H2MG_OK;
  try {
    for (int i = 0; i < nprob; ++i) hs[i]->stream = user;
    if (nprob > 1) {
      lanes.create(std::min(nprob, GROUP_LANES));
      t_lanes = &lanes;
    }
    for (int i = 0; i < nprob; ++i) {
      bs[i].reset(new BlockSolve);
      const h2mg_status st = bs[i]->begin(*hs[i], nrhs[i], b[i], ldb[i], x[i], ldx[i], sp);
      record(i, st);
      if (st != H2MG_OK) bs[i].reset();
    }
    for (;;) {
      std::vector<int> act;
      for (int i = 0; i < nprob; ++i)
        if (bs[i] && !bs[i]->done) act.push_back(i);
      if (act.empty()) break;
      // residuals R = B - A_H2 X of every active problem (FP64), one group product
      std::vector<GM> G64;
      std::vector<const void*> X, add;
      std::vector<void*> Y;
      for (int i : act) {
        G64.push_back(GM{hs[i], &bs[i]->w64});
        X.push_back(bs[i]->xt);
        Y.push_back(bs[i]->w64.r[1]);
        add.push_back(bs[i]->bt);
      }
      apply16_group(G64, P64, 1, X, Y, -1.0, &add, 1.0);
      for (int i : act) {
        launch_dot16(*hs[i], P64, hs[i]->n, bs[i]->w64.r[1], bs[i]->w64.r[1], bs[i]->npart);
        bs[i]->read_async();
      }
      std::vector<int> next;
      for (int i : act) {
        hip_check(hipEventSynchronize(bs[i]->ev), "sync");
        bs[i]->check();
        record(i, bs[i]->status);
        if (bs[i]->done) {
          bs[i]->finish(infos ? infos + i : nullptr, nullptr);
          bs[i].reset();
        } else {
          next.push_back(i);
        }
      }
      if (next.empty()) break;
      // one cycle of every remaining problem, the tile products of each step in one launch
      auto body = [&]() {
        std::vector<GM> G;
        for (int i : next) G.push_back(GM{hs[i], p == P64 ? &bs[i]->w64 : &bs[i]->wlp});
        if (p != P64) {
          MemberSection cast(G);
          for (int i : next)
            launch_cast(*hs[i], P32, bs[i]->wlp.r[1], P64, bs[i]->w64.r[1], int64_t(hs[i]->n) * NR);
          cast.end();
        }
        mg16_group(G, 1, sp.method, sp.n_fine, sp.n_coarse);
        MemberSection update(G);
        for (int i : next) {
          H2& H = *hs[i];
          const int64_t nf = int64_t(H.n) * NR;
          if (p == P64) {
            launch_axpby(H, P64, nf, 1.0, bs[i]->w64.et[1], 1.0, bs[i]->xt);
          } else {
            launch_cast(H, P64, bs[i]->w64.tmp, P32, bs[i]->wlp.et[1], nf);
            launch_axpby(H, P64, nf, 1.0, bs[i]->w64.tmp, 1.0, bs[i]->xt);
          }
        }
        update.end();
      };
      // A new active set (a member converged or failed) runs its first cycle
      // kernel by kernel, timed on the host (enqueue) and on the GPU.  When
      // the set repeats, its cycle is captured only if that cycle was
      // clearly launch-bound (enqueueing took at least twice the GPU time):
      // a graph saves only the enqueue time beyond the GPU time, while
      // capturing and instantiating a graph of every member's launches costs
      // several cycles' worth of enqueueing (measured: with an 80% threshold
      // four batched problems took 10.8 s against 6.6 s kernel by kernel).
      if (eager_pending) {
        float ms = 0.0f;
        hip_check(hipEventElapsedTime(&ms, eager_ev[0], eager_ev[1]), "cycle time");
        eager_launch_bound = eager_host_ms >= 2.0 * double(ms);
        eager_pending = false;
      }
      const bool capture_now = graphs && graph_set != next && next == eager_set && eager_launch_bound;
      if (graphs && graph_set != next && !capture_now) {
        if (next != eager_set) {
          if (!eager_ev[0]) {
            hip_check(hipEventCreate(&eager_ev[0]), "event");
            hip_check(hipEventCreate(&eager_ev[1]), "event");
          }
          eager_set = next;
          const auto t0 = std::chrono::steady_clock::now();
          hip_check(hipEventRecord(eager_ev[0], user), "event");
          body();
          hip_check(hipEventRecord(eager_ev[1], user), "event");
          eager_host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
          eager_pending = true;
        } else {
          body();
        }
      } else if (graphs) {
        if (capture_now) {
          // the active set changed: record the cycle of the new set
          graph.reset();
          if (!cap) hip_check(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "stream create");
          for (int i : next) hs[i]->stream = cap;
          hip_check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
          try {
            body();
          } catch (...) {
            hipGraph_t partial = nullptr;
            (void)hipStreamEndCapture(cap, &partial);
            if (partial) (void)hipGraphDestroy(partial);
            for (int i : next) hs[i]->stream = user;
            throw;
          }
          for (int i : next) hs[i]->stream = user;
          hip_check(hipStreamEndCapture(cap, &graph.graph), "end capture");
          hip_check(hipGraphInstantiate(&graph.exec, graph.graph, nullptr, nullptr, 0), "graph instantiate");
          graph_set = next;
        }
        hip_check(hipGraphLaunch(graph.exec, user), "graph launch");
      } else {
        body();
      }
      for (int i : next) ++bs[i]->cycles;
    }
  } catch (const std::bad_alloc&) {
    err = H2MG_ERR_OOM;
  } catch (const std::exception& ex) {
    err = H2MG_ERR_HIP;
    message[0] = ex.what();
  }
  if (err != H2MG_OK) {
    (void)hipDeviceSynchronize();
    cleanup();
    return err == H2MG_ERR_OOM ? fail(err, "device allocation failed in the group solve")
                               : fail(err, "%s", message[0].c_str());
  }
  cleanup();
  if (statuses)
    for (int i = 0; i < nprob; ++i) statuses[i] = result[i];
  for (int i = 0; i < nprob; ++i)
    if (result[i] != H2MG_OK) return fail(result[i], "problem %d: %s", i, message[i].c_str());
  return H2MG_OK;
}

}  // namespace h2mg
