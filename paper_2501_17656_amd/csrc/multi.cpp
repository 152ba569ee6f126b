// The H2 matvec of Section 3.1 on a block of up to 16 vectors (FP64): the
// same upsweep, couplings, downsweep and close leaf blocks as the single
// product, with the r x r tile products done 16 columns at a time on the
// matrix cores (kernels_multi.hip).  Needs rank r = 64 and the stored near
// field (its 64 x 64 tiles go through the same tile product).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <stdexcept>
#include <vector>

#include "h2_build.h"

namespace h2mg {

namespace {

constexpr int NR = MULTI_NR;
constexpr int RUN = 16;                // tiles per column-pass task

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
T* upload_owned(H2& h, const std::vector<T>& v) {
  T* d = h.arena.make<T>(std::max<size_t>(v.size(), 1));
  h.multi.owned.push_back(d);
  if (!v.empty())
    hip_check(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, h.stream), "upload");
  return d;
}

double* alloc_owned(H2& h, size_t n) {
  double* d = h.arena.make<double>(std::max<size_t>(n, 1));
  h.multi.owned.push_back(d);
  return d;
}

// Column-pass tasks over the off-diagonal tiles (rows[b] != cols[b]) among
// `ids`, by column (ascending column, then tile order): order, tasks and the
// per-column task ranges (ncol + 1 entries).
void column_tasks(const std::vector<int>& ids, const std::vector<int>& rows, const std::vector<int>& cols,
                  int ncol, std::vector<int>& order, std::vector<int>& tasks, std::vector<int>& ctp) {
  std::vector<std::pair<int, int>> cb;
  for (int b : ids)
    if (rows[b] != cols[b]) cb.emplace_back(cols[b], b);
  std::stable_sort(cb.begin(), cb.end(), [](const auto& u, const auto& v) { return u.first < v.first; });
  order.resize(cb.size());
  for (size_t i = 0; i < cb.size(); ++i) order[i] = cb[i].second;
  ctp.assign(ncol + 1, 0);
  for (size_t i = 0; i < cb.size();) {
    size_t e = i;
    while (e < cb.size() && cb[e].first == cb[i].first) ++e;
    for (size_t c = i; c < e; c += RUN) {
      tasks.push_back(cb[i].first);
      tasks.push_back(int(c));
      tasks.push_back(int(std::min(e, c + RUN)));
      ctp[cb[i].first + 1]++;
    }
    i = e;
  }
  for (int c = 0; c < ncol; ++c) ctp[c + 1] += ctp[c];
}

void ensure_multi(H2& h) {
  MultiWork& m = h.multi;
  if (m.ready) return;
  const size_t r = size_t(h.r);
  m.x = alloc_owned(h, size_t(h.n) * NR);
  m.y = alloc_owned(h, size_t(h.n) * NR);
  int64_t ptasks = 0;
  if (h.d_top >= 0) {
    m.xall = alloc_owned(h, size_t(h.ngid) * r * NR);
    m.yall = alloc_owned(h, size_t(h.ngid) * r * NR);
    hip_check(hipMemsetAsync(m.yall, 0, size_t(h.ngid) * r * NR * sizeof(double), h.stream), "memset");
    // row-pass ranges per gid from the single-vector tasks of every depth
    std::vector<int> rtp(h.ngid + 1, 0);
    std::vector<int> ids;
    for (int d = h.d_top; d <= h.L; ++d) {
      const View& v = h.sview[d];
      for (size_t i = 0; i < v.task.size(); i += 3) rtp[v.task[i] + 1]++;
      for (int b = h.s_first[d]; b < h.s_first[d] + h.s_count[d]; ++b) ids.push_back(b);
    }
    for (int g = 0; g < h.ngid; ++g) rtp[g + 1] += rtp[g];
    std::vector<int> order, tasks, ctp;
    column_tasks(ids, h.blk_row_h, h.blk_col_h, h.ngid, order, tasks, ctp);
    m.rtp = upload_owned(h, rtp);
    m.ctp = upload_owned(h, ctp);
    m.corder = upload_owned(h, order);
    m.ctask = upload_owned(h, tasks);
    m.nctask = int(tasks.size() / 3);
    ptasks = std::max<int64_t>(ptasks, int64_t(h.fine_launch.ntasks) + m.nctask);
  }
  const StoredNear& sn = h.snear;
  {
    std::vector<int> ids(sn.brow_h.size());
    for (size_t b = 0; b < ids.size(); ++b) ids[b] = int(b);
    std::vector<int> order, tasks, ctp;
    column_tasks(ids, sn.brow_h, sn.bcol_h, sn.nchunk, order, tasks, ctp);
    m.near_ctp = upload_owned(h, ctp);
    m.near_corder = upload_owned(h, order);
    m.near_ctask = upload_owned(h, tasks);
    m.near_nctask = int(tasks.size() / 3);
    ptasks = std::max<int64_t>(ptasks, int64_t(sn.ntasks) + m.near_nctask);
    if (!sn.identity) {
      const size_t nv = size_t(sn.nchunk) * 64 * NR;
      m.xc = alloc_owned(h, nv);
      hip_check(hipMemsetAsync(m.xc, 0, nv * sizeof(double), h.stream), "memset");
    }
    m.yc = alloc_owned(h, size_t(sn.nchunk) * 64 * NR);
  }
  m.partial = alloc_owned(h, size_t(std::max<int64_t>(ptasks, 1)) * 64 * NR);
  m.partial_tasks = ptasks;
  hip_check(hipStreamSynchronize(h.stream), "multi setup");
  m.ready = true;
}

}  // namespace

h2mg_status matvec_multi(H2& h, int nrhs, const double* x, int ldx, double* y, int ldy) {
  if (nrhs < 1 || nrhs > NR) return fail(H2MG_ERR_INVALID_ARG, "nrhs must be 1..%d (got %d)", NR, nrhs);
  if (ldx < nrhs || ldy < nrhs) return fail(H2MG_ERR_INVALID_ARG, "leading dimensions must be >= nrhs");
  if (h.r != 64) return fail(H2MG_ERR_INVALID_ARG, "products with vector blocks need rank 64 (got %d)", h.r);
  if (!h.snear.ready) return fail(H2MG_ERR_STATE, "products with vector blocks need h2mg_store_near first");
  try {
    ensure_multi(h);
    MultiWork& m = h.multi;
    const StoredNear& sn = h.snear;
    const int r = h.r;
    auto at = [&](double* base, int d) { return base + size_t((1 << d) - 1) * r * NR; };
    launch_gather16(h, nrhs, x, ldx, m.x);
    if (h.d_top >= 0) {
      launch_leaf_up16(h, m.x, at(m.xall, h.L));
      for (int d = h.L - 1; d >= h.d_top; --d) launch_transfer_up16(h, d, at(m.xall, d + 1), at(m.xall, d));
      const double* blk = static_cast<const double*>(h.prec[P64].blk);
      launch_gemm16(h, true, h.fine_launch.task, h.fine_launch.ntasks, blk, nullptr, h.blk_col, m.xall,
                    m.partial);
      launch_gemm16(h, false, m.ctask, m.nctask, blk, m.corder, h.blk_row, m.xall,
                    m.partial + size_t(h.fine_launch.ntasks) * 64 * NR);
      launch_reduce16(h, h.ngid, m.rtp, m.ctp, h.fine_launch.ntasks, m.partial, m.yall);
      for (int d = h.d_top + 1; d <= h.L; ++d)
        launch_transfer_down16(h, d - 1, at(m.yall, d - 1), at(m.yall, d), at(m.yall, d));
    }
    const double* xc = m.x;
    if (!sn.identity) {
      launch_near_pad16(h, m.x, m.xc);
      xc = m.xc;
    }
    int ev;
    h.time_begin(ev);
    launch_gemm16(h, true, sn.task, sn.ntasks, sn.tiles, nullptr, sn.blk_col, xc, m.partial);
    launch_gemm16(h, false, m.near_ctask, m.near_nctask, sn.tiles, m.near_corder, sn.blk_row, xc,
                  m.partial + size_t(sn.ntasks) * 64 * NR);
    h.time_end(KS_NEAR16, ev, 2.0 * double(sn.nblocks) * 64.0 * 64.0 * sizeof(double));
    launch_reduce16(h, sn.nchunk, sn.row_task_ptr, m.near_ctp, sn.ntasks, m.partial, m.yc);
    launch_fine_reduce16(h, h.d_top >= 0 ? at(m.yall, h.L) : nullptr, m.yc, m.y);
    launch_scatter16(h, nrhs, m.y, y, ldy);
  } catch (const std::bad_alloc&) {
    return fail(H2MG_ERR_OOM, "device allocation failed for the vector-block product");
  } catch (const std::exception& ex) {
    return fail(H2MG_ERR_HIP, "%s", ex.what());
  }
  return H2MG_OK;
}

}  // namespace h2mg
