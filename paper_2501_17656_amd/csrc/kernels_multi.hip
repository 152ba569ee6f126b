// Products with many right-hand sides at once (FP64, up to 16 columns).
//
// The H2 matvec of Section 3.1 applied to a block X of 16 vectors.  Vectors
// are stored row-interleaved: entry (i, k) of a block at i * 16 + k, and
// coefficients of cluster g at (g * r + j) * 16 + k, so that one wave load of
// 64 consecutive doubles covers 4 rows of all 16 columns.
//
// With 16 columns the stored r x r tiles become dense 64 x 16 products, done
// on the matrix cores with v_mfma_f64_16x16x4f64 (lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; D[4 t + l / 16][l % 16] comes back
// in accumulator t, as measured on gfx950).  A tile is read from HBM once per
// pass, in the coalesced 16-byte chunks of its storage layout, staged in LDS
// with an XOR
// swizzle of the column index (f(i) below, at most two-way bank conflicts for
// the staging writes and for both operand reads), and multiplied from there:
//   * row pass (tasks = runs of tiles of one block row s):
//       Y_s = sum_t B_st X_t, accumulated in registers over the run;
//   * column pass (tasks = runs of off-diagonal tiles of one block column t):
//       Y_t = sum_s B_st^T X_s.
// Each task writes one 64 x 16 partial; a reduce sums a row's row-pass and
// column-pass partials in a fixed order (deterministic, no atomics).  The
// upper-triangle storage is read twice, once per pass, which costs less than
// writing and re-reading 16-column column contributions per tile.
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>

#include "h2_impl.h"

namespace h2mg {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int NR = MULTI_NR;           // columns of a block

void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

inline unsigned blocks(int64_t n, int nt) { return unsigned((n + nt - 1) / nt); }

// LDS column swizzle: f(i) = M i over GF(2) (6 bits); row i of the staged
// tile holds column j at position j ^ f(i).
__device__ __forceinline__ int swz(int i) {
  return (__popc(i & 52) & 1) | ((__popc(i & 19) & 1) << 1) | ((__popc(i & 27) & 1) << 2) |
         ((__popc(i & 2) & 1) << 3) | ((__popc(i & 37) & 1) << 4) | ((__popc(i & 37) & 1) << 5);
}
__device__ __forceinline__ int lds_at(int i, int j) { return i * 64 + (j ^ swz(i)); }

// Stage one 64 x 64 FP64 tile (T = 8 storage layout: lane (a, b) owns rows
// 8a.., columns 8b.., chunk c holds elements 2c, 2c+1 of its 8 x 8 sub-block)
// in LDS.
__device__ __forceinline__ void stage_tile(const double* __restrict__ tile, double* lds, int lane) {
  const int a = lane >> 3, b = lane & 7;
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
#pragma unroll 8
  for (int c = 0; c < 32; ++c) {
    union { u4 q; double e[2]; } u;
    u.q = *reinterpret_cast<const u4*>(tile + (c * 64 + lane) * 2);
    const int e0 = 2 * c;
    const int i = 8 * a + (e0 >> 3), j = 8 * b + (e0 & 7);
    lds[lds_at(i, j)] = u.e[0];
    lds[lds_at(i, j + 1)] = u.e[1];
  }
}

// ROWS: task = (row, b0, b1) over tiles b0..b1-1; the other index of tile b
// is col[b], operand x of that cluster.  COLS: task = (col, i0, i1) over
// entries of `order` (off-diagonal tiles by column); tile b = order[i], the
// other index is row[b].  partial[task] = the 64 x 16 result.
template <bool ROWS>
__global__ __launch_bounds__(64) void k_gemm16(const int* __restrict__ tasks, int ntasks,
                                               const double* __restrict__ tiles,
                                               const int* __restrict__ order,
                                               const int* __restrict__ other,
                                               const double* __restrict__ x,
                                               double* __restrict__ partial) {
  __shared__ double lds[64 * 64];
  const int task = blockIdx.x;
  if (task >= ntasks) return;
  const int l = threadIdx.x, p = l & 15, q = l >> 4;
  const int i0 = tasks[3 * task + 1], i1 = tasks[3 * task + 2];
  d4 acc[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) acc[s] = d4{0.0, 0.0, 0.0, 0.0};
  for (int it = i0; it < i1; ++it) {
    const int b = ROWS ? it : order[it];
    const int o = other[b];
    __syncthreads();                   // previous tile's operand reads are done
    stage_tile(tiles + int64_t(b) * 4096, lds, l);
    __syncthreads();
    const double* xo = x + int64_t(o) * 64 * NR;
#pragma unroll 4
    for (int kb = 0; kb < 16; ++kb) {
      const double xb = xo[(4 * kb + q) * NR + p];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        // ROWS: A = B[16s + p][4kb + q];  COLS: A = B^T[16s + p][4kb + q] = B[4kb + q][16s + p]
        const double av = ROWS ? lds[lds_at(16 * s + p, 4 * kb + q)] : lds[lds_at(4 * kb + q, 16 * s + p)];
        acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, xb, acc[s], 0, 0, 0);
      }
    }
  }
  double* out = partial + int64_t(task) * 64 * NR;
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int t = 0; t < 4; ++t) out[(16 * s + 4 * t + q) * NR + p] = acc[s][t];
}

// out[row] = sum of the row-pass partials [rtp[row], rtp[row+1]) and the
// column-pass partials [ctp[row], ctp[row+1]) (offset cbase), fixed order.
__global__ __launch_bounds__(256) void k_reduce16(int nrows, const int* __restrict__ rtp,
                                                  const int* __restrict__ ctp, int cbase,
                                                  const double* __restrict__ partial,
                                                  double* __restrict__ out) {
  const int row = blockIdx.x;
  if (row >= nrows) return;
  for (int e = threadIdx.x; e < 64 * NR; e += 256) {
    double v = 0.0;
    for (int t = rtp[row]; t < rtp[row + 1]; ++t) v += partial[int64_t(t) * 64 * NR + e];
    for (int t = ctp[row]; t < ctp[row + 1]; ++t) v += partial[int64_t(cbase + t) * 64 * NR + e];
    out[int64_t(row) * 64 * NR + e] = v;
  }
}

// Tree-order block from user order (columns beyond nrhs zero), and back.
__global__ __launch_bounds__(256) void k_gather16(int64_t n, int nrhs, const int64_t* __restrict__ perm,
                                                  const double* __restrict__ user, int ldu,
                                                  double* __restrict__ tree) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= n * NR) return;
  const int64_t i = idx / NR;
  const int k = int(idx % NR);
  tree[idx] = k < nrhs ? user[perm[i] * ldu + k] : 0.0;
}

__global__ __launch_bounds__(256) void k_scatter16(int64_t n, int nrhs, const int64_t* __restrict__ perm,
                                                   const double* __restrict__ tree,
                                                   double* __restrict__ user, int ldu) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= n * NR) return;
  const int64_t i = idx / NR;
  const int k = int(idx % NR);
  if (k < nrhs) user[perm[i] * ldu + k] = tree[idx];
}

// xhat[leaf] (r x 16) = Q_leaf^T x_leaf.
__global__ __launch_bounds__(256) void k_leaf_up16(const int* __restrict__ leaf_off,
                                                   const double* __restrict__ Qr, int r,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ xhat) {
  const int leaf = blockIdx.x;
  const int s0 = leaf_off[leaf], n = leaf_off[leaf + 1] - s0;
  for (int e = threadIdx.x; e < r * NR; e += 256) {
    const int j = e / NR, k = e % NR;
    double v = 0.0;
    for (int i = 0; i < n; ++i) v += Qr[int64_t(s0 + i) * r + j] * x[int64_t(s0 + i) * NR + k];
    xhat[(int64_t(leaf) * r + j) * NR + k] = v;
  }
}

// xpar[s] = sum_c E_c^T xchild[c] (E tiles in the T-layout).
__global__ __launch_bounds__(256) void k_transfer_up16(int gidc0, const double* __restrict__ E, int r,
                                                       int T, const double* __restrict__ xchild,
                                                       double* __restrict__ xpar) {
  const int s = blockIdx.x;
  for (int e = threadIdx.x; e < r * NR; e += 256) {
    const int j = e / NR, k = e % NR;
    double v = 0.0;
    for (int c = 2 * s; c < 2 * s + 2; ++c) {
      const double* tile = E + int64_t(gidc0 + c) * tile_elems(T);
      for (int i = 0; i < r; ++i)
        v += tile[tile_offset<double>(i, j, T)] * xchild[(int64_t(c) * r + i) * NR + k];
    }
    xpar[(int64_t(s) * r + j) * NR + k] = v;
  }
}

// ychild[c] = addend[c] + E_c ypar[c / 2].
__global__ __launch_bounds__(256) void k_transfer_down16(int gidc0, const double* __restrict__ E, int r,
                                                         int T, const double* __restrict__ ypar,
                                                         double* __restrict__ ychild,
                                                         const double* __restrict__ addend) {
  const int c = blockIdx.x;
  const double* tile = E + int64_t(gidc0 + c) * tile_elems(T);
  for (int e = threadIdx.x; e < r * NR; e += 256) {
    const int i = e / NR, k = e % NR;
    double v = addend ? addend[(int64_t(c) * r + i) * NR + k] : 0.0;
    for (int j = 0; j < r; ++j) v += tile[tile_offset<double>(i, j, T)] * ypar[(int64_t(c >> 1) * r + j) * NR + k];
    ychild[(int64_t(c) * r + i) * NR + k] = v;
  }
}

// y (tree order, n x 16) = Q_leaf yhat_leaf + near (chunk-padded block).
__global__ __launch_bounds__(256) void k_fine_reduce16(const int* __restrict__ leaf_off,
                                                       const double* __restrict__ Qr, int r,
                                                       const double* __restrict__ yhat,
                                                       const double* __restrict__ near_y,
                                                       const int* __restrict__ chunk_base,
                                                       double* __restrict__ y) {
  const int leaf = blockIdx.x;
  const int s0 = leaf_off[leaf], n = leaf_off[leaf + 1] - s0;
  const int64_t nb = int64_t(chunk_base[leaf]) * 64;
  for (int e = threadIdx.x; e < n * NR; e += 256) {
    const int i = e / NR, k = e % NR;
    double v = 0.0;
    if (yhat)
      for (int j = 0; j < r; ++j) v += Qr[int64_t(s0 + i) * r + j] * yhat[(int64_t(leaf) * r + j) * NR + k];
    v += near_y[(nb + i) * NR + k];
    y[int64_t(s0 + i) * NR + k] = v;
  }
}

// Chunk-padded block from the tree-order block (padding stays zero).
__global__ __launch_bounds__(256) void k_near_pad16(const int* __restrict__ leaf_off,
                                                    const int* __restrict__ chunk_base,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ xc) {
  const int leaf = blockIdx.x;
  const int s0 = leaf_off[leaf], n = leaf_off[leaf + 1] - s0;
  double* dst = xc + int64_t(chunk_base[leaf]) * 64 * NR;
  for (int e = threadIdx.x; e < n * NR; e += 256) dst[e] = x[int64_t(s0) * NR + e];
}

}  // namespace

void launch_gemm16(H2& h, bool rows, const int* tasks, int ntasks, const double* tiles,
                   const int* order, const int* other, const double* x, double* partial) {
  if (ntasks == 0) return;
  if (rows)
    hipLaunchKernelGGL(k_gemm16<true>, dim3(ntasks), dim3(64), 0, h.stream, tasks, ntasks, tiles, order,
                       other, x, partial);
  else
    hipLaunchKernelGGL(k_gemm16<false>, dim3(ntasks), dim3(64), 0, h.stream, tasks, ntasks, tiles, order,
                       other, x, partial);
  check_launch("gemm16");
}

void launch_reduce16(H2& h, int nrows, const int* rtp, const int* ctp, int cbase, const double* partial,
                     double* out) {
  if (nrows == 0) return;
  hipLaunchKernelGGL(k_reduce16, dim3(nrows), dim3(256), 0, h.stream, nrows, rtp, ctp, cbase, partial, out);
  check_launch("reduce16");
}

void launch_gather16(H2& h, int nrhs, const double* user, int ldu, double* tree) {
  hipLaunchKernelGGL(k_gather16, dim3(blocks(int64_t(h.n) * NR, 256)), dim3(256), 0, h.stream,
                     int64_t(h.n), nrhs, h.perm, user, ldu, tree);
  check_launch("gather16");
}

void launch_scatter16(H2& h, int nrhs, const double* tree, double* user, int ldu) {
  hipLaunchKernelGGL(k_scatter16, dim3(blocks(int64_t(h.n) * NR, 256)), dim3(256), 0, h.stream,
                     int64_t(h.n), nrhs, h.perm, tree, user, ldu);
  check_launch("scatter16");
}

void launch_leaf_up16(H2& h, const double* x, double* xhat) {
  hipLaunchKernelGGL(k_leaf_up16, dim3(h.nleaf), dim3(256), 0, h.stream, h.leaf_off,
                     static_cast<const double*>(h.prec[P64].Qr), h.r, x, xhat);
  check_launch("leaf_up16");
}

void launch_transfer_up16(H2& h, int d, const double* xchild, double* xpar) {
  hipLaunchKernelGGL(k_transfer_up16, dim3(1 << d), dim3(256), 0, h.stream, (1 << (d + 1)) - 1,
                     static_cast<const double*>(h.prec[P64].E), h.r, h.T, xchild, xpar);
  check_launch("transfer_up16");
}

void launch_transfer_down16(H2& h, int d, const double* ypar, double* ychild, const double* addend) {
  hipLaunchKernelGGL(k_transfer_down16, dim3(1 << (d + 1)), dim3(256), 0, h.stream, (1 << (d + 1)) - 1,
                     static_cast<const double*>(h.prec[P64].E), h.r, h.T, ypar, ychild, addend);
  check_launch("transfer_down16");
}

void launch_fine_reduce16(H2& h, const double* yhat, const double* near_y, double* y) {
  hipLaunchKernelGGL(k_fine_reduce16, dim3(h.nleaf), dim3(256), 0, h.stream, h.leaf_off,
                     static_cast<const double*>(h.prec[P64].Qr), h.r, yhat, near_y, h.snear.chunk_base, y);
  check_launch("fine_reduce16");
}

void launch_near_pad16(H2& h, const double* x, double* xc) {
  hipLaunchKernelGGL(k_near_pad16, dim3(h.nleaf), dim3(256), 0, h.stream, h.leaf_off, h.snear.chunk_base,
                     x, xc);
  check_launch("near_pad16");
}

}  // namespace h2mg
