// Apply kernels of the H2 matvec and of the restricted operators.
//
// Section 3.1: y = A x is computed by the upsweep x_i = V_i x_{i-1} (leaf
// bases then transfers), the per-level coupling products, the downsweep
// y_{i-1} = D_i x_{i-1} + U_i y_i, and the close (near-field) leaf blocks
// y = D x + U_1 y_1.  Section 3.3: a restricted operator A_k has the same
// structure with the projected close blocks of its depth in place of D.
//
// Every r x r block product is HBM-bound (one FMA per stored word), so the
// blocks are stored once (upper triangle, symmetric operators) in the tiled
// layout of device_common.h and each wave streams one run of blocks of a
// block row: it accumulates B x_t for the row in registers and emits
// B^T x_s for the block's column, which a reduce pass gathers in a fixed
// order (deterministic, no atomics).
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>

#include "h2_impl.h"

namespace h2mg {

namespace {

void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

template <typename Tv> __device__ inline Tv zero() { return Tv(0); }

// ------------------------------------------------------------ symmetric block GEMV
// Sum over the 8 lanes that share b (lane bits 3..5 = a) of T values each,
// as a butterfly transpose-reduce: afterwards lane (a, b) holds the full sum
// of value index a (T = 8), or of index a >> (3 - log2 T) for smaller T.
template <int T, typename Tv>
__device__ inline Tv transpose_reduce_a(Tv (&z)[T], int a) {
  if constexpr (T == 1) {
    Tv s = z[0];
    s += shfl_xor(s, 8);
    s += shfl_xor(s, 16);
    s += shfl_xor(s, 32);
    return s;
  } else {
    // halve the value set at each step, masks 32, 16, 8 (a bits 2, 1, 0)
    constexpr int H = T / 2;
    const bool hi = (a >> 2) & 1;
    Tv v1[H];
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const Tv keep = hi ? z[k + H] : z[k];
      const Tv send = hi ? z[k] : z[k + H];
      v1[k] = keep + shfl_xor(send, 32);
    }
    if constexpr (H == 1) {
      Tv s = v1[0];
      s += shfl_xor(s, 16);
      s += shfl_xor(s, 8);
      return s;
    } else {
      constexpr int Q = H / 2;
      const bool mid = (a >> 1) & 1;
      Tv v2[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const Tv keep = mid ? v1[k + Q] : v1[k];
        const Tv send = mid ? v1[k] : v1[k + Q];
        v2[k] = keep + shfl_xor(send, 16);
      }
      if constexpr (Q == 1) {
        Tv s = v2[0];
        s += shfl_xor(s, 8);
        return s;
      } else {
        const bool lo = a & 1;
        const Tv keep = lo ? v2[1] : v2[0];
        const Tv send = lo ? v2[0] : v2[1];
        return keep + shfl_xor(send, 8);
      }
    }
  }
}

// Value index held by lane a after transpose_reduce_a.
template <int T>
__device__ inline int reduced_index(int a) {
  if constexpr (T == 1) return 0;
  else if constexpr (T == 2) return (a >> 2) & 1;
  else if constexpr (T == 4) return ((a >> 2) & 1) * 2 + ((a >> 1) & 1);
  else return ((a >> 2) & 1) * 4 + ((a >> 1) & 1) * 2 + (a & 1);
}

// One wave per task (row gid s, blocks [b0, b1)).  partial[task] = sum_b B_b x_{col b};
// colpart[slot of b] = B_b^T x_s for every off-diagonal block (slots are
// ordered by column, so the reduce reads each column's run contiguously).
// FULL: r == 8T (no padding, no guards).  Each iteration requests its tile
// first, then the coefficients of its column (the next column index is
// prefetched by a scalar load), so one tile is in flight per wave while the
// previous is consumed.  Every tile is read once per launch, with
// non-temporal loads (measured faster than ordinary loads for FP64, FP32 and
// BF16 tiles alike on the same machine and run).
template <int T, bool FULL, typename Tb, typename Tv>
__device__ __forceinline__ void bsr_gemv_wave(const int* __restrict__ tasks, int ntasks,
                                              const Tb* __restrict__ blk,
                                              const int* __restrict__ blk_col,
                                              const int* __restrict__ blk_slot,
                                              const Tv* __restrict__ x, Tv* __restrict__ partial,
                                              Tv* __restrict__ colpart, int r) {
  constexpr bool NTL = true;
  const int wave = __builtin_amdgcn_readfirstlane(int((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  if (wave >= ntasks) return;
  const int lane = threadIdx.x & 63;
  const int a = lane >> 3, b = lane & 7;
  const int row = tasks[3 * wave], b0 = tasks[3 * wave + 1], b1 = tasks[3 * wave + 2];
  const int rr = FULL ? 8 * T : r;
  Tv xs[T], acc[T];
#pragma unroll
  for (int u = 0; u < T; ++u) {
    const int i = a * T + u;
    xs[u] = (FULL || i < rr) ? x[int64_t(row) * rr + i] : zero<Tv>();
    acc[u] = zero<Tv>();
  }
  int col = blk_col[b0];
  for (int bi = b0; bi < b1; ++bi) {
    Tv B[T * T];
    load_subtile<T, Tb, Tv, NTL>(blk + int64_t(bi) * tile_elems(T), lane, B);
    const int col_next = bi + 1 < b1 ? blk_col[bi + 1] : col;
    Tv xt[T];
#pragma unroll
    for (int v = 0; v < T; ++v) {
      const int j = b * T + v;
      xt[v] = (FULL || j < rr) ? x[int64_t(col) * rr + j] : zero<Tv>();
    }
#pragma unroll
    for (int u = 0; u < T; ++u)
#pragma unroll
      for (int v = 0; v < T; ++v) acc[u] += B[u * T + v] * xt[v];
    if (col != row) {
      Tv z[T];
#pragma unroll
      for (int v = 0; v < T; ++v) {
        Tv s = zero<Tv>();
#pragma unroll
        for (int u = 0; u < T; ++u) s += B[u * T + v] * xs[u];
        z[v] = s;
      }
      const Tv zs = transpose_reduce_a<T, Tv>(z, a);
      const int v = reduced_index<T>(a);
      const int j = b * T + v;
      if ((T == 8 || (a & ((8 / T) - 1)) == 0) && (FULL || j < rr))
        colpart[int64_t(blk_slot[bi]) * rr + j] = zs;
    }
    col = col_next;
  }
#pragma unroll
  for (int u = 0; u < T; ++u) {
    Tv s = acc[u];
    s += shfl_xor(s, 1);
    s += shfl_xor(s, 2);
    s += shfl_xor(s, 4);
    acc[u] = s;
  }
  if (b == 0) {
#pragma unroll
    for (int u = 0; u < T; ++u) {
      const int i = a * T + u;
      if (FULL || i < rr) partial[int64_t(wave) * rr + i] = acc[u];
    }
  }
}

// Couplings and projected close blocks (r x r tiles).
template <int T, bool FULL, typename Tb, typename Tv>
__global__ __launch_bounds__(256) void k_bsr_gemv(const int* __restrict__ tasks, int ntasks,
                                                  const Tb* __restrict__ blk,
                                                  const int* __restrict__ blk_col,
                                                  const int* __restrict__ blk_slot,
                                                  const Tv* __restrict__ x, Tv* __restrict__ partial,
                                                  Tv* __restrict__ colpart, int r) {
  bsr_gemv_wave<T, FULL, Tb, Tv>(tasks, ntasks, blk, blk_col, blk_slot, x, partial, colpart, r);
}

// Stored near field: 64 x 64 FP64 tiles between leaf chunks (same body; a
// kernel of its own so profiles separate it from the coupling products).
__global__ __launch_bounds__(256) void k_near_gemv(const int* __restrict__ tasks, int ntasks,
                                                   const double* __restrict__ tiles,
                                                   const int* __restrict__ blk_col,
                                                   const int* __restrict__ blk_slot,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ partial,
                                                   double* __restrict__ colpart) {
  bsr_gemv_wave<8, true, double, double>(tasks, ntasks, tiles, blk_col, blk_slot, x, partial,
                                         colpart, 64);
}

// The same over FP32 copies of the tiles (close entries given by quadrature,
// which the FP32 products cannot evaluate on the fly).
__global__ __launch_bounds__(256) void k_near_gemv32(const int* __restrict__ tasks, int ntasks,
                                                     const float* __restrict__ tiles,
                                                     const int* __restrict__ blk_col,
                                                     const int* __restrict__ blk_slot,
                                                     const float* __restrict__ x,
                                                     float* __restrict__ partial,
                                                     float* __restrict__ colpart) {
  bsr_gemv_wave<8, true, float, float>(tasks, ntasks, tiles, blk_col, blk_slot, x, partial, colpart, 64);
}

// Sources of one depth for the reduce: task partials of the row (contiguous
// in the launch) and column contributions (contiguous slots).
struct RedDepth {
  const int* rtp[2];     // row -> task offsets within the view
  const int* cptr[2];    // row -> column-slot offsets within the view
  int base[2];           // task base of the view in the GEMV launch
  int slot[2];           // slot base of the view
  int nsrc;
  int row0;              // first grid row of this depth
  int64_t out_off;       // element offset of the depth in the output buffer
};
constexpr int MAX_RED_DEPTHS = 20;
struct RedArgs {
  RedDepth dep[MAX_RED_DEPTHS];
  int ndep;
  int nrows;
};

// One wave per row of any depth: out = sum of its partials, in a fixed order.
template <typename Tv>
__global__ __launch_bounds__(256) void k_reduce(RedArgs A, const Tv* __restrict__ partial,
                                                const Tv* __restrict__ colpart, Tv* __restrict__ out,
                                                Tv* __restrict__ out_last, int r) {
  const int grow = int((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int i = threadIdx.x & 63;
  if (grow >= A.nrows) return;
  int q = 0;
  while (q + 1 < A.ndep && A.dep[q + 1].row0 <= grow) ++q;
  const RedDepth& D = A.dep[q];
  const int row = grow - D.row0;
  if (i >= r) return;
  Tv v0 = zero<Tv>(), v1 = zero<Tv>(), v2 = zero<Tv>(), v3 = zero<Tv>();
  for (int sidx = 0; sidx < D.nsrc; ++sidx) {
    const Tv* pp = partial + int64_t(D.base[sidx]) * r + i;
    int t = D.rtp[sidx][row];
    const int t1 = D.rtp[sidx][row + 1];
    for (; t + 4 <= t1; t += 4) {
      v0 += pp[int64_t(t) * r];
      v1 += pp[int64_t(t + 1) * r];
      v2 += pp[int64_t(t + 2) * r];
      v3 += pp[int64_t(t + 3) * r];
    }
    for (; t < t1; ++t) v0 += pp[int64_t(t) * r];
    const Tv* cp = colpart + int64_t(D.slot[sidx]) * r + i;
    int c = D.cptr[sidx][row];
    const int c1 = D.cptr[sidx][row + 1];
    for (; c + 4 <= c1; c += 4) {
      v0 += cp[int64_t(c) * r];
      v1 += cp[int64_t(c + 1) * r];
      v2 += cp[int64_t(c + 2) * r];
      v3 += cp[int64_t(c + 3) * r];
    }
    for (; c < c1; ++c) v0 += cp[int64_t(c) * r];
  }
  const Tv v = (v0 + v1) + (v2 + v3);
  if (out_last && q == A.ndep - 1) out_last[int64_t(row) * r + i] = v;
  else out[D.out_off + int64_t(row) * r + i] = v;
}

// ------------------------------------------------------------ transfers
// xpar[s] = sum_c E_c^T xchild[c] over the two children of s (depth d -> d+1 kids).
template <int T, typename Tb, typename Tv>
__global__ __launch_bounds__(256) void k_transfer_up(int nparents, int gidc0,
                                                     const Tb* __restrict__ E,
                                                     const Tv* __restrict__ xchild,
                                                     Tv* __restrict__ xpar, int r) {
  const int s = int((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (s >= nparents) return;
  const int lane = threadIdx.x & 63;
  const int a = lane >> 3, b = lane & 7;
  Tv z[T];
#pragma unroll
  for (int v = 0; v < T; ++v) z[v] = zero<Tv>();
  for (int q = 0; q < 2; ++q) {
    const int c = 2 * s + q;
    Tv xs[T];
#pragma unroll
    for (int u = 0; u < T; ++u) {
      const int i = a * T + u;
      xs[u] = i < r ? xchild[int64_t(c) * r + i] : zero<Tv>();
    }
    Tv B[T * T];
    load_subtile<T, Tb, Tv>(E + int64_t(gidc0 + c) * tile_elems(T), lane, B);
#pragma unroll
    for (int v = 0; v < T; ++v)
#pragma unroll
      for (int u = 0; u < T; ++u) z[v] += B[u * T + v] * xs[u];
  }
#pragma unroll
  for (int v = 0; v < T; ++v) {
    Tv s2 = z[v];
    s2 += shfl_xor(s2, 8);
    s2 += shfl_xor(s2, 16);
    s2 += shfl_xor(s2, 32);
    z[v] = s2;
  }
  if (a == 0) {
#pragma unroll
    for (int v = 0; v < T; ++v) {
      const int j = b * T + v;
      if (j < r) xpar[int64_t(s) * r + j] = z[v];
    }
  }
}

// ychild[c] = addend[c] + E_c ypar[c / 2] for every child c at depth d+1.
template <int T, typename Tb, typename Tv>
__global__ __launch_bounds__(256) void k_transfer_down(int nchildren, int gidc0,
                                                       const Tb* __restrict__ E,
                                                       const Tv* __restrict__ ypar,
                                                       Tv* __restrict__ ychild,
                                                       const Tv* __restrict__ addend, int r) {
  const int c = int((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (c >= nchildren) return;
  const int lane = threadIdx.x & 63;
  const int a = lane >> 3, b = lane & 7;
  const int s = c >> 1;
  Tv xt[T];
#pragma unroll
  for (int v = 0; v < T; ++v) {
    const int j = b * T + v;
    xt[v] = j < r ? ypar[int64_t(s) * r + j] : zero<Tv>();
  }
  Tv B[T * T];
  load_subtile<T, Tb, Tv>(E + int64_t(gidc0 + c) * tile_elems(T), lane, B);
  Tv acc[T];
#pragma unroll
  for (int u = 0; u < T; ++u) {
    Tv s2 = zero<Tv>();
#pragma unroll
    for (int v = 0; v < T; ++v) s2 += B[u * T + v] * xt[v];
    s2 += shfl_xor(s2, 1);
    s2 += shfl_xor(s2, 2);
    s2 += shfl_xor(s2, 4);
    acc[u] = s2;
  }
  if (b == 0) {
#pragma unroll
    for (int u = 0; u < T; ++u) {
      const int i = a * T + u;
      if (i < r)
        ychild[int64_t(c) * r + i] = acc[u] + (addend ? addend[int64_t(c) * r + i] : zero<Tv>());
    }
  }
}

// ------------------------------------------------------------ leaf bases
// xhat[leaf] = Q_leaf^T x_leaf; 4 waves split the leaf's rows.
template <typename Tq, typename Tv>
__global__ __launch_bounds__(256) void k_leaf_up(const int* __restrict__ leaf_off,
                                                 const Tq* __restrict__ Qr,
                                                 const Tv* __restrict__ x, Tv* __restrict__ xhat,
                                                 int r) {
  __shared__ Tv red[4][64];
  const int leaf = blockIdx.x;
  const int w = threadIdx.x >> 6, j = threadIdx.x & 63;
  const int s0 = leaf_off[leaf], n = leaf_off[leaf + 1] - s0;
  Tv acc = zero<Tv>();
  if (j < r)
    for (int i = w; i < n; i += 4)
      acc += ld_as<Tv, Tq>(Qr[int64_t(s0 + i) * r + j]) * x[s0 + i];
  red[w][j] = acc;
  __syncthreads();
  if (w == 0 && j < r) xhat[int64_t(leaf) * r + j] = (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
}

// ------------------------------------------------------------ near field
// Close leaf pairs (s <= t) evaluated on the fly from the points: one
// workgroup per task (row leaf s, pairs [p0, p1)), 16 x 16 threads, each
// thread an 8 x 8 sub-tile of a 128 x 128 tile.  Row sums go to
// partial[task], column sums of off-diagonal pairs to colpart[pair].
template <typename Tv, typename Te, int KIND, int DERIV>
__global__ __launch_bounds__(256) void k_near(const int* __restrict__ tasks,
                                              const int* __restrict__ pair_col,
                                              const int* __restrict__ leaf_off,
                                              const double* __restrict__ pts, int dim,
                                              const Tv* __restrict__ x, Tv* __restrict__ partial,
                                              Tv* __restrict__ colpart, int ld, KernelParams kp,
                                              const double* __restrict__ scale) {
  constexpr int TILE = 128;
  __shared__ double ps[TILE * 3];
  __shared__ double pt[TILE * 3];
  __shared__ Tv xsl[TILE];
  __shared__ Tv xtl[TILE];
  __shared__ Tv red[16][TILE + 1];
  const int task = blockIdx.x, tid = threadIdx.x;
  const int ti = tid >> 4, tj = tid & 15;
  const int sl = tasks[3 * task], p0 = tasks[3 * task + 1], p1 = tasks[3 * task + 2];
  const int s0 = leaf_off[sl], ns = leaf_off[sl + 1] - s0;
  for (int rt = 0; rt < ns; rt += TILE) {
    const int nrow = min(TILE, ns - rt);
    __syncthreads();
    for (int idx = tid; idx < TILE * dim; idx += 256) {
      const int i = idx / dim;
      ps[idx] = pts[int64_t(s0 + rt + min(i, nrow - 1)) * dim + idx % dim];
    }
    for (int i = tid; i < TILE; i += 256)
      xsl[i] = i < nrow ? (scale ? Tv(scale[s0 + rt + i]) * x[s0 + rt + i] : x[s0 + rt + i]) : zero<Tv>();
    __syncthreads();
    double pi[8][3];
    Tv xi[8], racc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = ti + 16 * u;
      for (int a = 0; a < 3; ++a) pi[u][a] = a < dim ? ps[i * dim + a] : 0.0;
      xi[u] = xsl[i];
      racc[u] = zero<Tv>();
    }
    for (int p = p0; p < p1; ++p) {
      const int tl = pair_col[p];
      const bool diag = tl == sl;
      const int t0 = leaf_off[tl], nt = leaf_off[tl + 1] - t0;
      for (int ct = 0; ct < nt; ct += TILE) {
        const int ncol = min(TILE, nt - ct);
        __syncthreads();
        for (int idx = tid; idx < TILE * dim; idx += 256) {
          const int j = idx / dim;
          pt[idx] = pts[int64_t(t0 + ct + min(j, ncol - 1)) * dim + idx % dim];
        }
        for (int j = tid; j < TILE; j += 256)
          xtl[j] = j < ncol ? (scale ? Tv(scale[t0 + ct + j]) * x[t0 + ct + j] : x[t0 + ct + j])
                            : zero<Tv>();
        __syncthreads();
#pragma unroll 2
        for (int v = 0; v < 8; ++v) {
          const int j = tj + 16 * v;
          double pj[3];
          for (int a = 0; a < 3; ++a) pj[a] = a < dim ? pt[j * dim + a] : 0.0;
          const Tv xj = xtl[j];
          Tv cacc = zero<Tv>();
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            double r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
              const double dx = pi[u][a] - pj[a];
              r2 += dx * dx;
            }
            Tv k = Tv(kernel_fixed<KIND, DERIV, Te>(Te(kp.inv_l), Te(kp.inv_2l2), Te(r2)));
            if (diag && rt + ti + 16 * u == ct + j) k += Tv(kp.shift);
            racc[u] += k * xj;
            cacc += k * xi[u];
          }
          red[ti][j] = cacc;
        }
        if (!diag) {
          __syncthreads();
          if (tid < TILE) {
            Tv s = zero<Tv>();
#pragma unroll
            for (int q = 0; q < 16; ++q) s += red[q][tid];
            if (tid < ncol) {
              if (scale) s *= Tv(scale[t0 + ct + tid]);
              Tv* dst = colpart + int64_t(p) * ld + ct + tid;
              *dst = rt == 0 ? s : *dst + s;
            }
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      Tv s = racc[u];
      s += shfl_xor(s, 1);
      s += shfl_xor(s, 2);
      s += shfl_xor(s, 4);
      s += shfl_xor(s, 8);
      racc[u] = s;
    }
    if (tj == 0) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = ti + 16 * u;
        if (i < nrow)
          partial[int64_t(task) * ld + rt + i] = scale ? Tv(scale[s0 + rt + i]) * racc[u] : racc[u];
      }
    }
  }
}

// out[idx(i)] = alpha * (Q_leaf yhat_leaf + near sums)_i + beta * add[idx(i)]
// for the rows i of one leaf per workgroup; idx = i or perm[i].
template <typename Tq, typename Tv>
__global__ __launch_bounds__(256) void k_fine_reduce(
    const int* __restrict__ leaf_off, const Tq* __restrict__ Qc, const Tv* __restrict__ yhat, int r,
    const int* __restrict__ row_task_ptr, const int* __restrict__ col_ptr,
    const int* __restrict__ col_pair, const Tv* __restrict__ partial,
    const Tv* __restrict__ colpart, int ld, const Tv* __restrict__ near_y,
    const int* __restrict__ chunk_base, const double* __restrict__ dg, const Tv* __restrict__ xin,
    const int64_t* __restrict__ perm, Tv* __restrict__ out, double alpha, const Tv* __restrict__ add,
    double beta) {
  __shared__ Tv yh[64];
  const int leaf = blockIdx.x;
  const int s0 = leaf_off[leaf], n = leaf_off[leaf + 1] - s0;
  if (threadIdx.x < r) yh[threadIdx.x] = yhat[int64_t(leaf) * r + threadIdx.x];
  __syncthreads();
  const int t0 = row_task_ptr[leaf], t1 = row_task_ptr[leaf + 1];
  const int c0 = col_ptr[leaf], c1 = col_ptr[leaf + 1];
  const Tq* Q = Qc + int64_t(s0) * r;
  for (int i = threadIdx.x; i < n; i += 256) {
    Tv v = zero<Tv>();
    for (int j = 0; j < r; ++j) v += ld_as<Tv, Tq>(Q[int64_t(j) * n + i]) * yh[j];
    if (near_y) {
      v += near_y[int64_t(chunk_base[leaf]) * 64 + i];
    } else {
      for (int t = t0; t < t1; ++t) v += partial[int64_t(t) * ld + i];
      for (int c = c0; c < c1; ++c) v += colpart[int64_t(col_pair[c]) * ld + i];
      if (dg) v += Tv(dg[s0 + i]) * xin[s0 + i];
    }
    const int64_t idx = perm ? perm[s0 + i] : int64_t(s0 + i);
    Tv o = Tv(alpha) * v;
    if (add) o += Tv(beta) * add[idx];
    out[idx] = o;
  }
}

// out[idx(i)] = alpha * (Q_leaf yhat_leaf)_i + beta * add[idx(i)] (prolongation
// from the depth-L coefficients to the points; tree order).
template <typename Tq, typename Tv>
__global__ __launch_bounds__(256) void k_leaf_down(const int* __restrict__ leaf_off,
                                                   const Tq* __restrict__ Qc,
                                                   const Tv* __restrict__ yhat, int r,
                                                   Tv* __restrict__ out, double alpha,
                                                   const Tv* __restrict__ add, double beta) {
  __shared__ Tv yh[64];
  const int leaf = blockIdx.x;
  const int s0 = leaf_off[leaf], n = leaf_off[leaf + 1] - s0;
  if (threadIdx.x < r) yh[threadIdx.x] = yhat[int64_t(leaf) * r + threadIdx.x];
  __syncthreads();
  const Tq* Q = Qc + int64_t(s0) * r;
  for (int i = threadIdx.x; i < n; i += 256) {
    Tv v = zero<Tv>();
    for (int j = 0; j < r; ++j) v += ld_as<Tv, Tq>(Q[int64_t(j) * n + i]) * yh[j];
    Tv o = Tv(alpha) * v;
    if (add) o += Tv(beta) * add[s0 + i];
    out[s0 + i] = o;
  }
}

// xc[chunk_base[leaf] * 64 + i] = x[leaf_off[leaf] + i]: the tree-order
// vector in the chunk-padded layout of the stored near field (padding
// entries are never written and stay zero).
template <typename Tv>
__global__ __launch_bounds__(256) void k_near_pad(const int* __restrict__ leaf_off,
                                                  const int* __restrict__ chunk_base,
                                                  const Tv* __restrict__ x,
                                                  Tv* __restrict__ xc) {
  const int leaf = blockIdx.x;
  const int s0 = leaf_off[leaf], n = leaf_off[leaf + 1] - s0;
  Tv* dst = xc + int64_t(chunk_base[leaf]) * 64;
  for (int i = threadIdx.x; i < n; i += 256) dst[i] = x[s0 + i];
}

// ------------------------------------------------------------ dispatch helpers
template <typename F>
void dispatch_T(int T, F&& f) {
  switch (T) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    default: f(std::integral_constant<int, 8>{}); break;
  }
}

inline int grid_waves(int64_t waves) { return int((waves + 3) / 4); }

}  // namespace

// ------------------------------------------------------------ launchers
void launch_gemv(H2& h, int p, const Launch& l, const void* x_all) {
  if (l.ntasks == 0) return;
  int ev;
  h.time_begin(ev);
  dispatch_T(h.T, [&](auto Tc) {
    constexpr int T = decltype(Tc)::value;
    const dim3 g(grid_waves(l.ntasks)), b(256);
    auto go = [&](auto fullc) {
      constexpr bool F = decltype(fullc)::value;
      if (p == P64)
        hipLaunchKernelGGL((k_bsr_gemv<T, F, double, double>), g, b, 0, h.stream, l.task, l.ntasks,
                           static_cast<const double*>(h.prec[P64].blk), h.blk_col, h.blk_slot,
                           static_cast<const double*>(x_all), h.partial, h.colpart, h.r);
      else if (p == P32)
        hipLaunchKernelGGL((k_bsr_gemv<T, F, float, float>), g, b, 0, h.stream, l.task, l.ntasks,
                           static_cast<const float*>(h.prec[P32].blk), h.blk_col, h.blk_slot,
                           static_cast<const float*>(x_all), reinterpret_cast<float*>(h.partial),
                           reinterpret_cast<float*>(h.colpart), h.r);
      else
        hipLaunchKernelGGL((k_bsr_gemv<T, F, bf16, float>), g, b, 0, h.stream, l.task, l.ntasks,
                           static_cast<const bf16*>(h.prec[P16].blk), h.blk_col, h.blk_slot,
                           static_cast<const float*>(x_all), reinterpret_cast<float*>(h.partial),
                           reinterpret_cast<float*>(h.colpart), h.r);
    };
    if (h.r == 8 * T) go(std::true_type{});
    else go(std::false_type{});
  });
  check_launch("bsr_gemv");
  h.time_end(KS_GEMV64 + p, ev, double(l.nblocks) * h.r * h.r * elem_bytes(p));
}

void launch_reduce(H2& h, int p, int d0, int d1, const View* const* v0, const int* base0,
                   const View* const* v1, const int* base1, void* out, void* out_last) {
  RedArgs A{};
  A.ndep = d1 - d0 + 1;
  if (A.ndep > MAX_RED_DEPTHS) throw std::runtime_error("too many depths for one reduce");
  int rows = 0;
  for (int q = 0; q < A.ndep; ++q) {
    const int d = d0 + q;
    RedDepth& D = A.dep[q];
    D.rtp[0] = v0[q]->row_task_ptr;
    D.cptr[0] = v0[q]->col_ptr;
    D.base[0] = base0[q];
    D.slot[0] = v0[q]->slot_base;
    D.nsrc = 1;
    if (v1 && v1[q]) {
      D.rtp[1] = v1[q]->row_task_ptr;
      D.cptr[1] = v1[q]->col_ptr;
      D.base[1] = base1[q];
      D.slot[1] = v1[q]->slot_base;
      D.nsrc = 2;
    }
    D.row0 = rows;
    D.out_off = int64_t((1 << d) - 1) * h.r;
    rows += 1 << d;
  }
  A.nrows = rows;
  const dim3 g(grid_waves(rows)), b(256);
  if (p == P64)
    hipLaunchKernelGGL(k_reduce<double>, g, b, 0, h.stream, A, h.partial, h.colpart,
                       static_cast<double*>(out), static_cast<double*>(out_last), h.r);
  else
    hipLaunchKernelGGL(k_reduce<float>, g, b, 0, h.stream, A, reinterpret_cast<const float*>(h.partial),
                       reinterpret_cast<const float*>(h.colpart), static_cast<float*>(out),
                       static_cast<float*>(out_last), h.r);
  check_launch("reduce");
}

void launch_transfer_up(H2& h, int p, int d, const void* xchild, void* xpar) {
  const int npar = 1 << d;
  const int gidc0 = (1 << (d + 1)) - 1;
  dispatch_T(h.T, [&](auto Tc) {
    constexpr int T = decltype(Tc)::value;
    const dim3 g(grid_waves(npar)), b(256);
    if (p == P64)
      hipLaunchKernelGGL((k_transfer_up<T, double, double>), g, b, 0, h.stream, npar, gidc0,
                         static_cast<const double*>(h.prec[P64].E), static_cast<const double*>(xchild),
                         static_cast<double*>(xpar), h.r);
    else if (p == P32)
      hipLaunchKernelGGL((k_transfer_up<T, float, float>), g, b, 0, h.stream, npar, gidc0,
                         static_cast<const float*>(h.prec[P32].E), static_cast<const float*>(xchild),
                         static_cast<float*>(xpar), h.r);
    else
      hipLaunchKernelGGL((k_transfer_up<T, bf16, float>), g, b, 0, h.stream, npar, gidc0,
                         static_cast<const bf16*>(h.prec[P16].E), static_cast<const float*>(xchild),
                         static_cast<float*>(xpar), h.r);
  });
  check_launch("transfer_up");
}

void launch_transfer_down(H2& h, int p, int d, const void* ypar, void* ychild, const void* addend) {
  const int nch = 1 << (d + 1);
  const int gidc0 = (1 << (d + 1)) - 1;
  dispatch_T(h.T, [&](auto Tc) {
    constexpr int T = decltype(Tc)::value;
    const dim3 g(grid_waves(nch)), b(256);
    if (p == P64)
      hipLaunchKernelGGL((k_transfer_down<T, double, double>), g, b, 0, h.stream, nch, gidc0,
                         static_cast<const double*>(h.prec[P64].E), static_cast<const double*>(ypar),
                         static_cast<double*>(ychild), static_cast<const double*>(addend), h.r);
    else if (p == P32)
      hipLaunchKernelGGL((k_transfer_down<T, float, float>), g, b, 0, h.stream, nch, gidc0,
                         static_cast<const float*>(h.prec[P32].E), static_cast<const float*>(ypar),
                         static_cast<float*>(ychild), static_cast<const float*>(addend), h.r);
    else
      hipLaunchKernelGGL((k_transfer_down<T, bf16, float>), g, b, 0, h.stream, nch, gidc0,
                         static_cast<const bf16*>(h.prec[P16].E), static_cast<const float*>(ypar),
                         static_cast<float*>(ychild), static_cast<const float*>(addend), h.r);
  });
  check_launch("transfer_down");
}

void launch_leaf_up(H2& h, int p, const void* xtree, void* xhat) {
  const dim3 g(h.nleaf), b(256);
  if (p == P64)
    hipLaunchKernelGGL((k_leaf_up<double, double>), g, b, 0, h.stream, h.leaf_off,
                       static_cast<const double*>(h.prec[P64].Qr), static_cast<const double*>(xtree),
                       static_cast<double*>(xhat), h.r);
  else if (p == P32)
    hipLaunchKernelGGL((k_leaf_up<float, float>), g, b, 0, h.stream, h.leaf_off,
                       static_cast<const float*>(h.prec[P32].Qr), static_cast<const float*>(xtree),
                       static_cast<float*>(xhat), h.r);
  else
    hipLaunchKernelGGL((k_leaf_up<bf16, float>), g, b, 0, h.stream, h.leaf_off,
                       static_cast<const bf16*>(h.prec[P16].Qr), static_cast<const float*>(xtree),
                       static_cast<float*>(xhat), h.r);
  check_launch("leaf_up");
}

void launch_near(H2& h, int p, const void* xtree) {
  if (h.nq > 0) throw std::runtime_error("close entries by quadrature are applied from the stored tiles only");
  if (h.near.ntasks == 0) return;
  int ev;
  h.time_begin(ev);
  const dim3 g(h.near.ntasks), b(256);
  KernelParams kp = h.kp;
  if (h.diag) kp.shift = 0.0;          // the per-point diagonal is added by k_fine_reduce
  dispatch_kernel(h.kp.kind, h.kp.deriv, [&](auto kc, auto dc) {
    constexpr int K = decltype(kc)::value, D = decltype(dc)::value;
    if (p == P64)
      hipLaunchKernelGGL((k_near<double, double, K, D>), g, b, 0, h.stream, h.near.task,
                         h.near.pair_col, h.leaf_off, h.pts, h.dim, static_cast<const double*>(xtree),
                         h.near_partial, h.near_colpart, h.near.ld, kp, h.scale);
    else
      hipLaunchKernelGGL((k_near<float, float, K, D>), g, b, 0, h.stream, h.near.task,
                         h.near.pair_col, h.leaf_off, h.pts, h.dim, static_cast<const float*>(xtree),
                         reinterpret_cast<float*>(h.near_partial),
                         reinterpret_cast<float*>(h.near_colpart), h.near.ld, kp, h.scale);
  });
  check_launch("near");
  h.time_end(p == P64 ? KS_NEAR64 : KS_NEAR32, ev, double(h.near_evals));
}

void launch_near_stored(H2& h, int p, const void* xtree) {
  StoredNear& sn = h.snear;
  if (sn.nblocks == 0) return;
  if (p != P64 && !sn.tiles32) throw std::runtime_error("no FP32 copy of the stored near field");
  RedArgs A{};
  A.ndep = 1;
  A.nrows = sn.nchunk;
  RedDepth& D = A.dep[0];
  D.rtp[0] = sn.row_task_ptr;
  D.cptr[0] = sn.col_ptr;
  D.base[0] = 0;
  D.slot[0] = 0;
  D.nsrc = 1;
  D.row0 = 0;
  D.out_off = 0;
  if (p == P64) {
    const double* xc = static_cast<const double*>(xtree);
    if (!sn.identity) {
      hipLaunchKernelGGL(k_near_pad<double>, dim3(h.nleaf), dim3(256), 0, h.stream, h.leaf_off,
                         sn.chunk_base, xc, sn.xc);
      check_launch("near_pad");
      xc = sn.xc;
    }
    int ev;
    h.time_begin(ev);
    hipLaunchKernelGGL(k_near_gemv, dim3(grid_waves(sn.ntasks)), dim3(256), 0, h.stream, sn.task,
                       sn.ntasks, sn.tiles, sn.blk_col, sn.blk_slot, xc, sn.partial, sn.colpart);
    check_launch("near_gemv");
    h.time_end(KS_NEARST64, ev, double(sn.nblocks) * 64.0 * 64.0 * sizeof(double));
    hipLaunchKernelGGL(k_reduce<double>, dim3(grid_waves(sn.nchunk)), dim3(256), 0, h.stream, A,
                       sn.partial, sn.colpart, sn.yc, static_cast<double*>(nullptr), 64);
  } else {
    // FP32 partials and output in the first half of the FP64 buffers; the
    // padded input has a zero-padded FP32 buffer of its own
    const float* xc = static_cast<const float*>(xtree);
    if (!sn.identity) {
      hipLaunchKernelGGL(k_near_pad<float>, dim3(h.nleaf), dim3(256), 0, h.stream, h.leaf_off,
                         sn.chunk_base, xc, sn.xc32);
      check_launch("near_pad");
      xc = sn.xc32;
    }
    float* part = reinterpret_cast<float*>(sn.partial);
    float* cpart = reinterpret_cast<float*>(sn.colpart);
    hipLaunchKernelGGL(k_near_gemv32, dim3(grid_waves(sn.ntasks)), dim3(256), 0, h.stream, sn.task,
                       sn.ntasks, sn.tiles32, sn.blk_col, sn.blk_slot, xc, part, cpart);
    check_launch("near_gemv32");
    hipLaunchKernelGGL(k_reduce<float>, dim3(grid_waves(sn.nchunk)), dim3(256), 0, h.stream, A,
                       static_cast<const float*>(part), static_cast<const float*>(cpart),
                       reinterpret_cast<float*>(sn.yc), static_cast<float*>(nullptr), 64);
  }
  check_launch("near_reduce");
}

void launch_fine_reduce(H2& h, int p, const void* yhat, void* out, bool to_user, double alpha,
                        const void* add, double beta, const void* xin) {
  const dim3 g(h.nleaf), b(256);
  const int64_t* perm = to_user ? h.perm : nullptr;
  const bool stored = near_stored_for(h, p);
  const double* dg = stored ? nullptr : h.diag;     // stored tiles hold the diagonal
  if (p == P64)
    hipLaunchKernelGGL((k_fine_reduce<double, double>), g, b, 0, h.stream, h.leaf_off,
                       static_cast<const double*>(h.prec[P64].Qc), static_cast<const double*>(yhat),
                       h.r, h.near.row_task_ptr, h.near.col_ptr, h.near.col_pair, h.near_partial,
                       h.near_colpart, h.near.ld, stored ? h.snear.yc : nullptr, h.snear.chunk_base, dg,
                       static_cast<const double*>(xin), perm, static_cast<double*>(out), alpha,
                       static_cast<const double*>(add), beta);
  else if (p == P32)
    hipLaunchKernelGGL((k_fine_reduce<float, float>), g, b, 0, h.stream, h.leaf_off,
                       static_cast<const float*>(h.prec[P32].Qc), static_cast<const float*>(yhat),
                       h.r, h.near.row_task_ptr, h.near.col_ptr, h.near.col_pair,
                       reinterpret_cast<const float*>(h.near_partial),
                       reinterpret_cast<const float*>(h.near_colpart), h.near.ld,
                       stored ? reinterpret_cast<const float*>(h.snear.yc) : nullptr, h.snear.chunk_base, dg,
                       static_cast<const float*>(xin), perm, static_cast<float*>(out), alpha,
                       static_cast<const float*>(add), beta);
  else
    hipLaunchKernelGGL((k_fine_reduce<bf16, float>), g, b, 0, h.stream, h.leaf_off,
                       static_cast<const bf16*>(h.prec[P16].Qc), static_cast<const float*>(yhat),
                       h.r, h.near.row_task_ptr, h.near.col_ptr, h.near.col_pair,
                       reinterpret_cast<const float*>(h.near_partial),
                       reinterpret_cast<const float*>(h.near_colpart), h.near.ld,
                       stored ? reinterpret_cast<const float*>(h.snear.yc) : nullptr, h.snear.chunk_base, dg,
                       static_cast<const float*>(xin), perm, static_cast<float*>(out), alpha,
                       static_cast<const float*>(add), beta);
  check_launch("fine_reduce");
}

void launch_leaf_down(H2& h, int p, const void* yhat, void* out, double alpha, const void* add,
                      double beta) {
  const dim3 g(h.nleaf), b(256);
  if (p == P64)
    hipLaunchKernelGGL((k_leaf_down<double, double>), g, b, 0, h.stream, h.leaf_off,
                       static_cast<const double*>(h.prec[P64].Qc), static_cast<const double*>(yhat),
                       h.r, static_cast<double*>(out), alpha, static_cast<const double*>(add), beta);
  else if (p == P32)
    hipLaunchKernelGGL((k_leaf_down<float, float>), g, b, 0, h.stream, h.leaf_off,
                       static_cast<const float*>(h.prec[P32].Qc), static_cast<const float*>(yhat),
                       h.r, static_cast<float*>(out), alpha, static_cast<const float*>(add), beta);
  else
    hipLaunchKernelGGL((k_leaf_down<bf16, float>), g, b, 0, h.stream, h.leaf_off,
                       static_cast<const bf16*>(h.prec[P16].Qc), static_cast<const float*>(yhat),
                       h.r, static_cast<float*>(out), alpha, static_cast<const float*>(add), beta);
  check_launch("leaf_down");
}

}  // namespace h2mg
