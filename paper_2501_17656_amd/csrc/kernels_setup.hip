// Setup kernels: nested orthonormal bases, couplings, restricted operators.
//
// Section 3.1 defines the H2 pieces (bases U, transfers, couplings S, close
// blocks D); Section 3.3 requires orthonormal bases and defines the
// restricted operators A_{k+1} = U_k^T A_k V_k^T (eq. a2_str), whose close
// part is the projection of the finer close blocks.  Here:
//   * leaf bases: tensor Chebyshev interpolants evaluated at the points,
//     orthonormalised by Householder QR in LDS (Q, R with R_kk > 0);
//   * transfers: the parent's Lagrange polynomials at the children's nodes,
//     stacked as [R_c1 E_c1; R_c2 E_c2] and orthonormalised the same way, so
//     the nested orthonormal basis of a parent is the QR of its direct basis;
//   * couplings: S = k(xi_s, xi_t) between node sets, then R_s S R_t^T;
//   * projected close blocks: Q_s^T K_st Q_t on close leaf pairs and
//     sum E_c^T M_cc' E_c' over child pairs above;
//   * the coarsest operator assembled densely and factored by Cholesky.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>

#include "h2_impl.h"

namespace h2mg {

namespace {

constexpr int NT = 256;   // threads per workgroup of the setup kernels

__device__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < int(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

__device__ inline double lagrange1(const double* t, int m, int k, double x) {
  double p = 1.0;
  for (int j = 0; j < m; ++j)
    if (j != k) p *= (x - t[j]) / (t[k] - t[j]);
  return p;
}

// prod_a L_{nu_a}((x_a - c_a) / h_a), tensor index with axis 0 fastest.
__device__ inline double tensor_basis(const double* x, const double* c, const double* h,
                                      const double* t, int m, int dim, int nu) {
  double v = 1.0;
  for (int a = 0; a < dim; ++a) {
    const int k = nu % m;
    nu /= m;
    v *= lagrange1(t, m, k, (x[a] - c[a]) / h[a]);
  }
  return v;
}

__device__ inline void node_coord(const double* c, const double* h, const double* t, int m,
                                  int dim, int nu, double* out) {
  for (int a = 0; a < dim; ++a) {
    out[a] = c[a] + h[a] * t[nu % m];
    nu /= m;
  }
}

// Householder QR of the n x nc column-major matrix A (LDS, lda = n), nc <= 64.
// On exit the upper triangle holds R (diagonal = beta_k) and the part below
// the diagonal the Householder vectors (unit leading entry implied).
__device__ void qr_householder(double* A, int n, int nc, double* tau, double* red) {
  const int tid = threadIdx.x;
  for (int k = 0; k < nc; ++k) {
    double* col = A + size_t(k) * n;
    double part = 0.0;
    for (int i = k + 1 + tid; i < n; i += blockDim.x) part += col[i] * col[i];
    const double xn2 = block_sum(part, red);
    const double alpha = col[k];
    double beta = alpha, t = 0.0, scale = 0.0;
    if (xn2 != 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    __syncthreads();
    if (xn2 != 0.0)
      for (int i = k + 1 + tid; i < n; i += blockDim.x) col[i] *= scale;
    if (tid == 0) {
      col[k] = beta;
      tau[k] = t;
    }
    __syncthreads();
    const int ncol = nc - k - 1;
    if (ncol > 0 && t != 0.0) {
      for (int base = 0; base < ncol * 4; base += blockDim.x) {
        const int g = base + tid;
        const bool active = g < ncol * 4;
        const int j = k + 1 + g / 4, part4 = g & 3;
        double w = 0.0;
        if (active) {
          const double* cj = A + size_t(j) * n;
          if (part4 == 0) w = cj[k];
          for (int i = k + 1 + part4; i < n; i += 4) w += col[i] * cj[i];
        }
        w += __shfl_xor(w, 1, 64);
        w += __shfl_xor(w, 2, 64);
        if (active) {
          double* cj = A + size_t(j) * n;
          const double tw = t * w;
          if (part4 == 0) cj[k] -= tw;
          for (int i = k + 1 + part4; i < n; i += 4) cj[i] -= tw * col[i];
        }
      }
    }
    __syncthreads();
  }
}

// Overwrite the factored A with the n x nc matrix Q of orthonormal columns
// (product of the reflectors applied to the first nc unit vectors).
__device__ void qr_form_q(double* A, int n, int nc, const double* tau) {
  const int tid = threadIdx.x;
  for (int k = nc - 1; k >= 0; --k) {
    double* col = A + size_t(k) * n;
    const double t = tau[k];
    if (k < nc - 1) {
      if (tid == 0) col[k] = 1.0;
      __syncthreads();
      const int ncol = nc - k - 1;
      if (t != 0.0) {
        for (int base = 0; base < ncol * 4; base += blockDim.x) {
          const int g = base + tid;
          const bool active = g < ncol * 4;
          const int j = k + 1 + g / 4, part4 = g & 3;
          double w = 0.0;
          if (active) {
            const double* cj = A + size_t(j) * n;
            for (int i = k + part4; i < n; i += 4) w += col[i] * cj[i];
          }
          w += __shfl_xor(w, 1, 64);
          w += __shfl_xor(w, 2, 64);
          if (active) {
            double* cj = A + size_t(j) * n;
            const double tw = t * w;
            for (int i = k + part4; i < n; i += 4) cj[i] -= tw * col[i];
          }
        }
      }
      __syncthreads();
    }
    for (int i = k + 1 + tid; i < n; i += blockDim.x) col[i] *= -t;
    for (int i = tid; i < k; i += blockDim.x) col[i] = 0.0;
    if (tid == 0) col[k] = 1.0 - t;
    __syncthreads();
  }
}

__device__ inline double* tile_ptr(double* base, int64_t id, int T) {
  return base + id * tile_elems(T);
}

// ------------------------------------------------------------ leaf bases
__global__ __launch_bounds__(NT) void k_leaf_basis_qr(
    const double* __restrict__ pts, int dim, const int* __restrict__ leaf_off,
    const double* __restrict__ cbox, const double* __restrict__ hbox,
    const double* __restrict__ nodes, int m, int r, int gid0, const double* __restrict__ scale,
    double* __restrict__ Rall, double* __restrict__ Qr, double* __restrict__ Qc) {
  extern __shared__ double smem[];
  const int leaf = blockIdx.x, tid = threadIdx.x;
  const int s0 = leaf_off[leaf], n = leaf_off[leaf + 1] - s0;
  double* A = smem;
  double* tau = A + size_t(n) * r;
  double* sgn = tau + 64;
  double* red = sgn + 64;
  double* tn = red + 8;
  if (tid < m) tn[tid] = nodes[tid];
  __syncthreads();
  const int gid = gid0 + leaf;
  const double* c = cbox + size_t(gid) * dim;
  const double* h = hbox + size_t(gid) * dim;
  for (int idx = tid; idx < n * r; idx += NT) {
    const int i = idx % n, nu = idx / n;
    const double u = tensor_basis(pts + size_t(s0 + i) * dim, c, h, tn, m, dim, nu);
    A[size_t(nu) * n + i] = scale ? scale[s0 + i] * u : u;
  }
  __syncthreads();
  qr_householder(A, n, r, tau, red);
  if (tid < r) sgn[tid] = A[size_t(tid) * n + tid] < 0.0 ? -1.0 : 1.0;
  __syncthreads();
  double* Rg = Rall + size_t(gid) * r * r;
  for (int idx = tid; idx < r * r; idx += NT) {
    const int i = idx / r, j = idx % r;
    Rg[idx] = i <= j ? sgn[i] * A[size_t(j) * n + i] : 0.0;
  }
  __syncthreads();
  qr_form_q(A, n, r, tau);
  for (int idx = tid; idx < n * r; idx += NT) {
    const int i = idx / r, j = idx % r;
    const double q = sgn[j] * A[size_t(j) * n + i];
    Qr[size_t(s0 + i) * r + j] = q;
    Qc[size_t(s0) * r + size_t(j) * n + i] = q;
  }
}

// ------------------------------------------------------------ transfers
__global__ __launch_bounds__(NT) void k_transfer_qr(
    int d, int dim, const double* __restrict__ cbox, const double* __restrict__ hbox,
    const double* __restrict__ nodes, int m, int r, int T, double* __restrict__ Rall,
    double* __restrict__ E) {
  extern __shared__ double smem[];
  const int tid = threadIdx.x;
  const int sig = blockIdx.x;
  const int gp = (1 << d) - 1 + sig;
  const int n = 2 * r;
  double* A = smem;                      // 2r x r column-major
  double* Eb = A + size_t(n) * r;        // r x r row-major
  double* tau = Eb + size_t(r) * r;
  double* sgn = tau + 64;
  double* red = sgn + 64;
  double* tn = red + 8;
  if (tid < m) tn[tid] = nodes[tid];
  __syncthreads();
  const double* cp = cbox + size_t(gp) * dim;
  const double* hp = hbox + size_t(gp) * dim;
  for (int q = 0; q < 2; ++q) {
    const int gc = (1 << (d + 1)) - 1 + 2 * sig + q;
    const double* cc = cbox + size_t(gc) * dim;
    const double* hc = hbox + size_t(gc) * dim;
    for (int idx = tid; idx < r * r; idx += NT) {
      const int nup = idx / r, nu = idx % r;   // E[nu'][nu] = L^parent_nu(xi^child_nu')
      double xi[3];
      node_coord(cc, hc, tn, m, dim, nup, xi);
      Eb[idx] = tensor_basis(xi, cp, hp, tn, m, dim, nu);
    }
    __syncthreads();
    const double* Rc = Rall + size_t(gc) * r * r;
    for (int idx = tid; idx < r * r; idx += NT) {
      const int i = idx / r, nu = idx % r;
      double s = 0.0;
      for (int p = i; p < r; ++p) s += Rc[size_t(i) * r + p] * Eb[size_t(p) * r + nu];
      A[size_t(nu) * n + q * r + i] = s;
    }
    __syncthreads();
  }
  qr_householder(A, n, r, tau, red);
  if (tid < r) sgn[tid] = A[size_t(tid) * n + tid] < 0.0 ? -1.0 : 1.0;
  __syncthreads();
  double* Rg = Rall + size_t(gp) * r * r;
  for (int idx = tid; idx < r * r; idx += NT) {
    const int i = idx / r, j = idx % r;
    Rg[idx] = i <= j ? sgn[i] * A[size_t(j) * n + i] : 0.0;
  }
  __syncthreads();
  qr_form_q(A, n, r, tau);
  for (int q = 0; q < 2; ++q) {
    const int gc = (1 << (d + 1)) - 1 + 2 * sig + q;
    double* Et = tile_ptr(E, gc, T);
    for (int idx = tid; idx < r * r; idx += NT) {
      const int i = idx / r, j = idx % r;
      Et[tile_offset<double>(i, j, T)] = sgn[j] * A[size_t(j) * n + q * r + i];
    }
  }
}

// ------------------------------------------------------------ couplings
__global__ __launch_bounds__(NT) void k_coupling(
    int b0, const int* __restrict__ blk_row, const int* __restrict__ blk_col, int dim,
    const double* __restrict__ cbox, const double* __restrict__ hbox,
    const double* __restrict__ nodes, int m, int r, int T, KernelParams kp,
    const double* __restrict__ Rall, double* __restrict__ blk) {
  extern __shared__ double smem[];
  const int tid = threadIdx.x;
  const int b = b0 + blockIdx.x;
  const int gs = blk_row[b], gt = blk_col[b];
  double* S = smem;                  // r x r row-major
  double* T1 = S + size_t(r) * r;
  double* tn = T1 + size_t(r) * r;
  if (tid < m) tn[tid] = nodes[tid];
  __syncthreads();
  const double* cs = cbox + size_t(gs) * dim;
  const double* hs = hbox + size_t(gs) * dim;
  const double* ct = cbox + size_t(gt) * dim;
  const double* ht = hbox + size_t(gt) * dim;
  for (int idx = tid; idx < r * r; idx += NT) {
    const int nu = idx / r, mu = idx % r;
    double xs[3], xt[3];
    node_coord(cs, hs, tn, m, dim, nu, xs);
    node_coord(ct, ht, tn, m, dim, mu, xt);
    double r2 = 0.0;
    for (int a = 0; a < dim; ++a) {
      const double dx = xs[a] - xt[a];
      r2 += dx * dx;
    }
    S[idx] = kernel_r2(kp, r2);
  }
  __syncthreads();
  const double* Rs = Rall + size_t(gs) * r * r;
  const double* Rt = Rall + size_t(gt) * r * r;
  for (int idx = tid; idx < r * r; idx += NT) {     // T1 = S Rt^T
    const int nu = idx / r, q = idx % r;
    double s = 0.0;
    for (int mu = q; mu < r; ++mu) s += S[size_t(nu) * r + mu] * Rt[size_t(q) * r + mu];
    T1[idx] = s;
  }
  __syncthreads();
  double* out = tile_ptr(blk, b, T);
  for (int idx = tid; idx < r * r; idx += NT) {     // Rs T1
    const int i = idx / r, q = idx % r;
    double s = 0.0;
    for (int nu = i; nu < r; ++nu) s += Rs[size_t(i) * r + nu] * T1[size_t(nu) * r + q];
    out[tile_offset<double>(i, q, T)] = s;
  }
}

// ------------------------------------------------------------ projected leaf blocks
// Pi = Q_s^T K_st Q_t for a close leaf pair (K with the shift on the diagonal
// of a diagonal pair).
__global__ __launch_bounds__(NT) void k_pi_leaf(
    int b0, const int* __restrict__ blk_row, const int* __restrict__ blk_col, int gid0,
    const int* __restrict__ leaf_off, const double* __restrict__ pts, int dim, int r, int T,
    KernelParams kp, PointScale ps, const double* __restrict__ Qr, double* __restrict__ blk) {
  extern __shared__ double smem[];
  const int tid = threadIdx.x;
  const int b = b0 + blockIdx.x;
  const int ls = blk_row[b] - gid0, lt = blk_col[b] - gid0;
  const int s0 = leaf_off[ls], ns = leaf_off[ls + 1] - s0;
  const int t0 = leaf_off[lt], nt = leaf_off[lt + 1] - t0;
  const bool diag = ls == lt;
  double* Tm = smem;                      // ns x r row-major
  double* pt = Tm + size_t(ns) * r;       // nt x dim
  for (int idx = tid; idx < nt * dim; idx += NT) pt[idx] = pts[size_t(t0) * dim + idx];
  __syncthreads();
  const int half = (r + 1) / 2;
  for (int i0 = 0; i0 < ns; i0 += 128) {
    const int i = i0 + (tid & 127);
    const int c0 = (tid >> 7) * half;
    const int c1 = min(r, c0 + half);
    double acc[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) acc[q] = 0.0;
    if (i < ns) {
      double pi[3];
      for (int a = 0; a < dim; ++a) pi[a] = pts[size_t(s0 + i) * dim + a];
      for (int j = 0; j < nt; ++j) {
        double r2 = 0.0;
        for (int a = 0; a < dim; ++a) {
          const double dx = pi[a] - pt[j * dim + a];
          r2 += dx * dx;
        }
        const double k = near_entry(kp, ps, dim, r2, s0 + i, t0 + j, diag && i == j);
        const double* qrow = Qr + size_t(t0 + j) * r + c0;
#pragma unroll
        for (int q = 0; q < 32; ++q)
          if (c0 + q < c1) acc[q] += k * qrow[q];
      }
#pragma unroll
      for (int q = 0; q < 32; ++q)
        if (c0 + q < c1) Tm[size_t(i) * r + c0 + q] = acc[q];
    }
  }
  __syncthreads();
  double* out = tile_ptr(blk, b, T);
  for (int idx = tid; idx < r * r; idx += NT) {
    const int mu = idx / r, nu = idx % r;
    double s = 0.0;
    for (int i = 0; i < ns; ++i) s += Qr[size_t(s0 + i) * r + mu] * Tm[size_t(i) * r + nu];
    out[tile_offset<double>(mu, nu, T)] = s;
  }
}

// ------------------------------------------------------------ projected upper blocks
// Pi_st = sum over child pairs (c, c') of E_c^T M_cc' E_c', M = stored child
// block (Pi or S), transposed when the child pair is below the diagonal.
__global__ __launch_bounds__(NT) void k_pi_upper(
    int b0, const int* __restrict__ blk_row, const int* __restrict__ blk_col,
    const int* __restrict__ child_map, int r, int T, const double* __restrict__ E,
    double* __restrict__ blk) {
  extern __shared__ double smem[];
  const int tid = threadIdx.x;
  const int b = b0 + blockIdx.x;
  const int gs = blk_row[b], gt = blk_col[b];
  double* Mb = smem;
  double* Eb = Mb + size_t(r) * r;
  double* W = Eb + size_t(r) * r;
  double* acc = W + size_t(r) * r;       // r x r accumulator
  for (int idx = tid; idx < r * r; idx += NT) acc[idx] = 0.0;
  for (int ab = 0; ab < 4; ++ab) {
    const int a = ab >> 1, bb = ab & 1;
    const int id = child_map[4 * blockIdx.x + ab];
    const bool trans = id < 0;
    const int cid = trans ? -id - 1 : id;
    const double* Mt = blk + int64_t(cid) * tile_elems(T);
    const int gcs = 2 * gs + 1 + a, gct = 2 * gt + 1 + bb;   // child gids
    const double* Et = E + int64_t(gct) * tile_elems(T);
    __syncthreads();
    for (int idx = tid; idx < r * r; idx += NT) {
      const int i = idx / r, j = idx % r;
      Mb[idx] = trans ? Mt[tile_offset<double>(j, i, T)] : Mt[tile_offset<double>(i, j, T)];
      Eb[idx] = Et[tile_offset<double>(i, j, T)];
    }
    __syncthreads();
    for (int idx = tid; idx < r * r; idx += NT) {     // W = M E_c'
      const int i = idx / r, j = idx % r;
      double s = 0.0;
      for (int q = 0; q < r; ++q) s += Mb[size_t(i) * r + q] * Eb[size_t(q) * r + j];
      W[idx] = s;
    }
    __syncthreads();
    const double* Es = E + int64_t(gcs) * tile_elems(T);
    for (int idx = tid; idx < r * r; idx += NT) {
      const int i = idx / r, j = idx % r;
      Eb[idx] = Es[tile_offset<double>(i, j, T)];
    }
    __syncthreads();
    for (int idx = tid; idx < r * r; idx += NT) {     // acc += E_c^T W
      const int mu = idx / r, nu = idx % r;
      double s = 0.0;
      for (int i = 0; i < r; ++i) s += Eb[size_t(i) * r + mu] * W[size_t(i) * r + nu];
      acc[idx] += s;
    }
  }
  __syncthreads();
  double* out = blk + int64_t(b) * tile_elems(T);
  for (int idx = tid; idx < r * r; idx += NT)
    out[tile_offset<double>(idx / r, idx % r, T)] = acc[idx];
}

// ------------------------------------------------------------ dense coarsest operator
__global__ __launch_bounds__(NT) void k_assemble_dense(
    int b0, const int* __restrict__ blk_row, const int* __restrict__ blk_col, int gid0,
    int r, int T, const double* __restrict__ blk, double* __restrict__ A, int64_t lda) {
  const int b = b0 + blockIdx.x;
  const int s = blk_row[b] - gid0, t = blk_col[b] - gid0;
  const double* tl = blk + int64_t(b) * tile_elems(T);
  for (int idx = threadIdx.x; idx < r * r; idx += NT) {
    const int i = idx / r, j = idx % r;
    const double v = tl[tile_offset<double>(i, j, T)];
    const int64_t gi = int64_t(s) * r + i, gj = int64_t(t) * r + j;
    A[gi + gj * lda] = v;
    A[gj + gi * lda] = v;
  }
}

__global__ __launch_bounds__(NT) void k_assemble_kernel_dense(
    const double* __restrict__ pts, int dim, int64_t n, KernelParams kp, PointScale ps,
    double* __restrict__ A) {
  const int64_t idx = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx % n, j = idx / n;
  double r2 = 0.0;
  for (int a = 0; a < dim; ++a) {
    const double dx = pts[i * dim + a] - pts[j * dim + a];
    r2 += dx * dx;
  }
  A[i + j * n] = near_entry(kp, ps, dim, r2, i, j, i == j);
}

// ------------------------------------------------------------ Cholesky (lower, blocked)
constexpr int NB = 64;

__global__ __launch_bounds__(NT) void k_potrf_diag(double* A, int64_t N, int64_t k0, int* flag) {
  if (*flag) return;
  __shared__ double D[NB][NB + 1];
  const int nb = int(min<int64_t>(NB, N - k0));
  const int tid = threadIdx.x;
  for (int idx = tid; idx < nb * nb; idx += NT) {
    const int i = idx % nb, j = idx / nb;
    D[i][j] = A[(k0 + i) + (k0 + j) * N];
  }
  __syncthreads();
  for (int c = 0; c < nb; ++c) {
    const double piv = D[c][c];
    __syncthreads();
    if (!(piv > 0.0)) {
      if (tid == 0) atomicOr(flag, 1);
      return;
    }
    const double dc = sqrt(piv);
    for (int i = c + tid; i < nb; i += NT) D[i][c] = i == c ? dc : D[i][c] / dc;
    __syncthreads();
    const int rem = nb - c - 1;
    for (int idx = tid; idx < rem * rem; idx += NT) {
      const int i = c + 1 + idx % rem, j = c + 1 + idx / rem;
      if (j <= i) D[i][j] -= D[i][c] * D[j][c];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < nb * nb; idx += NT) {
    const int i = idx % nb, j = idx / nb;
    A[(k0 + i) + (k0 + j) * N] = j <= i ? D[i][j] : 0.0;
  }
}

// L_ik = A_ik L_kk^{-T} for every row block i below k (one row per thread).
__global__ __launch_bounds__(NB) void k_trsm_panel(double* A, int64_t N, int64_t k0, const int* flag) {
  if (*flag) return;
  __shared__ double D[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  const int nb = int(min<int64_t>(NB, N - k0));
  const int tid = threadIdx.x;
  for (int idx = tid; idx < nb * nb; idx += NB) {
    const int i = idx % nb, j = idx / nb;
    D[i][j] = A[(k0 + i) + (k0 + j) * N];
  }
  const int64_t row = k0 + nb + int64_t(blockIdx.x) * NB + tid;
  const bool ok = row < N;
  for (int c = 0; c < nb; ++c) X[tid][c] = ok ? A[row + (k0 + c) * N] : 0.0;
  __syncthreads();
  if (!ok) return;
  for (int c = 0; c < nb; ++c) {
    double s = X[tid][c];
    for (int q = 0; q < c; ++q) s -= X[tid][q] * D[c][q];
    X[tid][c] = s / D[c][c];
  }
  for (int c = 0; c < nb; ++c) A[row + (k0 + c) * N] = X[tid][c];
}

// A_ij -= L_ik L_jk^T for row blocks i >= j > k (lower triangle only).
__global__ __launch_bounds__(NT) void k_syrk_update(double* A, int64_t N, int64_t k0, int nbrem,
                                                    const int* flag) {
  if (*flag) return;
  // triangular index of (bi, bj), bi >= bj, over the nbrem trailing blocks
  int p = blockIdx.x, bi = 0;
  while (p > bi) { p -= bi + 1; ++bi; }
  const int bj = p;
  const int nbk = int(min<int64_t>(NB, N - k0));
  const int64_t r0 = k0 + nbk + int64_t(bi) * NB, c0 = k0 + nbk + int64_t(bj) * NB;
  const int ni = int(min<int64_t>(NB, N - r0)), nj = int(min<int64_t>(NB, N - c0));
  __shared__ double Li[NB][NB + 1], Lj[NB][NB + 1];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < NB * NB; idx += NT) {
    const int i = idx % NB, q = idx / NB;
    Li[i][q] = (i < ni && q < nbk) ? A[(r0 + i) + (k0 + q) * N] : 0.0;
    Lj[i][q] = (i < nj && q < nbk) ? A[(c0 + i) + (k0 + q) * N] : 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < NB * NB; idx += NT) {
    const int i = idx % NB, j = idx / NB;
    if (i >= ni || j >= nj) continue;
    if (bi == bj && j > i) continue;
    double s = 0.0;
    for (int q = 0; q < nbk; ++q) s += Li[i][q] * Lj[j][q];
    A[(r0 + i) + (c0 + j) * N] -= s;
  }
}

// ------------------------------------------------------------ block-Jacobi inverses
// In-place Gauss-Jordan inversion of an n x n SPD matrix in LDS (row-major,
// stride n), without pivoting (the pivots of an SPD matrix stay positive).
__device__ void gauss_jordan_spd(double* A, int n, double* fk, int* flag) {
  const int tid = threadIdx.x;
  for (int k = 0; k < n; ++k) {
    __syncthreads();
    const double piv = A[k * n + k];
    if (!(piv > 0.0)) {
      if (tid == 0) atomicOr(flag, 1);
      return;
    }
    const double ip = 1.0 / piv;
    for (int i = tid; i < n; i += NT) fk[i] = A[i * n + k];
    __syncthreads();
    for (int j = tid; j < n; j += NT) A[k * n + j] = (j == k ? 1.0 : A[k * n + j]) * ip;
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += NT) {
      const int i = idx / n, j = idx % n;
      if (i == k) continue;
      const double a = j == k ? 0.0 : A[idx];
      A[idx] = a - fk[i] * A[k * n + j];
    }
  }
  __syncthreads();
}

// Inverse of K_ss + shift I for every leaf s, written as ld x ld blocks
// (entries beyond the leaf size are zero).
__global__ __launch_bounds__(NT) void k_bj_inv_fine(const int* __restrict__ leaf_off,
                                                    const double* __restrict__ pts, int dim,
                                                    KernelParams kp, PointScale ps,
                                                    double* __restrict__ out, int ld, int* flag) {
  extern __shared__ double smem[];
  const int leaf = blockIdx.x, tid = threadIdx.x;
  const int s0 = leaf_off[leaf], n = leaf_off[leaf + 1] - s0;
  double* A = smem;
  double* fk = A + size_t(n) * n;
  for (int idx = tid; idx < n * n; idx += NT) {
    const int i = idx / n, j = idx % n;
    double r2 = 0.0;
    for (int a = 0; a < dim; ++a) {
      const double dx = pts[int64_t(s0 + i) * dim + a] - pts[int64_t(s0 + j) * dim + a];
      r2 += dx * dx;
    }
    A[idx] = near_entry(kp, ps, dim, r2, s0 + i, s0 + j, i == j);
  }
  gauss_jordan_spd(A, n, fk, flag);
  double* o = out + int64_t(leaf) * ld * ld;
  for (int idx = tid; idx < ld * ld; idx += NT) {
    const int i = idx / ld, j = idx % ld;
    o[idx] = (i < n && j < n) ? A[i * n + j] : 0.0;
  }
}

// Inverse of the diagonal block of every cluster at depth d (its projected
// close block with itself), written r x r at the cluster's gid.
__global__ __launch_bounds__(NT) void k_bj_inv_coarse(int d, const int* __restrict__ diag_blk,
                                                      const double* __restrict__ blk, int r, int T,
                                                      double* __restrict__ out, int* flag) {
  extern __shared__ double smem[];
  const int c = blockIdx.x, tid = threadIdx.x;
  double* A = smem;
  double* fk = A + size_t(r) * r;
  const double* tl = blk + int64_t(diag_blk[c]) * tile_elems(T);
  for (int idx = tid; idx < r * r; idx += NT) A[idx] = tl[tile_offset<double>(idx / r, idx % r, T)];
  gauss_jordan_spd(A, r, fk, flag);
  double* o = out + int64_t((1 << d) - 1 + c) * r * r;
  for (int idx = tid; idx < r * r; idx += NT) o[idx] = A[idx];
}

// ------------------------------------------------------------ precision copies
template <typename Td>
__global__ __launch_bounds__(NT) void k_cast_tiles(const double* __restrict__ src, Td* __restrict__ dst,
                                                   int64_t id0, int r, int T) {
  const int64_t id = id0 + blockIdx.x;
  const double* s = src + id * tile_elems(T);
  Td* d = dst + id * tile_elems(T);
  for (int idx = threadIdx.x; idx < r * r; idx += NT) {
    const int i = idx / r, j = idx % r;
    d[tile_offset<Td>(i, j, T)] = Conv<Td>::from_f64(s[tile_offset<double>(i, j, T)]);
  }
}

template <typename Td>
__global__ __launch_bounds__(NT) void k_cast_flat(const double* __restrict__ src, Td* __restrict__ dst,
                                                  int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (i < n) dst[i] = Conv<Td>::from_f64(src[i]);
}

// ------------------------------------------------------------ stored near field
// One wave per 64 x 64 tile between a row chunk and a column chunk of close
// leaves: lane (a, b) evaluates rows 8a .. 8a+7 and columns 8b .. 8b+7 of
// the tile (kernel plus the shift where a point meets itself) and writes
// them as 16-byte chunks of the T = 8 tile layout.  Entries outside the
// chunks' point counts are zero.
__global__ __launch_bounds__(NT) void k_near_tiles(int64_t nblocks, const int* __restrict__ blk_row,
                                                   const int* __restrict__ blk_col,
                                                   const int* __restrict__ chunk_start,
                                                   const int* __restrict__ chunk_n,
                                                   const double* __restrict__ pts, int dim,
                                                   KernelParams kp, PointScale ps,
                                                   double* __restrict__ tiles) {
  const int64_t blk = (int64_t(blockIdx.x) * NT + threadIdx.x) >> 6;
  if (blk >= nblocks) return;
  const int lane = threadIdx.x & 63;
  const int a = lane >> 3, b = lane & 7;
  const int cs = blk_row[blk], ct = blk_col[blk];
  const int s0 = chunk_start[cs], ns = chunk_n[cs];
  const int t0 = chunk_start[ct], nt = chunk_n[ct];
  double pi[8][3], pj[8][3];
  for (int u = 0; u < 8; ++u) {
    const int i = min(8 * a + u, ns - 1), j = min(8 * b + u, nt - 1);
    for (int q = 0; q < 3; ++q) {
      pi[u][q] = q < dim ? pts[int64_t(s0 + i) * dim + q] : 0.0;
      pj[u][q] = q < dim ? pts[int64_t(t0 + j) * dim + q] : 0.0;
    }
  }
  double* tile = tiles + blk * tile_elems(8);
#pragma unroll
  for (int c = 0; c < 32; ++c) {
    const int u = c >> 2, v0 = 2 * (c & 3);
    const int i = 8 * a + u;
    double val[2];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const int j = 8 * b + v0 + w;
      double r2 = 0.0;
      for (int q = 0; q < 3; ++q) {
        const double dx = pi[u][q] - pj[v0 + w][q];
        r2 += dx * dx;
      }
      const double k = near_entry(kp, ps, dim, r2, s0 + min(i, ns - 1), t0 + min(j, nt - 1),
                                  cs == ct && i == j);
      val[w] = (i < ns && j < nt) ? k : 0.0;
    }
    double2 out;
    out.x = val[0];
    out.y = val[1];
    *reinterpret_cast<double2*>(tile + (c * 64 + lane) * 2) = out;
  }
}

void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

// Allow dynamic LDS beyond the default limit (gfx950 has 160 KB per CU).
template <typename K>
void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

// ------------------------------------------------------------ launchers
void launch_leaf_basis_qr(H2& h) {
  const size_t lds = (size_t(h.leaf_max) * h.r + 64 + 64 + 8 + 64) * sizeof(double);
  allow_lds(k_leaf_basis_qr, lds);
  hipLaunchKernelGGL(k_leaf_basis_qr, dim3(h.nleaf), dim3(NT), lds, h.stream, h.pts, h.dim,
                     h.leaf_off, h.cbox, h.hbox, h.nodes1d, h.m, h.r, h.nleaf - 1, h.scale, h.R,
                     static_cast<double*>(h.prec[P64].Qr), static_cast<double*>(h.prec[P64].Qc));
  check_launch("leaf_basis_qr");
}

void launch_transfer_qr(H2& h, int d) {
  const size_t lds = (size_t(3) * h.r * h.r + 64 + 64 + 8 + 64) * sizeof(double);
  allow_lds(k_transfer_qr, lds);
  hipLaunchKernelGGL(k_transfer_qr, dim3(1 << d), dim3(NT), lds, h.stream, d, h.dim, h.cbox,
                     h.hbox, h.nodes1d, h.m, h.r, h.T, h.R, static_cast<double*>(h.prec[P64].E));
  check_launch("transfer_qr");
}

void launch_couplings(H2& h, int d) {
  if (h.s_count[d] == 0) return;
  const size_t lds = (size_t(2) * h.r * h.r + 64) * sizeof(double);
  hipLaunchKernelGGL(k_coupling, dim3(h.s_count[d]), dim3(NT), lds, h.stream, h.s_first[d],
                     h.blk_row, h.blk_col, h.dim, h.cbox, h.hbox, h.nodes1d, h.m, h.r, h.T, h.kp,
                     h.R, static_cast<double*>(h.prec[P64].blk));
  check_launch("coupling");
}

void launch_near_tiles(H2& h) {
  const StoredNear& sn = h.snear;
  if (sn.nblocks == 0) return;
  const int64_t groups = (sn.nblocks + 3) / 4;
  hipLaunchKernelGGL(k_near_tiles, dim3(unsigned(groups)), dim3(NT), 0, h.stream, sn.nblocks,
                     sn.blk_row, sn.blk_col, sn.chunk_start, sn.chunk_n, h.pts, h.dim, h.kp,
                     near_scale(h), sn.tiles);
  check_launch("near_tiles");
}

void launch_cast_near_tiles(H2& h) {
  StoredNear& sn = h.snear;
  if (sn.nblocks == 0) return;
  hipLaunchKernelGGL(k_cast_tiles<float>, dim3(unsigned(sn.nblocks)), dim3(NT), 0, h.stream, sn.tiles,
                     sn.tiles32, int64_t(0), 64, 8);
  check_launch("cast_near_tiles");
}

__global__ __launch_bounds__(NT) void k_gather_rows(int64_t n, int width, const int64_t* __restrict__ perm,
                                                    const double* __restrict__ user, double* __restrict__ tree) {
  const int64_t idx = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (idx >= n * width) return;
  const int64_t i = idx / width, c = idx % width;
  tree[idx] = user[perm[i] * width + c];
}

void launch_gather_rows(H2& h, int width, const double* user, double* tree) {
  const int64_t total = int64_t(h.n) * width;
  if (total == 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3(unsigned((total + NT - 1) / NT)), dim3(NT), 0, h.stream, int64_t(h.n),
                     width, h.perm, user, tree);
  check_launch("gather_rows");
}

void launch_pi_leaf(H2& h) {
  if (h.p_count[h.L] == 0) return;
  const size_t lds = (size_t(h.leaf_max) * h.r + size_t(h.leaf_max) * h.dim) * sizeof(double);
  allow_lds(k_pi_leaf, lds);
  hipLaunchKernelGGL(k_pi_leaf, dim3(h.p_count[h.L]), dim3(NT), lds, h.stream, h.p_first[h.L],
                     h.blk_row, h.blk_col, h.nleaf - 1, h.leaf_off, h.pts, h.dim, h.r, h.T, h.kp,
                     near_scale(h), static_cast<const double*>(h.prec[P64].Qr),
                     static_cast<double*>(h.prec[P64].blk));
  check_launch("pi_leaf");
}

void launch_pi_upper(H2& h, int d, const int* child_map) {
  if (h.p_count[d] == 0) return;
  const size_t lds = size_t(4) * h.r * h.r * sizeof(double);
  allow_lds(k_pi_upper, lds);
  hipLaunchKernelGGL(k_pi_upper, dim3(h.p_count[d]), dim3(NT), lds, h.stream, h.p_first[d],
                     h.blk_row, h.blk_col, child_map, h.r, h.T,
                     static_cast<const double*>(h.prec[P64].E), static_cast<double*>(h.prec[P64].blk));
  check_launch("pi_upper");
}

void launch_assemble_dense(H2& h, double* A, int64_t lda) {
  const int d = h.d_top;
  const int gid0 = (1 << d) - 1;
  if (h.s_count[d])
    hipLaunchKernelGGL(k_assemble_dense, dim3(h.s_count[d]), dim3(NT), 0, h.stream, h.s_first[d],
                       h.blk_row, h.blk_col, gid0, h.r, h.T,
                       static_cast<const double*>(h.prec[P64].blk), A, lda);
  if (h.p_count[d])
    hipLaunchKernelGGL(k_assemble_dense, dim3(h.p_count[d]), dim3(NT), 0, h.stream, h.p_first[d],
                       h.blk_row, h.blk_col, gid0, h.r, h.T,
                       static_cast<const double*>(h.prec[P64].blk), A, lda);
  check_launch("assemble_dense");
}

void launch_assemble_kernel_dense(H2& h, double* A, int64_t lda) {
  const int64_t nn = int64_t(h.n) * h.n;
  hipLaunchKernelGGL(k_assemble_kernel_dense, dim3((nn + NT - 1) / NT), dim3(NT), 0, h.stream,
                     h.pts, h.dim, int64_t(h.n), h.kp, near_scale(h), A);
  (void)lda;
  check_launch("assemble_kernel_dense");
}

void launch_potrf(H2& h, double* A, int64_t N) {
  for (int64_t k0 = 0; k0 < N; k0 += NB) {
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(NT), 0, h.stream, A, N, k0, h.flags);
    const int64_t below = N - k0 - std::min<int64_t>(NB, N - k0);
    if (below > 0) {
      const int nrb = int((below + NB - 1) / NB);
      hipLaunchKernelGGL(k_trsm_panel, dim3(nrb), dim3(NB), 0, h.stream, A, N, k0, h.flags);
      const int npairs = nrb * (nrb + 1) / 2;
      hipLaunchKernelGGL(k_syrk_update, dim3(npairs), dim3(NT), 0, h.stream, A, N, k0, nrb,
                         h.flags);
    }
  }
  check_launch("potrf");
}

void launch_bj_inverse_fine(H2& h, double* out, int ld) {
  const int n = h.leaf_max;
  const size_t lds = (size_t(n) * n + n) * sizeof(double);
  allow_lds(k_bj_inv_fine, lds);
  hipLaunchKernelGGL(k_bj_inv_fine, dim3(h.nleaf), dim3(NT), lds, h.stream, h.leaf_off, h.pts,
                     h.dim, h.kp, near_scale(h), out, ld, h.flags);
  check_launch("bj_inv_fine");
}

void launch_bj_inverse_coarse(H2& h, int d, const int* diag_blk, double* out) {
  const size_t lds = (size_t(h.r) * h.r + h.r) * sizeof(double);
  hipLaunchKernelGGL(k_bj_inv_coarse, dim3(1 << d), dim3(NT), lds, h.stream, d, diag_blk,
                     static_cast<const double*>(h.prec[P64].blk), h.r, h.T, out, h.flags);
  check_launch("bj_inv_coarse");
}

void launch_cast_precision(H2& h, int p) {
  const int64_t te = tile_elems(h.T);
  const double* blk = static_cast<const double*>(h.prec[P64].blk);
  const double* E = static_cast<const double*>(h.prec[P64].E);
  const int64_t nQ = int64_t(h.n) * h.r;
  const int64_t gidE0 = (int64_t(1) << (h.d_top + 1)) - 1;   // first gid with a transfer
  if (p == P32) {
    float* dblk = static_cast<float*>(h.prec[p].blk);
    float* dE = static_cast<float*>(h.prec[p].E);
    if (h.nblk) hipLaunchKernelGGL(k_cast_tiles<float>, dim3(h.nblk), dim3(NT), 0, h.stream, blk, dblk, int64_t(0), h.r, h.T);
    if (h.ngid > gidE0) hipLaunchKernelGGL(k_cast_tiles<float>, dim3(h.ngid - gidE0), dim3(NT), 0, h.stream, E, dE, gidE0, h.r, h.T);
    hipLaunchKernelGGL(k_cast_flat<float>, dim3((nQ + NT - 1) / NT), dim3(NT), 0, h.stream,
                       static_cast<const double*>(h.prec[P64].Qr), static_cast<float*>(h.prec[p].Qr), nQ);
    hipLaunchKernelGGL(k_cast_flat<float>, dim3((nQ + NT - 1) / NT), dim3(NT), 0, h.stream,
                       static_cast<const double*>(h.prec[P64].Qc), static_cast<float*>(h.prec[p].Qc), nQ);
  } else {
    bf16* dblk = static_cast<bf16*>(h.prec[p].blk);
    bf16* dE = static_cast<bf16*>(h.prec[p].E);
    if (h.nblk) hipLaunchKernelGGL(k_cast_tiles<bf16>, dim3(h.nblk), dim3(NT), 0, h.stream, blk, dblk, int64_t(0), h.r, h.T);
    if (h.ngid > gidE0) hipLaunchKernelGGL(k_cast_tiles<bf16>, dim3(h.ngid - gidE0), dim3(NT), 0, h.stream, E, dE, gidE0, h.r, h.T);
    hipLaunchKernelGGL(k_cast_flat<bf16>, dim3((nQ + NT - 1) / NT), dim3(NT), 0, h.stream,
                       static_cast<const double*>(h.prec[P64].Qr), static_cast<bf16*>(h.prec[p].Qr), nQ);
    hipLaunchKernelGGL(k_cast_flat<bf16>, dim3((nQ + NT - 1) / NT), dim3(NT), 0, h.stream,
                       static_cast<const double*>(h.prec[P64].Qc), static_cast<bf16*>(h.prec[p].Qc), nQ);
  }
  check_launch("cast_precision");
}

}  // namespace h2mg
