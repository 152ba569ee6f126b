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
#include <type_traits>

#include "h2_impl.h"

namespace h2mg {

namespace {

constexpr int NT = 256;   // threads per workgroup of the setup kernels

typedef double d4 __attribute__((ext_vector_type(4)));

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

// ------------------------------------------------------------ Galerkin products
// Couplings, projected close leaf blocks and projected upper blocks are all
//   out[mu][nu] = sum_i sum_j QS(i, mu) K(i, j) QT(j, nu)       (r x r)
// for an inner matrix K and two thin factors:
//   * coupling of a far pair (s, t): K = k(xi_s, xi_t) on the Chebyshev nodes,
//     QS(i, mu) = R_s[mu][i], QT(j, nu) = R_t[nu][j]  (out = R_s K R_t^T);
//   * close leaf pair: K = the kernel entries of the two leaves (shift on a
//     diagonal pair's diagonal), QS = Q_s, QT = Q_t (out = Q_s^T K Q_t);
//   * close pair above the leaves: K = the 2 x 2 arrangement of the stored
//     child blocks M_cc' (i = child a * RM + row, j likewise), QS and QT the
//     stacked child transfers [E_c1; E_c2] (out = sum E_c^T M_cc' E_c').
// One wave per output tile, on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; result element t of lane l is D[4 t + l / 16][l % 16]).
// The rows i are taken 16 at a time: W = K[i0 : i0 + 16, :] QT is formed in
// RS accumulators (RS = RM / 16 column slabs of 16, RM = max(16, 8T)), the
// kernel entries computed (or loaded) by the lane that supplies them, and
// then folded into out += QS[i0 : i0 + 16, :]^T W; a W accumulator holds,
// in element t, exactly the B operand of the fold's k-step t, so the fold
// needs no data movement.  Entries outside the matrices (i, j beyond the
// point or node count, mu, nu >= r) are zero.
template <int RS, typename Acc>
__device__ __forceinline__ void galerkin_wave(const Acc& acc, int ni, int nj, d4 (&out)[RS][RS]) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int a = 0; a < RS; ++a)
#pragma unroll
    for (int b = 0; b < RS; ++b) out[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  for (int i0 = 0; i0 < ni; i0 += 16) {
    const auto row = acc.row(i0 + li);
    d4 w[RS];
#pragma unroll
    for (int c = 0; c < RS; ++c) w[c] = d4{0.0, 0.0, 0.0, 0.0};
    // operands of k-step j0 + 4 are fetched (and K evaluated) while the
    // matrix cores run k-step j0
    double a = acc.k(row, i0 + li, lk), q[RS];
#pragma unroll
    for (int c = 0; c < RS; ++c) q[c] = acc.qt(lk, c * 16 + li);
    for (int j0 = 0; j0 < nj; j0 += 4) {
      const int jn = j0 + 4 + lk;
      const bool more = j0 + 4 < nj;
      const double an = more ? acc.k(row, i0 + li, jn) : 0.0;
      double qn[RS];
#pragma unroll
      for (int c = 0; c < RS; ++c) qn[c] = more ? acc.qt(jn, c * 16 + li) : 0.0;
#pragma unroll
      for (int c = 0; c < RS; ++c) w[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, q[c], w[c], 0, 0, 0);
      a = an;
#pragma unroll
      for (int c = 0; c < RS; ++c) q[c] = qn[c];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = i0 + 4 * t + lk;
#pragma unroll
      for (int mu = 0; mu < RS; ++mu) {
        const double q = acc.qs(i, mu * 16 + li);
#pragma unroll
        for (int nu = 0; nu < RS; ++nu)
          out[mu][nu] = __builtin_amdgcn_mfma_f64_16x16x4f64(q, w[nu][t], out[mu][nu], 0, 0, 0);
      }
    }
  }
}

template <int RS>
__device__ __forceinline__ void store_galerkin(const d4 (&out)[RS][RS], int r, int T, double* tile) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int mu = 0; mu < RS; ++mu)
#pragma unroll
    for (int nu = 0; nu < RS; ++nu)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = mu * 16 + 4 * t + lk, j = nu * 16 + li;
        if (i < r && j < r) tile[tile_offset<double>(i, j, T)] = out[mu][nu][t];
      }
}

__device__ inline int wave_id() {
  return __builtin_amdgcn_readfirstlane(int((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
}

// Couplings of a far pair: K on the two node sets, QS / QT from the R factors
// of the direct bases (row-major r x r, upper triangular).
struct CouplingAcc {
  const double* cs; const double* hs; const double* ct; const double* ht;
  const double* tn; const double* Rs; const double* Rt;
  KernelParams kp; int m, dim, r;
  struct Row { double x[3]; };
  __device__ __forceinline__ Row row(int i) const {
    Row p{{0.0, 0.0, 0.0}};
    if (i < r) {
      int nu = i;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        if (a < dim) {
          p.x[a] = cs[a] + hs[a] * tn[nu % m];
          nu /= m;
        }
    }
    return p;
  }
  __device__ __forceinline__ double k(const Row& p, int i, int j) const {
    if (i >= r || j >= r) return 0.0;
    double r2 = 0.0;
    int nu = j;
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (a < dim) {
        const double dx = p.x[a] - (ct[a] + ht[a] * tn[nu % m]);
        nu /= m;
        r2 += dx * dx;
      }
    return kernel_r2(kp, r2);
  }
  __device__ __forceinline__ double qs(int i, int mu) const { return i < r && mu < r ? Rs[size_t(mu) * r + i] : 0.0; }
  __device__ __forceinline__ double qt(int j, int nu) const { return j < r && nu < r ? Rt[size_t(nu) * r + j] : 0.0; }
};

template <int RS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_coupling(
    int b0, int nb, const int* __restrict__ blk_row, const int* __restrict__ blk_col, int dim,
    const double* __restrict__ cbox, const double* __restrict__ hbox,
    const double* __restrict__ nodes, int m, int r, int T, KernelParams kp,
    const double* __restrict__ Rall, double* __restrict__ blk) {
  const int w = wave_id();
  if (w >= nb) return;
  const int b = b0 + w;
  const int gs = blk_row[b], gt = blk_col[b];
  const CouplingAcc acc{cbox + size_t(gs) * dim, hbox + size_t(gs) * dim, cbox + size_t(gt) * dim,
                        hbox + size_t(gt) * dim, nodes, Rall + size_t(gs) * r * r,
                        Rall + size_t(gt) * r * r, kp, m, dim, r};
  d4 out[RS][RS];
  galerkin_wave<RS>(acc, (r + 15) & ~15, (r + 3) & ~3, out);
  store_galerkin<RS>(out, r, T, tile_ptr(blk, b, T));
}

// Projected close leaf blocks: K = the kernel (shift on the diagonal of a
// diagonal pair), QS / QT the orthonormal leaf bases (row-major, per point).
// KIND >= 0: the kernel fixed at compile time (point values, no derivative);
// KIND < 0: the general close entry (derivative kernels, quadrature).
template <int KIND>
struct LeafAcc {
  const double* pts; const double* Qr;
  KernelParams kp; PointScale ps;
  int s0, ns, t0, nt, dim, r;
  bool diag;
  struct Row { double x[3]; };
  __device__ __forceinline__ Row row(int i) const {
    Row p{{0.0, 0.0, 0.0}};
    if (i < ns) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
        if (a < dim) p.x[a] = pts[size_t(s0 + i) * dim + a];
    }
    return p;
  }
  __device__ __forceinline__ double k(const Row& p, int i, int j) const {
    if (i >= ns || j >= nt) return 0.0;
    double r2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (a < dim) {
        const double dx = p.x[a] - pts[size_t(t0 + j) * dim + a];
        r2 += dx * dx;
      }
    const bool self = diag && i == j;
    if constexpr (KIND >= 0)
      return scaled_entry(kernel_fixed<KIND, DER_NONE, double>(kp.inv_l, kp.inv_2l2, r2), s0 + i, t0 + j,
                          self, ps, kp.shift);
    else
      return near_entry(kp, ps, dim, r2, s0 + i, t0 + j, self);
  }
  __device__ __forceinline__ double qs(int i, int mu) const { return i < ns && mu < r ? Qr[size_t(s0 + i) * r + mu] : 0.0; }
  __device__ __forceinline__ double qt(int j, int nu) const { return j < nt && nu < r ? Qr[size_t(t0 + j) * r + nu] : 0.0; }
};

template <int RS, int KIND>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_pi_leaf(
    int b0, int nb, const int* __restrict__ blk_row, const int* __restrict__ blk_col, int gid0,
    const int* __restrict__ leaf_off, const double* __restrict__ pts, int dim, int r, int T,
    KernelParams kp, PointScale ps, const double* __restrict__ Qr, double* __restrict__ blk) {
  const int w = wave_id();
  if (w >= nb) return;
  const int b = b0 + w;
  const int ls = blk_row[b] - gid0, lt = blk_col[b] - gid0;
  const int s0 = leaf_off[ls], t0 = leaf_off[lt];
  const LeafAcc<KIND> acc{pts, Qr, kp, ps, s0, leaf_off[ls + 1] - s0, t0, leaf_off[lt + 1] - t0, dim, r,
                          ls == lt};
  d4 out[RS][RS];
  galerkin_wave<RS>(acc, (acc.ns + 15) & ~15, (acc.nt + 3) & ~3, out);
  store_galerkin<RS>(out, r, T, tile_ptr(blk, b, T));
}

// Projected blocks above the leaves: K = [M_11 M_12; M_21 M_22] over the
// child pairs (a stored child block, transposed when the child pair is below
// the diagonal: child_map entry -id - 1), rows and columns of child a at
// a * RM; QS / QT the children's transfer tiles.
struct UpperAcc {
  const double* blk; const double* E;
  const int* map;            // the four child block ids (negative: transposed)
  int gcs0, gct0, r, T, RM;
  struct Row { int id0, id1; };
  __device__ __forceinline__ Row row(int i) const {
    const int a = i >= RM;
    return Row{map[2 * a], map[2 * a + 1]};
  }
  __device__ __forceinline__ double k(const Row& p, int i, int j) const {
    const int a = i >= RM, b = j >= RM;
    const int ii = i - a * RM, jj = j - b * RM;
    if (ii >= r || jj >= r) return 0.0;
    const int id = b ? p.id1 : p.id0;
    return id >= 0 ? blk[int64_t(id) * tile_elems(T) + tile_offset<double>(ii, jj, T)]
                   : blk[int64_t(-id - 1) * tile_elems(T) + tile_offset<double>(jj, ii, T)];
  }
  __device__ __forceinline__ double qs(int i, int mu) const {
    const int a = i >= RM, ii = i - a * RM;
    return ii < r && mu < r ? E[int64_t(gcs0 + a) * tile_elems(T) + tile_offset<double>(ii, mu, T)] : 0.0;
  }
  __device__ __forceinline__ double qt(int j, int nu) const {
    const int b = j >= RM, jj = j - b * RM;
    return jj < r && nu < r ? E[int64_t(gct0 + b) * tile_elems(T) + tile_offset<double>(jj, nu, T)] : 0.0;
  }
};

template <int RS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_pi_upper(
    int b0, int nb, const int* __restrict__ blk_row, const int* __restrict__ blk_col,
    const int* __restrict__ child_map, int r, int T, const double* __restrict__ E,
    double* __restrict__ blk) {
  const int w = wave_id();
  if (w >= nb) return;
  const int b = b0 + w;
  constexpr int RM = RS * 16;
  const UpperAcc acc{blk, E, child_map + 4 * w,
               2 * blk_row[b] + 1, 2 * blk_col[b] + 1, r, T, RM};
  d4 out[RS][RS];
  galerkin_wave<RS>(acc, 2 * RM, 2 * RM, out);
  store_galerkin<RS>(out, r, T, tile_ptr(blk, b, T));
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

// The Galerkin kernels take RS = 16-column slabs of the padded rank.
template <typename F>
void with_slabs(int T, F&& f) {
  if (T <= 2) f(std::integral_constant<int, 1>{});
  else if (T == 4) f(std::integral_constant<int, 2>{});
  else f(std::integral_constant<int, 4>{});
}

inline dim3 wave_grid(int nb) { return dim3(unsigned((nb + NT / 64 - 1) / (NT / 64))); }

void launch_couplings(H2& h, int d) {
  if (h.s_count[d] == 0) return;
  with_slabs(h.T, [&](auto rs) {
    constexpr int RS = decltype(rs)::value;
    hipLaunchKernelGGL(k_coupling<RS>, wave_grid(h.s_count[d]), dim3(NT), 0, h.stream, h.s_first[d],
                       h.s_count[d], h.blk_row, h.blk_col, h.dim, h.cbox, h.hbox, h.nodes1d, h.m, h.r,
                       h.T, h.kp, h.R, static_cast<double*>(h.prec[P64].blk));
  });
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
  const int nb = h.p_count[h.L];
  if (nb == 0) return;
  const PointScale ps = near_scale(h);
  auto go = [&](auto rs, auto kc) {
    constexpr int RS = decltype(rs)::value, KIND = decltype(kc)::value;
    hipLaunchKernelGGL((k_pi_leaf<RS, KIND>), wave_grid(nb), dim3(NT), 0, h.stream, h.p_first[h.L], nb,
                       h.blk_row, h.blk_col, h.nleaf - 1, h.leaf_off, h.pts, h.dim, h.r, h.T, h.kp, ps,
                       static_cast<const double*>(h.prec[P64].Qr), static_cast<double*>(h.prec[P64].blk));
  };
  with_slabs(h.T, [&](auto rs) {
    using I = int;
    if (ps.qy || h.kp.deriv != DER_NONE) go(rs, std::integral_constant<I, -1>{});
    else dispatch_kernel(h.kp.kind, DER_NONE, [&](auto kc, auto) { go(rs, kc); });
  });
  check_launch("pi_leaf");
}

void launch_pi_upper(H2& h, int d, const int* child_map) {
  const int nb = h.p_count[d];
  if (nb == 0) return;
  with_slabs(h.T, [&](auto rs) {
    constexpr int RS = decltype(rs)::value;
    hipLaunchKernelGGL(k_pi_upper<RS>, wave_grid(nb), dim3(NT), 0, h.stream, h.p_first[d], nb,
                       h.blk_row, h.blk_col, child_map, h.r, h.T,
                       static_cast<const double*>(h.prec[P64].E), static_cast<double*>(h.prec[P64].blk));
  });
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
