// Vector kernels of the V-cycle: permutations, axpby, FP64-accumulated dot
// products, the two halves of a CG step with device-resident scalars, and
// the triangular solves with the Cholesky factor of the coarsest operator.
//
// Section 3.3: the smoother Iter(A, r, e0) is CG, and the coarsest level is
// solved directly with a Cholesky factorisation.  Dot products are reduced
// in two fixed-order stages (per-workgroup partials, then a one-wave sum in
// the consumer) so results are deterministic and no host round trip is
// needed between CG steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>
#include <string>

#include "h2_impl.h"

namespace h2mg {

namespace {

constexpr int NT = 256;
constexpr int MAX_PARTS = 512;

void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

__device__ double block_sum(double v) {
  __shared__ double red[NT / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

// Sum of np partials in a fixed order, computed by wave 0 and broadcast.
__device__ double sum_parts(const double* part, int np) {
  __shared__ double bc;
  __syncthreads();
  if (threadIdx.x < 64) {
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += 64) s += part[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x == 0) bc = s;
  }
  __syncthreads();
  return bc;
}

__global__ __launch_bounds__(NT) void k_gather(int64_t n, const int64_t* __restrict__ perm,
                                               const double* __restrict__ user,
                                               double* __restrict__ tree) {
  const int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (i < n) tree[i] = user[perm[i]];
}

__global__ __launch_bounds__(NT) void k_scatter(int64_t n, const int64_t* __restrict__ perm,
                                                const double* __restrict__ tree,
                                                double* __restrict__ user) {
  const int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (i < n) user[perm[i]] = tree[i];
}

template <typename Td, typename Ts>
__global__ __launch_bounds__(NT) void k_cast(int64_t n, const Ts* __restrict__ s, Td* __restrict__ d) {
  const int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (i < n) d[i] = Td(s[i]);
}

template <typename Tv>
__global__ __launch_bounds__(NT) void k_axpby(int64_t n, double a, const Tv* __restrict__ x,
                                              double b, Tv* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (i < n) y[i] = Tv(a) * x[i] + (b == 0.0 ? Tv(0) : Tv(b) * y[i]);
}

// y = x and y = 0 as kernels (no memset or memcpy nodes when a cycle is
// captured into a graph).
template <typename Tv>
__global__ __launch_bounds__(NT) void k_copy(int64_t n, const Tv* __restrict__ x, Tv* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (i < n) y[i] = x[i];
}

template <typename Tv>
__global__ __launch_bounds__(NT) void k_zero(int64_t n, Tv* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (i < n) y[i] = Tv(0);
}

// ---------------------------------------------------------------- gradient helpers
// user[perm[i]] = tree[i] for rows of dim coordinates.
__global__ __launch_bounds__(NT) void k_scatter_rows(int64_t n, int dim, const int64_t* __restrict__ perm,
                                                     const double* __restrict__ tree,
                                                     double* __restrict__ user) {
  const int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (i < n)
    for (int a = 0; a < dim; ++a) user[perm[i] * dim + a] = tree[i * dim + a];
}

// w_i = x_i * p_{i,a} (tree order).
__global__ __launch_bounds__(NT) void k_coord_mul(int64_t n, int dim, int a, const double* __restrict__ x,
                                                  const double* __restrict__ pts, double* __restrict__ w) {
  const int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (i < n) w[i] = x[i] * pts[i * dim + a];
}

// grad[perm[i], a] = -2 scale x_i (p_{i,a} v_i - u_i), v = G x, u = G (x * p_.a).
__global__ __launch_bounds__(NT) void k_coord_grad(int64_t n, int dim, int a, double scale,
                                                   const int64_t* __restrict__ perm,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ pts,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ u,
                                                   double* __restrict__ grad) {
  const int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (i < n) grad[perm[i] * dim + a] = -2.0 * scale * x[i] * (pts[i * dim + a] * v[i] - u[i]);
}

template <typename Tv>
__global__ __launch_bounds__(NT) void k_dot(int64_t n, const Tv* __restrict__ x,
                                            const Tv* __restrict__ y, double* __restrict__ part) {
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT)
    acc += double(x[i]) * double(y[i]);
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// alpha = gamma / delta; e += alpha p; s -= alpha q; partials of s.s.
// gamma == 0 (exact convergence) gives alpha = 0; delta <= 0 with gamma > 0
// flags a non-SPD operator and freezes the iterate.
template <typename Tv>
__global__ __launch_bounds__(NT) void k_cg_update(int64_t n, Tv* __restrict__ e,
                                                  const Tv* __restrict__ p, Tv* __restrict__ s,
                                                  const Tv* __restrict__ q,
                                                  const double* __restrict__ gpart,
                                                  const double* __restrict__ dpart, int np,
                                                  double* __restrict__ gnew, int* __restrict__ flag) {
  const double gamma = sum_parts(gpart, np);
  const double delta = sum_parts(dpart, np);
  double alpha = 0.0;
  if (gamma != 0.0) {
    if (delta > 0.0) {
      alpha = gamma / delta;
    } else if (blockIdx.x == 0 && threadIdx.x == 0) {
      atomicOr(flag, 1);
    }
  }
  double acc = 0.0;
  const Tv al = Tv(alpha);
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT) {
    e[i] += al * p[i];
    const Tv sn = s[i] - al * q[i];
    s[i] = sn;
    acc += double(sn) * double(sn);
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) gnew[blockIdx.x] = t;
}

// beta = gamma_new / gamma_old; p = s + beta p.
template <typename Tv>
__global__ __launch_bounds__(NT) void k_cg_pupdate(int64_t n, Tv* __restrict__ p,
                                                   const Tv* __restrict__ s,
                                                   const double* __restrict__ gold,
                                                   const double* __restrict__ gnew, int np) {
  const double go = sum_parts(gold, np);
  const double gn = sum_parts(gnew, np);
  const Tv beta = Tv(go == 0.0 ? 0.0 : gn / go);
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT)
    p[i] = s[i] + beta * p[i];
}

template <typename Tv>
__global__ __launch_bounds__(NT) void k_check_finite(int64_t n, const Tv* __restrict__ x,
                                                     int* __restrict__ flag) {
  const int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (i < n && !isfinite(double(x[i]))) atomicOr(flag, 1);
}

// z_b = M_b^{-1} s_b for every diagonal block b (one workgroup per block):
// rows [off[b], off[b+1]) when off is given, else [b*stride, (b+1)*stride).
// The stored inverses are symmetric, so thread i reads column i of block b,
// coalesced across threads.
template <typename Tm, typename Tv>
__global__ __launch_bounds__(NT) void k_bj_apply(const int* __restrict__ off, int stride,
                                                 const Tm* __restrict__ Minv, int ld,
                                                 const Tv* __restrict__ s, Tv* __restrict__ z) {
  __shared__ Tv sl[256];
  const int b = blockIdx.x;
  const int s0 = off ? off[b] : b * stride;
  const int n = off ? off[b + 1] - s0 : stride;
  for (int i = threadIdx.x; i < n; i += NT) sl[i] = s[s0 + i];
  __syncthreads();
  const Tm* M = Minv + int64_t(b) * ld * ld;
  for (int i = threadIdx.x; i < n; i += NT) {
    Tv acc = Tv(0);
    for (int j = 0; j < n; ++j) acc += Tv(M[int64_t(j) * ld + i]) * sl[j];
    z[s0 + i] = acc;
  }
}

// ------------------------------------------------------------ triangular solves
constexpr int NB = 64;

// x_k = L_kk^{-1} x_k (one wave).
__global__ __launch_bounds__(64) void k_trsv_fwd_diag(const double* __restrict__ L, int64_t N,
                                                      int64_t k0, double* __restrict__ x) {
  __shared__ double D[NB][NB + 1];
  const int nb = int(min<int64_t>(NB, N - k0));
  const int i = threadIdx.x;
  for (int idx = i; idx < nb * nb; idx += 64) D[idx % nb][idx / nb] = L[(k0 + idx % nb) + (k0 + idx / nb) * N];
  __syncthreads();
  double xi = i < nb ? x[k0 + i] : 0.0;
  for (int c = 0; c < nb; ++c) {
    const double xc = __shfl(xi, c, 64) / D[c][c];
    if (i == c) xi = xc;
    else if (i > c) xi -= D[i][c] * xc;
  }
  if (i < nb) x[k0 + i] = xi;
}

// x_i -= L_ik x_k for rows below block k.
__global__ __launch_bounds__(NT) void k_gemv_fwd(const double* __restrict__ L, int64_t N, int64_t k0,
                                                 double* __restrict__ x) {
  __shared__ double xk[NB];
  const int nb = int(min<int64_t>(NB, N - k0));
  if (threadIdx.x < nb) xk[threadIdx.x] = x[k0 + threadIdx.x];
  __syncthreads();
  const int64_t row = k0 + nb + int64_t(blockIdx.x) * NT + threadIdx.x;
  if (row >= N) return;
  double s = 0.0;
  for (int c = 0; c < nb; ++c) s += L[row + (k0 + c) * N] * xk[c];
  x[row] -= s;
}

// x_k = L_kk^{-T} x_k (one wave).
__global__ __launch_bounds__(64) void k_trsv_bwd_diag(const double* __restrict__ L, int64_t N,
                                                      int64_t k0, double* __restrict__ x) {
  __shared__ double D[NB][NB + 1];
  const int nb = int(min<int64_t>(NB, N - k0));
  const int i = threadIdx.x;
  for (int idx = i; idx < nb * nb; idx += 64) D[idx % nb][idx / nb] = L[(k0 + idx % nb) + (k0 + idx / nb) * N];
  __syncthreads();
  double xi = i < nb ? x[k0 + i] : 0.0;
  for (int c = nb - 1; c >= 0; --c) {
    const double xc = __shfl(xi, c, 64) / D[c][c];
    if (i == c) xi = xc;
    else if (i < c) xi -= D[c][i] * xc;
  }
  if (i < nb) x[k0 + i] = xi;
}

// x_j -= sum_i L[k0 + i][j] x_{k0 + i} for rows j above block k.
__global__ __launch_bounds__(NT) void k_gemv_bwd(const double* __restrict__ L, int64_t N, int64_t k0,
                                                 double* __restrict__ x) {
  __shared__ double xk[NB];
  const int nb = int(min<int64_t>(NB, N - k0));
  if (threadIdx.x < nb) xk[threadIdx.x] = x[k0 + threadIdx.x];
  __syncthreads();
  const int64_t j = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (j >= k0) return;
  double s = 0.0;
  const double* col = L + j * N + k0;
  for (int i = 0; i < nb; ++i) s += col[i] * xk[i];
  x[j] -= s;
}

inline unsigned blocks(int64_t n) { return unsigned((n + NT - 1) / NT); }

}  // namespace

int dot_parts(int64_t n) {
  return int(std::max<int64_t>(1, std::min<int64_t>(MAX_PARTS, (n + 4095) / 4096)));
}

void launch_gather(H2& h, const double* user, double* tree) {
  hipLaunchKernelGGL(k_gather, dim3(blocks(h.n)), dim3(NT), 0, h.stream, int64_t(h.n), h.perm, user, tree);
  check_launch("gather");
}

void launch_scatter(H2& h, const double* tree, double* user) {
  hipLaunchKernelGGL(k_scatter, dim3(blocks(h.n)), dim3(NT), 0, h.stream, int64_t(h.n), h.perm, tree, user);
  check_launch("scatter");
}

void launch_copy(H2& h, int p, const void* src, void* dst, int64_t n) {
  if (n <= 0) return;
  if (p == P64)
    hipLaunchKernelGGL(k_copy<double>, dim3(blocks(n)), dim3(NT), 0, h.stream, n,
                       static_cast<const double*>(src), static_cast<double*>(dst));
  else
    hipLaunchKernelGGL(k_copy<float>, dim3(blocks(n)), dim3(NT), 0, h.stream, n,
                       static_cast<const float*>(src), static_cast<float*>(dst));
  check_launch("copy");
}

void launch_zero(H2& h, int p, void* dst, int64_t n) {
  if (n <= 0) return;
  if (p == P64)
    hipLaunchKernelGGL(k_zero<double>, dim3(blocks(n)), dim3(NT), 0, h.stream, n, static_cast<double*>(dst));
  else
    hipLaunchKernelGGL(k_zero<float>, dim3(blocks(n)), dim3(NT), 0, h.stream, n, static_cast<float*>(dst));
  check_launch("zero");
}

void launch_cast(H2& h, int pdst, void* dst, int psrc, const void* src, int64_t n) {
  const bool d64 = pdst == P64, s64 = psrc == P64;
  if (d64 == s64) { launch_copy(h, pdst, src, dst, n); return; }
  if (d64)
    hipLaunchKernelGGL((k_cast<double, float>), dim3(blocks(n)), dim3(NT), 0, h.stream, n,
                       static_cast<const float*>(src), static_cast<double*>(dst));
  else
    hipLaunchKernelGGL((k_cast<float, double>), dim3(blocks(n)), dim3(NT), 0, h.stream, n,
                       static_cast<const double*>(src), static_cast<float*>(dst));
  check_launch("cast");
}

void launch_axpby(H2& h, int p, int64_t n, double a, const void* x, double b, void* y) {
  if (p == P64)
    hipLaunchKernelGGL(k_axpby<double>, dim3(blocks(n)), dim3(NT), 0, h.stream, n, a,
                       static_cast<const double*>(x), b, static_cast<double*>(y));
  else
    hipLaunchKernelGGL(k_axpby<float>, dim3(blocks(n)), dim3(NT), 0, h.stream, n, a,
                       static_cast<const float*>(x), b, static_cast<float*>(y));
  check_launch("axpby");
}

void launch_dot(H2& h, int p, int64_t n, const void* x, const void* y, double* part) {
  const int np = dot_parts(n);
  if (p == P64)
    hipLaunchKernelGGL(k_dot<double>, dim3(np), dim3(NT), 0, h.stream, n,
                       static_cast<const double*>(x), static_cast<const double*>(y), part);
  else
    hipLaunchKernelGGL(k_dot<float>, dim3(np), dim3(NT), 0, h.stream, n,
                       static_cast<const float*>(x), static_cast<const float*>(y), part);
  check_launch("dot");
}

void launch_cg_update(H2& h, int p, int64_t n, void* e, const void* pv, void* s, const void* q,
                      const double* gamma_part, const double* delta_part, double* gamma_new_part) {
  const int np = dot_parts(n);
  if (p == P64)
    hipLaunchKernelGGL(k_cg_update<double>, dim3(np), dim3(NT), 0, h.stream, n,
                       static_cast<double*>(e), static_cast<const double*>(pv),
                       static_cast<double*>(s), static_cast<const double*>(q), gamma_part,
                       delta_part, np, gamma_new_part, h.flags);
  else
    hipLaunchKernelGGL(k_cg_update<float>, dim3(np), dim3(NT), 0, h.stream, n,
                       static_cast<float*>(e), static_cast<const float*>(pv),
                       static_cast<float*>(s), static_cast<const float*>(q), gamma_part,
                       delta_part, np, gamma_new_part, h.flags);
  check_launch("cg_update");
}

void launch_cg_pupdate(H2& h, int p, int64_t n, void* pv, const void* s,
                       const double* gamma_old_part, const double* gamma_new_part) {
  const int np = dot_parts(n);
  if (p == P64)
    hipLaunchKernelGGL(k_cg_pupdate<double>, dim3(np), dim3(NT), 0, h.stream, n,
                       static_cast<double*>(pv), static_cast<const double*>(s), gamma_old_part,
                       gamma_new_part, np);
  else
    hipLaunchKernelGGL(k_cg_pupdate<float>, dim3(np), dim3(NT), 0, h.stream, n,
                       static_cast<float*>(pv), static_cast<const float*>(s), gamma_old_part,
                       gamma_new_part, np);
  check_launch("cg_pupdate");
}

void launch_chol_solve(H2& h, const double* L, int64_t N, double* x) {
  for (int64_t k0 = 0; k0 < N; k0 += NB) {
    hipLaunchKernelGGL(k_trsv_fwd_diag, dim3(1), dim3(64), 0, h.stream, L, N, k0, x);
    const int64_t below = N - k0 - std::min<int64_t>(NB, N - k0);
    if (below > 0)
      hipLaunchKernelGGL(k_gemv_fwd, dim3(blocks(below)), dim3(NT), 0, h.stream, L, N, k0, x);
  }
  const int64_t last = ((N - 1) / NB) * NB;
  for (int64_t k0 = last; k0 >= 0; k0 -= NB) {
    hipLaunchKernelGGL(k_trsv_bwd_diag, dim3(1), dim3(64), 0, h.stream, L, N, k0, x);
    if (k0 > 0)
      hipLaunchKernelGGL(k_gemv_bwd, dim3(blocks(k0)), dim3(NT), 0, h.stream, L, N, k0, x);
  }
  check_launch("chol_solve");
}

void launch_bj_apply(H2& h, int p, int k, const void* s, void* z) {
  const bool fine = k == 1;
  const int d = h.level_depth(k);
  const int nb = fine ? h.nleaf : (1 << d);
  const int* off = fine ? h.leaf_off : nullptr;
  const int ld = fine ? h.bj_ld : h.r;
  const int stride = h.r;
  const size_t eb = p == P64 ? 8 : 4;
  const char* base = static_cast<const char*>(fine ? h.bj_fine[p == P64 ? P64 : P32]
                                                   : h.bj_coarse[p == P64 ? P64 : P32]);
  if (!fine) base += size_t((1 << d) - 1) * h.r * h.r * eb;
  if (p == P64)
    hipLaunchKernelGGL((k_bj_apply<double, double>), dim3(nb), dim3(NT), 0, h.stream, off, stride,
                       reinterpret_cast<const double*>(base), ld, static_cast<const double*>(s),
                       static_cast<double*>(z));
  else
    hipLaunchKernelGGL((k_bj_apply<float, float>), dim3(nb), dim3(NT), 0, h.stream, off, stride,
                       reinterpret_cast<const float*>(base), ld, static_cast<const float*>(s),
                       static_cast<float*>(z));
  check_launch("bj_apply");
}

void launch_scatter_rows(H2& h, const double* tree, double* user) {
  hipLaunchKernelGGL(k_scatter_rows, dim3(blocks(h.n)), dim3(NT), 0, h.stream, int64_t(h.n), h.dim,
                     h.perm, tree, user);
  check_launch("scatter_rows");
}

void launch_coord_mul(H2& h, int a, const double* x, double* w) {
  hipLaunchKernelGGL(k_coord_mul, dim3(blocks(h.n)), dim3(NT), 0, h.stream, int64_t(h.n), h.dim, a, x,
                     h.pts, w);
  check_launch("coord_mul");
}

void launch_coord_grad(H2& h, int a, double scale, const double* x, const double* v, const double* u,
                       double* grad) {
  hipLaunchKernelGGL(k_coord_grad, dim3(blocks(h.n)), dim3(NT), 0, h.stream, int64_t(h.n), h.dim, a,
                     scale, h.perm, x, h.pts, v, u, grad);
  check_launch("coord_grad");
}

void launch_check_finite(H2& h, int p, int64_t n, const void* x) {
  if (p == P64)
    hipLaunchKernelGGL(k_check_finite<double>, dim3(blocks(n)), dim3(NT), 0, h.stream, n,
                       static_cast<const double*>(x), h.flags + 1);
  else
    hipLaunchKernelGGL(k_check_finite<float>, dim3(blocks(n)), dim3(NT), 0, h.stream, n,
                       static_cast<const float*>(x), h.flags + 1);
  check_launch("check_finite");
}

}  // namespace h2mg
