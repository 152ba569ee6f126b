// Panel quantities of the boundary-element matrix of the Laplace single
// layer (Section 4.3) in its symmetric scaled form.
//
// Per triangle i: centroid y_i (the collocation point), area w_i, scale
// s_i = sqrt(w_i), and the diagonal entry d_i = I_i / (4 pi), with I_i the
// integral of 1 / |y_i - y| over the flat triangle (the potential of the
// panel's own uniform density at its centroid), in closed form edge by edge:
// d_e ln((s_2 + r_2) / (s_1 + r_1)), where d_e is the distance from the
// centroid to the edge line, s_1, s_2 the positions of the edge end points
// along it and r_1, r_2 their distances to the centroid.  The right-hand side
// of a point source x_0 in the scaled form is s_i / (4 pi |y_i - x_0|).
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>

#include "h2_impl.h"

namespace h2mg {

namespace {

constexpr int NT = 256;
constexpr double INV_4PI = 0.07957747154594767;

struct V3 {
  double x, y, z;
};
__device__ inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline double norm(V3 a) { return sqrt(dot(a, a)); }
__device__ inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline V3 load(const double* V, int64_t v) { return {V[3 * v], V[3 * v + 1], V[3 * v + 2]}; }

// Contribution of edge p1 -> p2 to the integral of 1/r around c.
__device__ inline double edge_term(V3 p1, V3 p2, V3 c) {
  const V3 e = sub(p2, p1);
  const double le = norm(e);
  const V3 t = {e.x / le, e.y / le, e.z / le};
  const double s1 = dot(sub(p1, c), t), s2 = dot(sub(p2, c), t);
  const V3 foot = {p1.x - s1 * t.x, p1.y - s1 * t.y, p1.z - s1 * t.z};
  const double d = norm(sub(c, foot));
  const double r1 = norm(sub(p1, c)), r2 = norm(sub(p2, c));
  return d * log((s2 + r2) / (s1 + r1));
}

__global__ __launch_bounds__(NT) void k_bem_panels(int64_t nt, const double* __restrict__ V,
                                                   const int64_t* __restrict__ T,
                                                   double* __restrict__ y, double* __restrict__ s,
                                                   double* __restrict__ d) {
  const int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (i >= nt) return;
  const V3 a = load(V, T[3 * i]), b = load(V, T[3 * i + 1]), c = load(V, T[3 * i + 2]);
  const V3 g = {(a.x + b.x + c.x) / 3.0, (a.y + b.y + c.y) / 3.0, (a.z + b.z + c.z) / 3.0};
  const double w = 0.5 * norm(cross(sub(b, a), sub(c, a)));
  y[3 * i] = g.x;
  y[3 * i + 1] = g.y;
  y[3 * i + 2] = g.z;
  s[i] = sqrt(w);
  d[i] = INV_4PI * (edge_term(a, b, g) + edge_term(b, c, g) + edge_term(c, a, g));
}

// Radon's seven-point rule on triangle i (exact for polynomials of degree
// <= 5): the centroid with weight 9/40 and the two orbits of barycentric
// points (a, a, 1 - 2a), a = (6 -+ sqrt 15) / 21, with weights
// (155 -+ sqrt 15) / 1200; the weights are multiplied by the area w_i and
// divided by s_i = sqrt(w_i) (the symmetric form's scaling), so
// u_ip = sqrt(w_i) * rule weight.  qy: 7 points of 3 coordinates.
__global__ __launch_bounds__(NT) void k_bem_quadrature7(int64_t nt, const double* __restrict__ V,
                                                        const int64_t* __restrict__ T,
                                                        double* __restrict__ qy, double* __restrict__ qu) {
  const int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (i >= nt) return;
  const V3 a = load(V, T[3 * i]), b = load(V, T[3 * i + 1]), c = load(V, T[3 * i + 2]);
  const double w = 0.5 * norm(cross(sub(b, a), sub(c, a)));
  const double sw = sqrt(w);
  const double r15 = sqrt(15.0);
  const double orb[2] = {(6.0 - r15) / 21.0, (6.0 + r15) / 21.0};
  const double wt[2] = {(155.0 - r15) / 1200.0, (155.0 + r15) / 1200.0};
  double* py = qy + i * 21;
  double* pu = qu + i * 7;
  auto put = [&](int k, double la, double lb, double lc, double weight) {
    py[3 * k] = la * a.x + lb * b.x + lc * c.x;
    py[3 * k + 1] = la * a.y + lb * b.y + lc * c.y;
    py[3 * k + 2] = la * a.z + lb * b.z + lc * c.z;
    pu[k] = sw * weight;
  };
  put(0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, 9.0 / 40.0);
  for (int o = 0; o < 2; ++o) {
    const double t = orb[o], u = 1.0 - 2.0 * t;
    put(1 + 3 * o, u, t, t, wt[o]);
    put(2 + 3 * o, t, u, t, wt[o]);
    put(3 + 3 * o, t, t, u, wt[o]);
  }
}

__global__ __launch_bounds__(NT) void k_bem_rhs(int64_t n, const double* __restrict__ y,
                                                double x0, double x1, double x2,
                                                const double* __restrict__ s, double* __restrict__ f) {
  const int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (i >= n) return;
  const double dx = y[3 * i] - x0, dy = y[3 * i + 1] - x1, dz = y[3 * i + 2] - x2;
  f[i] = s[i] * INV_4PI / sqrt(dx * dx + dy * dy + dz * dz);
}

struct Harmonic {
  double c[9];
};

// f_i = s_i * sum_k c_k h_k(y_i) over 1, x, y, z, xy, yz, zx, x^2 - y^2,
// x^2 + y^2 - 2 z^2.
__global__ __launch_bounds__(NT) void k_bem_harmonic(int64_t n, const double* __restrict__ y, Harmonic h,
                                                     const double* __restrict__ s, double* __restrict__ f) {
  const int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (i >= n) return;
  const double x0 = y[3 * i], x1 = y[3 * i + 1], x2 = y[3 * i + 2];
  const double v = h.c[0] + h.c[1] * x0 + h.c[2] * x1 + h.c[3] * x2 + h.c[4] * x0 * x1 + h.c[5] * x1 * x2 +
                   h.c[6] * x2 * x0 + h.c[7] * (x0 * x0 - x1 * x1) +
                   h.c[8] * (x0 * x0 + x1 * x1 - 2.0 * x2 * x2);
  f[i] = s[i] * v;
}

__global__ __launch_bounds__(NT) void k_div(int64_t n, const double* __restrict__ x,
                                            const double* __restrict__ s, double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (i < n) out[i] = x[i] / s[i];
}

inline unsigned blocks(int64_t n) { return unsigned((n + NT - 1) / NT); }

void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

void launch_bem_panels(hipStream_t st, int64_t nt, const double* V, const int64_t* T, double* y,
                       double* s, double* d) {
  if (nt == 0) return;
  hipLaunchKernelGGL(k_bem_panels, dim3(blocks(nt)), dim3(NT), 0, st, nt, V, T, y, s, d);
  check_launch("bem_panels");
}

void launch_bem_quadrature7(hipStream_t st, int64_t nt, const double* V, const int64_t* T, double* qy,
                            double* qu) {
  if (nt == 0) return;
  hipLaunchKernelGGL(k_bem_quadrature7, dim3(blocks(nt)), dim3(NT), 0, st, nt, V, T, qy, qu);
  check_launch("bem_quadrature7");
}

void launch_bem_rhs(hipStream_t st, int64_t n, const double* y, const double* x0, const double* s,
                    double* f) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_bem_rhs, dim3(blocks(n)), dim3(NT), 0, st, n, y, x0[0], x0[1], x0[2], s, f);
  check_launch("bem_rhs");
}

void launch_bem_harmonic(hipStream_t st, int64_t n, const double* y, const double* coeffs, const double* s,
                         double* f) {
  if (n == 0) return;
  Harmonic h;
  for (int k = 0; k < 9; ++k) h.c[k] = coeffs[k];
  hipLaunchKernelGGL(k_bem_harmonic, dim3(blocks(n)), dim3(NT), 0, st, n, y, h, s, f);
  check_launch("bem_harmonic");
}

void launch_div(hipStream_t st, int64_t n, const double* x, const double* s, double* out) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_div, dim3(blocks(n)), dim3(NT), 0, st, n, x, s, out);
  check_launch("div");
}

}  // namespace h2mg
