// Device-side helpers shared by the setup and apply kernels.
//
// Tiled block layout.  Every r x r block (couplings S, projected close
// blocks, transfers E) is stored for a 64-lane wave laid out as an 8 x 8
// lane grid: lane l = 8a + b owns rows a*T .. a*T+T-1 and columns
// b*T .. b*T+T-1 of the block, where T is the smallest power of two with
// 8T >= r (entries beyond r are zero).  The T*T elements of a lane are cut
// into chunks of K consecutive elements (K = min(16 bytes / element size,
// T*T)), and chunk c of lane l lives at element offset (c*64 + l)*K, so a
// wave reads each chunk row as one contiguous 64*K-element segment.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace h2mg {

// ---------------------------------------------------------------- bf16
struct bf16 {
  uint16_t bits;
};

__host__ __device__ inline float bf16_to_float(bf16 v) {
  union { uint32_t u; float f; } c;
  c.u = uint32_t(v.bits) << 16;
  return c.f;
}

// Round-to-nearest-even of an FP32 value to BF16 (finite inputs).
__host__ __device__ inline bf16 float_to_bf16(float f) {
  union { uint32_t u; float f; } c;
  c.f = f;
  uint32_t lsb = (c.u >> 16) & 1u;
  bf16 r;
  r.bits = uint16_t((c.u + 0x7fffu + lsb) >> 16);
  return r;
}

template <typename T> struct Conv;
template <> struct Conv<double> {
  __device__ static double to_f64(double v) { return v; }
  __device__ static double from_f64(double v) { return v; }
};
template <> struct Conv<float> {
  __device__ static double to_f64(float v) { return v; }
  __device__ static float from_f64(double v) { return float(v); }
};
template <> struct Conv<bf16> {
  __device__ static double to_f64(bf16 v) { return bf16_to_float(v); }
  __device__ static bf16 from_f64(double v) { return float_to_bf16(float(v)); }
};

// Load one stored element as the accumulation type.
template <typename Tacc, typename Tb> __device__ inline Tacc ld_as(Tb v);
template <> __device__ inline double ld_as<double, double>(double v) { return v; }
template <> __device__ inline float ld_as<float, float>(float v) { return v; }
template <> __device__ inline float ld_as<float, bf16>(bf16 v) { return bf16_to_float(v); }
template <> __device__ inline double ld_as<double, float>(float v) { return v; }

// ---------------------------------------------------------------- tiles
__host__ __device__ constexpr int tile_T(int r) {
  return r <= 8 ? 1 : r <= 16 ? 2 : r <= 32 ? 4 : 8;
}
template <typename Tb>
__host__ __device__ constexpr int tile_K(int T) {
  return (16 / int(sizeof(Tb))) < T * T ? (16 / int(sizeof(Tb))) : T * T;
}
// Elements per stored tile.
__host__ __device__ constexpr int64_t tile_elems(int T) { return 64LL * T * T; }

// Element offset of block entry (i, j) inside a tile.
template <typename Tb>
__host__ __device__ inline int tile_offset(int i, int j, int T) {
  const int K = tile_K<Tb>(T);
  const int a = i / T, u = i % T, b = j / T, v = j % T;
  const int lane = 8 * a + b;
  const int e = u * T + v;
  return ((e / K) * 64 + lane) * K + (e % K);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Load the T*T elements of this lane's sub-tile (row-major u*T + v) from
// the tile starting at `tile`.  NT: non-temporal (streaming) loads, for
// blocks read once per product so they do not evict reused vectors.
template <int T, typename Tb, typename Tacc, bool NT = false>
__device__ inline void load_subtile(const Tb* __restrict__ tile, int lane, Tacc (&B)[T * T]) {
  constexpr int K = tile_K<Tb>(T);
  constexpr int NC = T * T / K;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const Tb* p = tile + (c * 64 + lane) * K;
    if constexpr (K * sizeof(Tb) == 16) {
      // one 16-byte load per chunk
      union { u32x4 q; Tb e[K]; } u;
      if constexpr (NT) u.q = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
      else u.q = *reinterpret_cast<const u32x4*>(p);
#pragma unroll
      for (int k = 0; k < K; ++k) B[c * K + k] = ld_as<Tacc, Tb>(u.e[k]);
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) B[c * K + k] = ld_as<Tacc, Tb>(p[k]);
    }
  }
}

// ---------------------------------------------------------------- kernels
enum { KER_EXP = 0, KER_GAUSS = 1, KER_MATERN32 = 2, KER_LAPLACE = 3 };
// deriv: the kernel itself, its derivative in the length scale at fixed r,
// or g(r) = k'(r) / r (0 at r = 0, where its self term cancels in the
// coordinate gradient).
enum { DER_NONE = 0, DER_LENGTH = 1, DER_RADIAL = 2 };

struct KernelParams {
  int kind;
  int deriv;
  double inv_l;        // 1 / l
  double inv_2l2;      // 1 / (2 l^2)
  double shift;
};

// k (or its derivative) as a function of the squared distance (no shift),
// for a kernel fixed at compile time.
template <int KIND, int DERIV, typename T>
__device__ inline T kernel_fixed(T inv_l, T inv_2l2, T r2) {
  if constexpr (KIND == KER_LAPLACE) {
    // 1 / (4 pi r); 0 at r = 0 (the matrix supplies its own diagonal)
    return r2 == T(0) ? T(0) : T(0.07957747154594767) / sqrt(r2);
  }
  if constexpr (DERIV == DER_RADIAL) {
    if (r2 == T(0)) return T(0);
  }
  if constexpr (KIND == KER_GAUSS) {
    const T e = exp(-r2 * inv_2l2);
    if constexpr (DERIV == DER_NONE) return e;
    else if constexpr (DERIV == DER_LENGTH) return r2 * inv_l * inv_l * inv_l * e;
    else return -inv_l * inv_l * e;
  } else if constexpr (KIND == KER_EXP) {
    const T rr = sqrt(r2);
    const T e = exp(-rr * inv_l);
    if constexpr (DERIV == DER_NONE) return e;
    else if constexpr (DERIV == DER_LENGTH) return rr * inv_l * inv_l * e;
    else return -inv_l * e / rr;
  } else {
    const T rr = sqrt(r2);
    const T z = T(1.7320508075688772) * rr * inv_l;
    const T e = exp(-z);
    if constexpr (DERIV == DER_NONE) return (T(1) + z) * e;
    else if constexpr (DERIV == DER_LENGTH) return z * z * inv_l * e;
    else return T(-3) * inv_l * inv_l * e;
  }
}

// Call f(integral_constant<KIND>, integral_constant<DERIV>) for a runtime pair.
template <typename F>
__host__ __device__ inline void dispatch_kernel(int kind, int deriv, F&& f) {
  using I = int;
  auto d = [&](auto kc) {
    if (deriv == DER_LENGTH) f(kc, std::integral_constant<I, DER_LENGTH>{});
    else if (deriv == DER_RADIAL) f(kc, std::integral_constant<I, DER_RADIAL>{});
    else f(kc, std::integral_constant<I, DER_NONE>{});
  };
  if (kind == KER_GAUSS) d(std::integral_constant<I, KER_GAUSS>{});
  else if (kind == KER_EXP) d(std::integral_constant<I, KER_EXP>{});
  else if (kind == KER_LAPLACE)   // no length scale, so no derivative kernels
    f(std::integral_constant<I, KER_LAPLACE>{}, std::integral_constant<I, DER_NONE>{});
  else d(std::integral_constant<I, KER_MATERN32>{});
}

template <typename T>
__device__ inline T kernel_r2_t(int kind, int deriv, T inv_l, T inv_2l2, T r2) {
  T v = T(0);
  dispatch_kernel(kind, deriv, [&](auto kc, auto dc) {
    v = kernel_fixed<decltype(kc)::value, decltype(dc)::value, T>(inv_l, inv_2l2, r2);
  });
  return v;
}

__device__ inline double kernel_r2(const KernelParams& kp, double r2) {
  return kernel_r2_t<double>(kp.kind, kp.deriv, kp.inv_l, kp.inv_2l2, r2);
}

__device__ inline float kernel_r2(const KernelParams& kp, float r2) {
  return kernel_r2_t<float>(kp.kind, kp.deriv, float(kp.inv_l), float(kp.inv_2l2), r2);
}

// Per-point scale s (on rows and columns) and diagonal d of the scaled form
// diag(s) K diag(s) + diag(d), tree order; null pointers mean s = 1 and
// d = the constant shift.  Optional quadrature of the close entries: point i
// carries nq sub-points qy[i] (nq x dim, row-major) with weights qu[i] (nq),
// and the entry between distinct points i, j of a close leaf pair is
// sum_p sum_q qu[i][p] qu[j][q] k(|qy[i][p] - qy[j][q]|) (the weights carry
// any scaling; far blocks keep the point values).
struct PointScale {
  const double* s;
  const double* d;
  const double* qy;
  const double* qu;
  int nq;
};

// One entry of the scaled matrix from the kernel value k between tree
// positions i and j (self: the same point).
__device__ inline double scaled_entry(double k, int64_t i, int64_t j, bool self, const PointScale& ps,
                                      double shift) {
  if (ps.s) k *= ps.s[i] * ps.s[j];
  if (self) k += ps.d ? ps.d[i] : shift;
  return k;
}

// The close entry (i, j) of a leaf pair: the point kernel value (squared
// distance r2 of the two points) in the scaled form, or the quadrature sum
// when the close entries are given by quadrature (its diagonal is d or the
// shift).
__device__ inline double near_entry(const KernelParams& kp, const PointScale& ps, int dim, double r2,
                                    int64_t i, int64_t j, bool self) {
  if (!ps.qy) return scaled_entry(kernel_r2(kp, r2), i, j, self, ps, kp.shift);
  if (self) return ps.d ? ps.d[i] : kp.shift;
  const int nq = ps.nq;
  const double* yi = ps.qy + i * nq * dim;
  const double* yj = ps.qy + j * nq * dim;
  const double* ui = ps.qu + i * nq;
  const double* uj = ps.qu + j * nq;
  double sum = 0.0;
  for (int p = 0; p < nq; ++p) {
    double part = 0.0;
    for (int q = 0; q < nq; ++q) {
      double d2 = 0.0;
      for (int a = 0; a < dim; ++a) {
        const double dx = yi[p * dim + a] - yj[q * dim + a];
        d2 += dx * dx;
      }
      part += uj[q] * kernel_r2(kp, d2);
    }
    sum += ui[p] * part;
  }
  return sum;
}

// ---------------------------------------------------------------- shuffles
__device__ inline double shfl_xor(double v, int m) { return __shfl_xor(v, m, 64); }
__device__ inline float shfl_xor(float v, int m) { return __shfl_xor(v, m, 64); }

}  // namespace h2mg
