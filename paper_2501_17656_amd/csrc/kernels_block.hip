// Kernels on blocks of NR = 16 vectors (the H2 matvec of Section 3.1 and the
// steps of Algorithm 1 applied to 16 right-hand sides at once), in FP64 or in
// FP32 vectors over FP32 or BF16 operators.
//
// Block layout.  Entry (i, k) of a block at i * 16 + k; coefficients of
// cluster g at (g * r + j) * 16 + k.  One wave load of 64 consecutive
// elements covers 4 rows of all 16 columns.
//
// Tile products.  With 16 columns a stored tile B (r x r coupling or
// projected close block, 64 x 64 near-field tile) times a 16-column block is
// a dense product, done on the matrix cores: v_mfma_f64_16x16x4f64 for FP64
// and v_mfma_f32_16x16x4f32 for FP32 (BF16 tiles are widened to FP32 while
// staged).  For both, lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// the 16 x 16 result comes back as D[4 t + l / 16][l % 16] in accumulator t
// for FP64 and as D[4 (l / 16) + t][l % 16] for FP32 (measured on gfx950).
// A tile is read from HBM once per pass, in the coalesced 16-byte chunks of
// its storage layout, staged in LDS with an XOR swizzle of the column index
// (f(i) below, chosen per tile size and element width so that the staging
// writes and both operand read patterns have at most the minimum number of
// bank conflicts), and multiplied from there:
//   * row pass (tasks = runs of tiles of one block row s):
//       Y_s = sum_t B_st X_t, accumulated in registers over the run;
//   * column pass (tasks = runs of off-diagonal tiles of one block column t):
//       Y_t = sum_s B_st^T X_s.
// Each task writes one partial; a reduce sums a row's row-pass and
// column-pass partials in a fixed order (deterministic, no atomics).
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>
#include <type_traits>

#include "h2_impl.h"

namespace h2mg {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int NR = MULTI_NR;           // columns of a block
constexpr int NT = 256;

void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

inline unsigned blocks(int64_t n, int nt) { return unsigned((n + nt - 1) / nt); }

// LDS column swizzle f(i) = M i over GF(2): bit t of f(i) is the parity of
// i & m_t.  Row i of a staged RP x RP tile holds column j at j ^ f(i).
template <int RP, int EB>
__device__ __forceinline__ int swz(int i) {
  int m0, m1, m2, m3, m4 = 0, m5 = 0;
  if constexpr (RP == 16) {
    m0 = 4; m1 = 15; m2 = 4; m3 = 11;
  } else if constexpr (RP == 32 && EB == 4) {
    m0 = 20; m1 = 7; m2 = 13; m3 = 19; m4 = 16;
  } else if constexpr (RP == 32) {
    m0 = 18; m1 = 5; m2 = 11; m3 = 26; m4 = 30;
  } else if constexpr (EB == 4) {
    m0 = 48; m1 = 23; m2 = 26; m3 = 31; m4 = 3; m5 = 2;
  } else {
    m0 = 52; m1 = 19; m2 = 27; m3 = 2; m4 = 37; m5 = 37;
  }
  return (__popc(i & m0) & 1) | ((__popc(i & m1) & 1) << 1) | ((__popc(i & m2) & 1) << 2) |
         ((__popc(i & m3) & 1) << 3) | ((__popc(i & m4) & 1) << 4) | ((__popc(i & m5) & 1) << 5);
}

template <typename Tc> struct Mfma;
template <> struct Mfma<double> {
  typedef d4 acc_t;
  __device__ static d4 mma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int t, int q) { return 4 * t + q; }
};
template <> struct Mfma<float> {
  typedef f4 acc_t;
  __device__ static f4 mma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int t, int q) { return 4 * q + t; }
};

// Tile products of one launch.  MODE_LIST: blocks [0, nrt) run the
// row-pass tasks (index, i0, i1) over rorder, blocks [nrt, nrt + nct) the
// column-pass tasks over corder.  Tile b joins block row brow[b] and block
// column bcol[b]; the operand of a row task is the block of bcol[b], of a
// column task that of brow[b], at x + index * rr * 16 (rr rows: the rank for
// coupling tiles, 64 for near-field tiles; rows >= rr of the RP = 8T padded
// tile are zero).  out[block] = the rr x 16 result.
// MODE_UP (transfer to the parents): block s sums E_c^T x[c] over its two
// children c = 2s, 2s+1 (tiles base + c).  MODE_DOWN (transfer to the
// children): block c computes E_c x[c / 2] (tile base + c), plus addend[c]
// when addend is not null.
// A block has one wave per 16-row slab of the result (RP / 16 = T / 2
// waves); all of them stage the tile into LDS together, then wave w runs the
// matrix-core products of slab w.  The stage object fills LDS: load(b, regs)
// issues this thread's share of the tile's global loads, store(b, regs, put)
// writes entry (i, j) through put(i, j, value).  When Stage::PREFETCH, the
// loads of the next tile are issued as soon as the current one is in LDS, so
// they overlap its products; the operand rows are loaded before staging.
// DUAL (MODE_LIST, no column-pass tasks): each staged off-diagonal tile also
// gives its transposed product B^T X_s, with X_s the task's block-row
// operand, written as the rr x 16 column contribution of slot rslot[it]
// (the tile's place among the off-diagonal tiles ordered by column) after
// the nrt row partials: every tile is read once instead of twice.
enum { MODE_LIST = 0, MODE_UP = 1, MODE_DOWN = 2 };

template <int T, int MODE, typename Tv, typename Stage, bool DUAL = false>
__device__ __forceinline__ void tgemm_body(int blk, const int* __restrict__ rtask, int nrt,
                                           const int* __restrict__ rorder,
                                           const int* __restrict__ ctask,
                                           const int* __restrict__ corder,
                                           const int* __restrict__ brow,
                                           const int* __restrict__ bcol, int base, int rr,
                                           const Tv* __restrict__ x, Tv* out_base, const Tv* addend,
                                           Tv* lds, const Stage& stage,
                                           const int* __restrict__ rslot = nullptr) {
  constexpr int RP = 8 * T, NKB = RP / 4;
  constexpr int EB = int(sizeof(Tv));
  using M = Mfma<Tv>;
  bool tr;
  int i0, i1;
  const int* order = nullptr;
  const int* other = nullptr;
  int task_row = 0;
  if constexpr (MODE == MODE_LIST) {
    tr = blk >= nrt;
    const int* task = tr ? ctask + 3 * (blk - nrt) : rtask + 3 * blk;
    task_row = task[0];
    order = tr ? corder : rorder;
    other = tr ? brow : bcol;
    i0 = task[1];
    i1 = task[2];
  } else if constexpr (MODE == MODE_UP) {
    tr = true;
    i0 = 2 * blk;
    i1 = 2 * blk + 2;
  } else {
    tr = false;
    i0 = blk;
    i1 = blk + 1;
  }
  auto tile_of = [&](int it) {
    if constexpr (MODE == MODE_LIST) return order[it];
    else return base + it;
  };
  auto other_of = [&](int it, int b) {
    if constexpr (MODE == MODE_LIST) return other[b];
    else if constexpr (MODE == MODE_UP) return it;
    else return it >> 1;
  };
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, p = l & 15, q = l >> 4;
  const int nkb = (rr + 3) >> 2;
  auto put = [&](int i, int j, Tv v) { lds[i * RP + (j ^ swz<RP, EB>(i))] = v; };
  typename M::acc_t acc = typename M::acc_t{Tv(0), Tv(0), Tv(0), Tv(0)};
  const int slab = 16 * w + p;          // this lane's result row (row pass) / column (transposed)
  // The pass (row or transposed) is uniform per block; each has its own loop
  // with the LDS addressing fixed at compile time.
  auto run = [&](auto trc) {
    constexpr bool TR = decltype(trc)::value;
    const int slabsw = swz<RP, EB>(slab);
    auto mma_step = [&](int kb, Tv xb) {
      const int kr = 4 * kb + q;
      if constexpr (TR) acc = M::mma(lds[kr * RP + (slab ^ swz<RP, EB>(kr))], xb, acc);
      else acc = M::mma(lds[slab * RP + (kr ^ slabsw)], xb, acc);
    };
    typename Stage::Regs regs;
    int b = tile_of(i0);
    if constexpr (Stage::PREFETCH) stage.load(b, regs);
    // DUAL: operand of the transposed products (the task's own block row)
    Tv xs[DUAL ? NKB : 1];
    if constexpr (DUAL) {
      const Tv* xso = x + int64_t(task_row) * rr * NR;
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        const int kr = 4 * kb + q;
        xs[kb] = kr < rr ? xso[kr * NR + p] : Tv(0);
      }
    }
    for (int it = i0; it < i1; ++it) {
      const int o = other_of(it, b);
      const Tv* xo = x + int64_t(o) * rr * NR;
      Tv xr[NKB];
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        const int kr = 4 * kb + q;
        xr[kb] = kr < rr ? xo[kr * NR + p] : Tv(0);
      }
      __syncthreads();                 // every wave's operand reads of the previous tile are done
      if constexpr (!Stage::PREFETCH) stage.load(b, regs);
      stage.store(b, regs, put);
      if (it + 1 < i1) {
        b = tile_of(it + 1);
        if constexpr (Stage::PREFETCH) stage.load(b, regs);
      }
      __syncthreads();
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb)
        if (kb < nkb) mma_step(kb, xr[kb]);
      if constexpr (DUAL && !TR) {
        const int slot = rslot[it];
        if (slot >= 0) {
          typename M::acc_t at = typename M::acc_t{Tv(0), Tv(0), Tv(0), Tv(0)};
#pragma unroll
          for (int kb = 0; kb < NKB; ++kb) {
            const int kr = 4 * kb + q;
            if (kb < nkb) at = M::mma(lds[kr * RP + (slab ^ swz<RP, EB>(kr))], xs[kb], at);
          }
          Tv* oc = out_base + int64_t(nrt + slot) * rr * NR;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int row = 16 * w + M::row(t, q);
            if (row < rr) oc[row * NR + p] = at[t];
          }
        }
      }
    }
  };
  if (tr) run(std::integral_constant<bool, true>{});
  else run(std::integral_constant<bool, false>{});
  Tv* out = out_base + int64_t(blk) * rr * NR;
  const Tv* add = addend ? addend + int64_t(blk) * rr * NR : nullptr;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int row = 16 * w + M::row(t, q);
    if (row < rr) out[row * NR + p] = add ? acc[t] + add[row * NR + p] : acc[t];
  }
}

// Stored tiles: lane (a, b) of the 8 x 8 lane grid holds the T x T sub-block
// of rows aT.., columns bT.. of the storage layout, cut into NCH chunks of 16
// bytes; wave w of the block loads chunks w, w + W, ... (W = T / 2 waves),
// so each thread keeps NCH / W chunks in registers while they are in flight.
template <int T, typename Te, typename Tv>
struct StageStored {
  static constexpr int W = T / 2;
  static constexpr int K = tile_K<Te>(T), NCH = T * T / K, NPW = NCH / W;
  static constexpr bool PREFETCH = true;
  static_assert(NCH % W == 0, "chunks must split evenly over the waves");
  union Chunk {
    u32x4 q4;
    Te e[16 / sizeof(Te)];
  };
  struct Regs {
    Chunk c[NPW];
  };
  const Te* tiles;
  __device__ __forceinline__ static void load_chunk(const Te* src, Chunk& u) {
    if constexpr (K * sizeof(Te) == 16) {
      u.q4 = *reinterpret_cast<const u32x4*>(src);
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) u.e[k] = src[k];
    }
  }
  __device__ __forceinline__ void load(int b, Regs& R) const {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const Te* tile = tiles + int64_t(b) * tile_elems(T);
#pragma unroll
    for (int cc = 0; cc < NPW; ++cc) load_chunk(tile + ((w + W * cc) * 64 + l) * K, R.c[cc]);
  }
  template <typename Put>
  __device__ __forceinline__ void store(int, const Regs& R, Put& put) const {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, a = l >> 3, bb = l & 7;
#pragma unroll
    for (int cc = 0; cc < NPW; ++cc)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int el = (w + W * cc) * K + k;
        put(T * a + el / T, T * bb + el % T, ld_as<Tv, Te>(R.c[cc].e[k]));
      }
  }
};

template <int T, typename Te, typename Tv, bool DUAL>
__global__ __launch_bounds__(32 * T) void k_tgemm(const int* __restrict__ rtask, int nrt,
                                                  const int* __restrict__ rorder,
                                                  const int* __restrict__ ctask,
                                                  const int* __restrict__ corder,
                                                  const Te* __restrict__ tiles,
                                                  const int* __restrict__ brow,
                                                  const int* __restrict__ bcol, int rr,
                                                  const Tv* __restrict__ x, Tv* __restrict__ partial,
                                                  const int* __restrict__ rslot) {
  __shared__ Tv lds[64 * T * T];
  tgemm_body<T, MODE_LIST, Tv, StageStored<T, Te, Tv>, DUAL>(
      blockIdx.x, rtask, nrt, rorder, ctask, corder, brow, bcol, 0, rr, x, partial,
      static_cast<const Tv*>(nullptr), lds, StageStored<T, Te, Tv>{tiles}, rslot);
}

// Transfers between depth d + 1 (children, gids base + c) and depth d.
template <int T, int MODE, typename Te, typename Tv>
__global__ __launch_bounds__(32 * T) void k_transfer16(const Te* __restrict__ E, int base, int r,
                                                       const Tv* __restrict__ x, Tv* out, const Tv* addend) {
  __shared__ Tv lds[64 * T * T];
  tgemm_body<T, MODE>(blockIdx.x, nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, base, r, x, out,
                      addend, lds, StageStored<T, Te, Tv>{E});
}

// Near-field tiles evaluated from the points: lane (a, b) of wave w
// evaluates rows 8a + 2w, 8a + 2w + 1 and columns 8b .. 8b+7 of the 64 x 64
// tile (4 waves).
template <typename Tv, int KIND, int DERIV>
struct StageEval {
  static constexpr bool PREFETCH = false;
  struct Regs {};
  const int* brow;
  const int* bcol;
  const int* chunk_start;
  const int* chunk_n;
  const double* pts;
  int dim;
  KernelParams kp;
  PointScale ps;
  __device__ __forceinline__ void load(int, Regs&) const {}
  template <typename Put>
  __device__ __forceinline__ void store(int b, const Regs&, Put& put) const {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, a = l >> 3, bb = l & 7;
    const Tv inv_l = Tv(kp.inv_l), inv_2l2 = Tv(kp.inv_2l2);
    const int rs = chunk_start[brow[b]], nr = chunk_n[brow[b]];
    const int cs = chunk_start[bcol[b]], nc = chunk_n[bcol[b]];
    double pc[8][3];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int j = 8 * bb + v;
#pragma unroll
      for (int d = 0; d < 3; ++d) pc[v][d] = (j < nc && d < dim) ? pts[int64_t(cs + j) * dim + d] : 0.0;
    }
#pragma unroll
    for (int uu = 0; uu < 2; ++uu) {
      const int i = 8 * a + 2 * w + uu;
      const bool rowok = i < nr;
      double pr[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) pr[d] = (rowok && d < dim) ? pts[int64_t(rs + i) * dim + d] : 0.0;
      const int64_t gi = int64_t(rs) + i;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int j = 8 * bb + v;
        Tv e = Tv(0);
        if (rowok && j < nc) {
          // coordinate differences in FP64 (no cancellation), their squares
          // in the vector precision
          Tv r2 = Tv(0);
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const Tv dx = Tv(pr[d] - pc[v][d]);
            r2 += dx * dx;
          }
          const int64_t gj = int64_t(cs) + j;
          e = kernel_fixed<KIND, DERIV, Tv>(inv_l, inv_2l2, r2);
          if (ps.s) e *= Tv(ps.s[gi] * ps.s[gj]);
          if (gi == gj) e += Tv(ps.d ? ps.d[gi] : kp.shift);
        }
        put(i, j, e);
      }
    }
  }
};

// Near-field tiles evaluated from the points instead of read: tile b is the
// block between chunk brow[b] and chunk bcol[b] (at most 64 consecutive
// points of a leaf each; chunk_start / chunk_n), entry (i, j) = the scaled
// kernel s_i k(|p_i - p_j|) s_j plus the diagonal (the per-point d, else the
// shift) where a point meets itself, zero outside the chunks.  Coordinate
// differences are formed in FP64, the rest in the vector precision.
template <typename Tv, int KIND, int DERIV, bool DUAL>
__global__ __launch_bounds__(256) void k_tgemm_eval(const int* __restrict__ rtask, int nrt,
                                                    const int* __restrict__ rorder,
                                                    const int* __restrict__ ctask,
                                                    const int* __restrict__ corder,
                                                    const int* __restrict__ brow,
                                                    const int* __restrict__ bcol,
                                                    const int* __restrict__ chunk_start,
                                                    const int* __restrict__ chunk_n,
                                                    const double* __restrict__ pts, int dim,
                                                    KernelParams kp, PointScale ps,
                                                    const Tv* __restrict__ x, Tv* __restrict__ partial,
                                                    const int* __restrict__ rslot) {
  __shared__ Tv lds[64 * 64];
  tgemm_body<8, MODE_LIST, Tv, StageEval<Tv, KIND, DERIV>, DUAL>(
      blockIdx.x, rtask, nrt, rorder, ctask, corder, brow, bcol, 0, 64, x, partial,
      static_cast<const Tv*>(nullptr), lds,
      StageEval<Tv, KIND, DERIV>{brow, bcol, chunk_start, chunk_n, pts, dim, kp, ps}, rslot);
}

// ------------------------------------------------------------ several problems in one launch
// The tile products of up to GROUP_MAX independent problems in one grid:
// member m owns the blocks [start[m], start[m + 1]) and runs them exactly as
// its own launch would (same tasks, same per-block arithmetic), so each
// problem's partial sums are bit for bit those of a launch of its own.
template <int T, typename Te, typename Tv, bool DUAL>
__global__ __launch_bounds__(32 * T) void k_tgemm_group(TgemmGroup G) {
  __shared__ Tv lds[64 * T * T];
  int m = 0;
  while (m + 1 < G.n && G.start[m + 1] <= int(blockIdx.x)) ++m;
  const TgemmMember& M = G.m[m];
  tgemm_body<T, MODE_LIST, Tv, StageStored<T, Te, Tv>, DUAL>(
      int(blockIdx.x) - G.start[m], M.rtask, M.nrt, M.rorder, M.ctask, M.corder, M.brow, M.bcol, 0, M.rr,
      static_cast<const Tv*>(M.x), static_cast<Tv*>(M.partial), static_cast<const Tv*>(nullptr), lds,
      StageStored<T, Te, Tv>{static_cast<const Te*>(M.tiles)}, M.rslot);
}

template <typename Tv, int KIND, int DERIV, bool DUAL>
__global__ __launch_bounds__(256) void k_tgemm_eval_group(TevalGroup G) {
  __shared__ Tv lds[64 * 64];
  int m = 0;
  while (m + 1 < G.n && G.start[m + 1] <= int(blockIdx.x)) ++m;
  const TevalMember& M = G.m[m];
  tgemm_body<8, MODE_LIST, Tv, StageEval<Tv, KIND, DERIV>, DUAL>(
      int(blockIdx.x) - G.start[m], M.rtask, M.nrt, M.rorder, M.ctask, M.corder, M.brow, M.bcol, 0, 64,
      static_cast<const Tv*>(M.x), static_cast<Tv*>(M.partial), static_cast<const Tv*>(nullptr), lds,
      StageEval<Tv, KIND, DERIV>{M.brow, M.bcol, M.chunk_start, M.chunk_n, M.pts, M.dim, M.kp, M.ps}, M.rslot);
}

// v += p[t * stride] for t = a .. b - 1, added in that order, with eight
// loads in flight (a row can have hundreds of column contributions).
template <typename Tv>
__device__ __forceinline__ void sum_run(Tv& v, const Tv* __restrict__ p, int64_t stride, int a, int b) {
  int t = a;
  for (; t + 8 <= b; t += 8) {
    Tv x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = p[int64_t(t + k) * stride];
#pragma unroll
    for (int k = 0; k < 8; ++k) v += x[k];
  }
  for (; t < b; ++t) v += p[int64_t(t) * stride];
}

// out[row] (rr x 16) = the row-pass partials [rtp[row], rtp[row+1]) plus the
// column-pass partials [ctp[row], ctp[row+1]) (after the nrt row-pass ones),
// summed in that order, for rows row0 .. row0 + nrows - 1.  Workgroup
// (row, y) sums elements y * NT .. of its row, one element per thread.
template <typename Tv>
__global__ __launch_bounds__(NT) void k_reduce16(int row0, const int* __restrict__ rtp,
                                                 const int* __restrict__ ctp, int nrt, int rr,
                                                 const Tv* __restrict__ partial, Tv* __restrict__ out) {
  const int row = row0 + blockIdx.x;
  const int e = blockIdx.y * NT + threadIdx.x;
  if (e >= rr * NR) return;
  const int64_t stride = int64_t(rr) * NR;
  Tv v = Tv(0);
  sum_run(v, partial + e, stride, rtp[row], rtp[row + 1]);
  sum_run(v, partial + e, stride, nrt + ctp[row], nrt + ctp[row + 1]);
  out[row * stride + e] = v;
}

// Tree-order FP64 block from user order (columns >= nrhs zero), and back.
__global__ __launch_bounds__(NT) void k_gather16(int64_t n, int nrhs, const int64_t* __restrict__ perm,
                                                 const double* __restrict__ user, int ldu,
                                                 double* __restrict__ tree) {
  const int64_t idx = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (idx >= n * NR) return;
  const int64_t i = idx / NR;
  const int k = int(idx % NR);
  tree[idx] = k < nrhs ? user[perm[i] * ldu + k] : 0.0;
}

__global__ __launch_bounds__(NT) void k_scatter16(int64_t n, int nrhs, const int64_t* __restrict__ perm,
                                                  const double* __restrict__ tree,
                                                  double* __restrict__ user, int ldu) {
  const int64_t idx = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (idx >= n * NR) return;
  const int64_t i = idx / NR;
  const int k = int(idx % NR);
  if (k < nrhs) user[perm[i] * ldu + k] = tree[idx];
}

// xhat[leaf] (r x 16) = Q_leaf^T x_leaf.
template <typename Tq, typename Tv>
__global__ __launch_bounds__(NT) void k_leaf_up16(const int* __restrict__ leaf_off,
                                                  const Tq* __restrict__ Qr, int r,
                                                  const Tv* __restrict__ x, Tv* __restrict__ xhat) {
  const int leaf = blockIdx.x;
  const int s0 = leaf_off[leaf], n = leaf_off[leaf + 1] - s0;
  for (int e = threadIdx.x; e < r * NR; e += NT) {
    const int j = e / NR, k = e % NR;
    Tv v = Tv(0);
    for (int i = 0; i < n; ++i)
      v += ld_as<Tv, Tq>(Qr[int64_t(s0 + i) * r + j]) * x[int64_t(s0 + i) * NR + k];
    xhat[(int64_t(leaf) * r + j) * NR + k] = v;
  }
}

// out = alpha * (Q_leaf yhat_leaf + near) + beta * add over the rows of one
// leaf per workgroup (tree order); yhat or near may be null, add is read
// only when beta != 0 (it may alias out).
template <typename Tq, typename Tv>
__global__ __launch_bounds__(NT) void k_leaf_down16(const int* __restrict__ leaf_off,
                                                    const Tq* __restrict__ Qr, int r,
                                                    const Tv* __restrict__ yhat,
                                                    const Tv* __restrict__ near_y,
                                                    const int* __restrict__ chunk_base, Tv* out,
                                                    double alpha, const Tv* add, double beta) {
  const int leaf = blockIdx.x;
  const int s0 = leaf_off[leaf], n = leaf_off[leaf + 1] - s0;
  for (int e = threadIdx.x; e < n * NR; e += NT) {
    const int i = e / NR, k = e % NR;
    Tv v = Tv(0);
    if (yhat)
      for (int j = 0; j < r; ++j)
        v += ld_as<Tv, Tq>(Qr[int64_t(s0 + i) * r + j]) * yhat[(int64_t(leaf) * r + j) * NR + k];
    if (near_y) v += near_y[(int64_t(chunk_base[leaf]) * 64 + i) * NR + k];
    const int64_t idx = int64_t(s0 + i) * NR + k;
    Tv o = Tv(alpha) * v;
    if (beta != 0.0) o += Tv(beta) * add[idx];
    out[idx] = o;
  }
}

// Chunk-padded block from the tree-order block (padding rows stay zero).
template <typename Tv>
__global__ __launch_bounds__(NT) void k_near_pad16(const int* __restrict__ leaf_off,
                                                   const int* __restrict__ chunk_base,
                                                   const Tv* __restrict__ x, Tv* __restrict__ xc) {
  const int leaf = blockIdx.x;
  const int s0 = leaf_off[leaf], n = leaf_off[leaf + 1] - s0;
  Tv* dst = xc + int64_t(chunk_base[leaf]) * 64 * NR;
  for (int e = threadIdx.x; e < n * NR; e += NT) dst[e] = x[int64_t(s0) * NR + e];
}

// ------------------------------------------------------------ column dots and CG steps
// Thread (g, k) = (threadIdx / 16, threadIdx % 16) of a 256-thread block
// works on column k and rows g, g + 16, ... of the block's grid stride.

// sums[k] = sum over b < np of part[b * 16 + k], in a fixed order.
__device__ inline void colsum16(const double* __restrict__ part, int np, double* sums, double* red) {
  const int k = threadIdx.x & 15, g = threadIdx.x >> 4;
  double s = 0.0;
  for (int b = g; b < np; b += 16) s += part[b * NR + k];
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < NR) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w * NR + threadIdx.x];
    sums[threadIdx.x] = t;
  }
  __syncthreads();
}

// Block partial of a per-column sum: part[blockIdx * 16 + k].
__device__ inline void colpart16(double acc, double* red, double* __restrict__ part) {
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < NR) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w * NR + threadIdx.x];
    part[blockIdx.x * NR + threadIdx.x] = t;
  }
}

template <typename Tv>
__global__ __launch_bounds__(NT) void k_dot16(int64_t nrows, const Tv* __restrict__ x,
                                              const Tv* __restrict__ y, double* __restrict__ part) {
  __shared__ double red[NT];
  const int k = threadIdx.x & 15, g = threadIdx.x >> 4;
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 16 + g; i < nrows; i += int64_t(gridDim.x) * 16)
    acc += double(x[i * NR + k]) * double(y[i * NR + k]);
  colpart16(acc, red, part);
}

// Per column: alpha = gamma / delta (0 when gamma == 0; delta <= 0 with
// gamma > 0 flags a non-SPD operator); e += alpha p; s -= alpha q; partials
// of s.s.
template <typename Tv>
__global__ __launch_bounds__(NT) void k_cg_update16(int64_t nrows, Tv* __restrict__ e,
                                                    const Tv* __restrict__ p, Tv* __restrict__ s,
                                                    const Tv* __restrict__ q,
                                                    const double* __restrict__ gpart,
                                                    const double* __restrict__ dpart, int np,
                                                    double* __restrict__ gnew, int* __restrict__ flag) {
  __shared__ double red[NT];
  __shared__ double gam[NR], del[NR], alp[NR];
  colsum16(gpart, np, gam, red);
  colsum16(dpart, np, del, red);
  if (threadIdx.x < NR) {
    double al = 0.0;
    if (gam[threadIdx.x] != 0.0) {
      if (del[threadIdx.x] > 0.0) al = gam[threadIdx.x] / del[threadIdx.x];
      else if (blockIdx.x == 0) atomicOr(flag, 1);
    }
    alp[threadIdx.x] = al;
  }
  __syncthreads();
  const int k = threadIdx.x & 15, g = threadIdx.x >> 4;
  const Tv al = Tv(alp[k]);
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 16 + g; i < nrows; i += int64_t(gridDim.x) * 16) {
    const int64_t idx = i * NR + k;
    e[idx] += al * p[idx];
    const Tv sn = s[idx] - al * q[idx];
    s[idx] = sn;
    acc += double(sn) * double(sn);
  }
  colpart16(acc, red, gnew);
}

// Per column: beta = gamma_new / gamma_old (0 when gamma_old == 0); p = s + beta p.
template <typename Tv>
__global__ __launch_bounds__(NT) void k_cg_pupdate16(int64_t nrows, Tv* __restrict__ p,
                                                     const Tv* __restrict__ s,
                                                     const double* __restrict__ gold,
                                                     const double* __restrict__ gnew, int np) {
  __shared__ double red[NT];
  __shared__ double go[NR], gn[NR];
  colsum16(gold, np, go, red);
  colsum16(gnew, np, gn, red);
  const int k = threadIdx.x & 15, g = threadIdx.x >> 4;
  const Tv beta = Tv(go[k] == 0.0 ? 0.0 : gn[k] / go[k]);
  for (int64_t i = int64_t(blockIdx.x) * 16 + g; i < nrows; i += int64_t(gridDim.x) * 16) {
    const int64_t idx = i * NR + k;
    p[idx] = s[idx] + beta * p[idx];
  }
}

// z_b = M_b^{-1} s_b for every diagonal block b (one workgroup per block,
// at most 128 rows): rows [off[b], off[b+1]) when off is given, else
// [b*stride, (b+1)*stride).  The stored inverses are symmetric.
template <typename Tm, typename Tv>
__global__ __launch_bounds__(NT) void k_bj_apply16(const int* __restrict__ off, int stride,
                                                   const Tm* __restrict__ Minv, int ld,
                                                   const Tv* __restrict__ s, Tv* __restrict__ z) {
  __shared__ Tv sl[128 * NR];
  const int b = blockIdx.x;
  const int s0 = off ? off[b] : b * stride;
  const int n = off ? off[b + 1] - s0 : stride;
  for (int e = threadIdx.x; e < n * NR; e += NT) sl[e] = s[int64_t(s0) * NR + e];
  __syncthreads();
  const Tm* M = Minv + int64_t(b) * ld * ld;
  for (int e = threadIdx.x; e < n * NR; e += NT) {
    const int i = e / NR, k = e % NR;
    Tv acc = Tv(0);
    for (int j = 0; j < n; ++j) acc += Tv(M[int64_t(j) * ld + i]) * sl[j * NR + k];
    z[int64_t(s0 + i) * NR + k] = acc;
  }
}

// ------------------------------------------------------------ triangular solves, 16 columns
// L: N x N column-major lower Cholesky factor; x: N x 16 block.
constexpr int NB = 64;

// x_k = L_kk^{-1} x_k: one wave per column.
__global__ __launch_bounds__(1024) void k_trsv_fwd_diag16(const double* __restrict__ L, int64_t N,
                                                          int64_t k0, double* __restrict__ x) {
  __shared__ double D[NB][NB + 1];
  const int nb = int(min<int64_t>(NB, N - k0));
  const int i = threadIdx.x & 63, k = threadIdx.x >> 6;
  for (int idx = threadIdx.x; idx < nb * nb; idx += 1024)
    D[idx % nb][idx / nb] = L[(k0 + idx % nb) + (k0 + idx / nb) * N];
  __syncthreads();
  double xi = i < nb ? x[(k0 + i) * NR + k] : 0.0;
  for (int c = 0; c < nb; ++c) {
    const double xc = __shfl(xi, c, 64) / D[c][c];
    if (i == c) xi = xc;
    else if (i > c) xi -= D[i][c] * xc;
  }
  if (i < nb) x[(k0 + i) * NR + k] = xi;
}

// x_i -= L_ik x_k for the rows below block k.
__global__ __launch_bounds__(NT) void k_gemv_fwd16(const double* __restrict__ L, int64_t N, int64_t k0,
                                                   double* __restrict__ x) {
  __shared__ double xk[NB * NR];
  const int nb = int(min<int64_t>(NB, N - k0));
  for (int e = threadIdx.x; e < nb * NR; e += NT) xk[e] = x[k0 * NR + e];
  __syncthreads();
  const int64_t idx = int64_t(blockIdx.x) * NT + threadIdx.x;
  const int64_t row = k0 + nb + idx / NR;
  const int k = int(idx % NR);
  if (row >= N) return;
  double s = 0.0;
  for (int c = 0; c < nb; ++c) s += L[row + (k0 + c) * N] * xk[c * NR + k];
  x[row * NR + k] -= s;
}

// x_k = L_kk^{-T} x_k: one wave per column.
__global__ __launch_bounds__(1024) void k_trsv_bwd_diag16(const double* __restrict__ L, int64_t N,
                                                          int64_t k0, double* __restrict__ x) {
  __shared__ double D[NB][NB + 1];
  const int nb = int(min<int64_t>(NB, N - k0));
  const int i = threadIdx.x & 63, k = threadIdx.x >> 6;
  for (int idx = threadIdx.x; idx < nb * nb; idx += 1024)
    D[idx % nb][idx / nb] = L[(k0 + idx % nb) + (k0 + idx / nb) * N];
  __syncthreads();
  double xi = i < nb ? x[(k0 + i) * NR + k] : 0.0;
  for (int c = nb - 1; c >= 0; --c) {
    const double xc = __shfl(xi, c, 64) / D[c][c];
    if (i == c) xi = xc;
    else if (i < c) xi -= D[c][i] * xc;
  }
  if (i < nb) x[(k0 + i) * NR + k] = xi;
}

// x_j -= sum_i L[k0 + i][j] x_{k0 + i} for the rows j above block k.
__global__ __launch_bounds__(NT) void k_gemv_bwd16(const double* __restrict__ L, int64_t N, int64_t k0,
                                                   double* __restrict__ x) {
  __shared__ double xk[NB * NR];
  const int nb = int(min<int64_t>(NB, N - k0));
  for (int e = threadIdx.x; e < nb * NR; e += NT) xk[e] = x[k0 * NR + e];
  __syncthreads();
  const int64_t idx = int64_t(blockIdx.x) * NT + threadIdx.x;
  const int64_t j = idx / NR;
  const int k = int(idx % NR);
  if (j >= k0) return;
  double s = 0.0;
  const double* col = L + j * N + k0;
  for (int i = 0; i < nb; ++i) s += col[i] * xk[i * NR + k];
  x[j * NR + k] -= s;
}

// ------------------------------------------------------------ dispatch helpers
template <typename F>
void dispatch_T16(int T, F&& f) {
  switch (T) {
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    default: throw std::runtime_error("tile products on blocks need a rank of 9 to 64");
  }
}

// f(Tv{}, Te{}) for an operator precision p (vectors FP64 for P64, else FP32).
template <typename F>
void dispatch_prec(int p, F&& f) {
  if (p == P64) f(double{}, double{});
  else if (p == P32) f(float{}, float{});
  else f(float{}, bf16{});
}

}  // namespace

int parts16(int64_t nrows) {
  const int64_t b = (nrows + 63) / 64;
  return int(b < 1 ? 1 : b > 256 ? 256 : b);
}

template <typename F>
void dispatch_dual(bool dual, F&& f) {
  if (dual) f(std::true_type{});
  else f(std::false_type{});
}

void launch_tgemm(H2& h, int tp, int T, const TileSet& ts, const void* tiles, int rr, const void* x,
                  void* partial) {
  const int nb = ts.nrt + ts.nct;
  if (nb == 0) return;
  dispatch_T16(T, [&](auto Tc) {
    constexpr int TT = decltype(Tc)::value;
    dispatch_prec(tp, [&](auto tv, auto te) {
      using Tv = decltype(tv);
      using Te = decltype(te);
      dispatch_dual(ts.dual, [&](auto dc) {
        constexpr bool D = decltype(dc)::value;
        hipLaunchKernelGGL((k_tgemm<TT, Te, Tv, D>), dim3(nb), dim3(32 * TT), 0, h.stream, ts.rtask, ts.nrt,
                           ts.rorder, ts.ctask, ts.corder, static_cast<const Te*>(tiles), ts.brow, ts.bcol,
                           rr, static_cast<const Tv*>(x), static_cast<Tv*>(partial), ts.rslot);
      });
    });
  });
  check_launch("tgemm");
}

void launch_tgemm_eval(H2& h, int p, const TileSet& ts, const void* x, void* partial) {
  const int nb = ts.nrt + ts.nct;
  if (nb == 0) return;
  if (h.nq > 0) throw std::runtime_error("close entries by quadrature are applied from the stored tiles only");
  const StoredNear& sn = h.snear;
  const PointScale ps{h.scale, h.diag, nullptr, nullptr, 0};
  dispatch_kernel(h.kp.kind, h.kp.deriv, [&](auto kc, auto dc) {
    constexpr int KIND = decltype(kc)::value, DERIV = decltype(dc)::value;
    dispatch_dual(ts.dual, [&](auto duc) {
      constexpr bool D = decltype(duc)::value;
      if (p == P64)
        hipLaunchKernelGGL((k_tgemm_eval<double, KIND, DERIV, D>), dim3(nb), dim3(256), 0, h.stream, ts.rtask,
                           ts.nrt, ts.rorder, ts.ctask, ts.corder, ts.brow, ts.bcol, sn.chunk_start, sn.chunk_n,
                           h.pts, h.dim, h.kp, ps, static_cast<const double*>(x), static_cast<double*>(partial),
                           ts.rslot);
      else
        hipLaunchKernelGGL((k_tgemm_eval<float, KIND, DERIV, D>), dim3(nb), dim3(256), 0, h.stream, ts.rtask,
                           ts.nrt, ts.rorder, ts.ctask, ts.corder, ts.brow, ts.bcol, sn.chunk_start, sn.chunk_n,
                           h.pts, h.dim, h.kp, ps, static_cast<const float*>(x), static_cast<float*>(partial),
                           ts.rslot);
    });
  });
  check_launch("tgemm_eval");
}

void launch_tgemm_group(hipStream_t st, int tp, const std::vector<GroupTiles>& items) {
  // one launch per tile width and pass form, at most GROUP_MAX members each
  for (int T : {2, 4, 8})
    for (bool dual : {false, true}) {
      std::vector<const GroupTiles*> sel;
      for (const GroupTiles& it : items)
        if (it.T == T && it.ts->dual == dual && it.ts->nrt + it.ts->nct > 0) sel.push_back(&it);
      for (size_t c0 = 0; c0 < sel.size(); c0 += GROUP_MAX) {
        TgemmGroup G{};
        G.n = int(std::min<size_t>(GROUP_MAX, sel.size() - c0));
        int64_t total = 0;
        for (int m = 0; m < G.n; ++m) {
          const GroupTiles& it = *sel[c0 + m];
          G.start[m] = int(total);
          G.m[m] = TgemmMember{it.ts->rtask, it.ts->rorder, it.ts->ctask, it.ts->corder, it.tiles, it.ts->brow,
                               it.ts->bcol, it.x, it.partial, it.ts->rslot, it.ts->nrt, it.rr};
          total += it.ts->nrt + it.ts->nct;
        }
        G.start[G.n] = int(total);
        if (total > INT32_MAX) throw std::runtime_error("tile-product group grid too large");
        dispatch_T16(T, [&](auto Tc) {
          constexpr int TT = decltype(Tc)::value;
          dispatch_prec(tp, [&](auto tv, auto te) {
            using Tv = decltype(tv);
            using Te = decltype(te);
            dispatch_dual(dual, [&](auto dc) {
              constexpr bool D = decltype(dc)::value;
              hipLaunchKernelGGL((k_tgemm_group<TT, Te, Tv, D>), dim3(unsigned(total)), dim3(32 * TT), 0, st, G);
            });
          });
        });
        check_launch("tgemm_group");
      }
    }
}

void launch_tgemm_eval_group(hipStream_t st, int p, const std::vector<GroupEval>& items) {
  // one launch per kernel family and pass form, at most GROUP_MAX members each
  std::vector<bool> done(items.size(), false);
  for (size_t i0 = 0; i0 < items.size(); ++i0) {
    if (done[i0]) continue;
    std::vector<const GroupEval*> sel;
    if (items[i0].h->nq > 0)
      throw std::runtime_error("close entries by quadrature are applied from the stored tiles only");
    const bool dual = items[i0].ts->dual;
    for (size_t i = i0; i < items.size(); ++i)
      if (!done[i] && items[i].h->kp.kind == items[i0].h->kp.kind && items[i].h->kp.deriv == items[i0].h->kp.deriv &&
          items[i].ts->dual == dual) {
        done[i] = true;
        if (items[i].ts->nrt + items[i].ts->nct > 0) sel.push_back(&items[i]);
      }
    for (size_t c0 = 0; c0 < sel.size(); c0 += GROUP_MAX) {
      TevalGroup G{};
      G.n = int(std::min<size_t>(GROUP_MAX, sel.size() - c0));
      int64_t total = 0;
      for (int m = 0; m < G.n; ++m) {
        const GroupEval& it = *sel[c0 + m];
        const H2& h = *it.h;
        G.start[m] = int(total);
        G.m[m] = TevalMember{it.ts->rtask, it.ts->rorder, it.ts->ctask, it.ts->corder, it.ts->brow, it.ts->bcol,
                             h.snear.chunk_start, h.snear.chunk_n, h.pts, it.x, it.partial, it.ts->rslot,
                             PointScale{h.scale, h.diag, nullptr, nullptr, 0}, h.kp, it.ts->nrt, h.dim};
        total += it.ts->nrt + it.ts->nct;
      }
      G.start[G.n] = int(total);
      if (total > INT32_MAX) throw std::runtime_error("near-field group grid too large");
      dispatch_kernel(sel[c0]->h->kp.kind, sel[c0]->h->kp.deriv, [&](auto kc, auto dc) {
        constexpr int KIND = decltype(kc)::value, DERIV = decltype(dc)::value;
        dispatch_dual(dual, [&](auto duc) {
          constexpr bool D = decltype(duc)::value;
          if (p == P64)
            hipLaunchKernelGGL((k_tgemm_eval_group<double, KIND, DERIV, D>), dim3(unsigned(total)), dim3(256), 0,
                               st, G);
          else
            hipLaunchKernelGGL((k_tgemm_eval_group<float, KIND, DERIV, D>), dim3(unsigned(total)), dim3(256), 0,
                               st, G);
        });
      });
      check_launch("tgemm_eval_group");
    }
  }
}

void launch_reduce16(H2& h, int p, const TileSet& ts, int rr, const void* partial, void* out) {
  if (ts.nrows == 0) return;
  const dim3 grid(ts.nrows, (rr * NR + NT - 1) / NT);
  if (p == P64)
    hipLaunchKernelGGL(k_reduce16<double>, grid, dim3(NT), 0, h.stream, ts.row0, ts.rtp, ts.ctp,
                       ts.nrt, rr, static_cast<const double*>(partial), static_cast<double*>(out));
  else
    hipLaunchKernelGGL(k_reduce16<float>, grid, dim3(NT), 0, h.stream, ts.row0, ts.rtp, ts.ctp,
                       ts.nrt, rr, static_cast<const float*>(partial), static_cast<float*>(out));
  check_launch("reduce16");
}

void launch_gather16(H2& h, int nrhs, const double* user, int ldu, double* tree) {
  hipLaunchKernelGGL(k_gather16, dim3(blocks(int64_t(h.n) * NR, NT)), dim3(NT), 0, h.stream,
                     int64_t(h.n), nrhs, h.perm, user, ldu, tree);
  check_launch("gather16");
}

void launch_scatter16(H2& h, int nrhs, const double* tree, double* user, int ldu) {
  hipLaunchKernelGGL(k_scatter16, dim3(blocks(int64_t(h.n) * NR, NT)), dim3(NT), 0, h.stream,
                     int64_t(h.n), nrhs, h.perm, tree, user, ldu);
  check_launch("scatter16");
}

void launch_leaf_up16(H2& h, int p, const void* x, void* xhat) {
  dispatch_prec(p, [&](auto tv, auto te) {
    using Tv = decltype(tv);
    using Te = decltype(te);
    hipLaunchKernelGGL((k_leaf_up16<Te, Tv>), dim3(h.nleaf), dim3(NT), 0, h.stream, h.leaf_off,
                       static_cast<const Te*>(h.prec[p].Qr), h.r, static_cast<const Tv*>(x),
                       static_cast<Tv*>(xhat));
  });
  check_launch("leaf_up16");
}

void launch_leaf_down16(H2& h, int p, const void* yhat, const void* near_y, void* out, double alpha,
                        const void* add, double beta) {
  dispatch_prec(p, [&](auto tv, auto te) {
    using Tv = decltype(tv);
    using Te = decltype(te);
    hipLaunchKernelGGL((k_leaf_down16<Te, Tv>), dim3(h.nleaf), dim3(NT), 0, h.stream, h.leaf_off,
                       static_cast<const Te*>(h.prec[p].Qr), h.r, static_cast<const Tv*>(yhat),
                       static_cast<const Tv*>(near_y), h.snear.chunk_base, static_cast<Tv*>(out), alpha,
                       static_cast<const Tv*>(add), beta);
  });
  check_launch("leaf_down16");
}

void launch_transfer_up16(H2& h, int p, int d, const void* xchild, void* xpar) {
  dispatch_T16(h.T, [&](auto Tc) {
    constexpr int TT = decltype(Tc)::value;
    dispatch_prec(p, [&](auto tv, auto te) {
      using Tv = decltype(tv);
      using Te = decltype(te);
      hipLaunchKernelGGL((k_transfer16<TT, MODE_UP, Te, Tv>), dim3(1 << d), dim3(32 * TT), 0, h.stream,
                         static_cast<const Te*>(h.prec[p].E), (1 << (d + 1)) - 1, h.r,
                         static_cast<const Tv*>(xchild), static_cast<Tv*>(xpar), static_cast<const Tv*>(nullptr));
    });
  });
  check_launch("transfer_up16");
}

void launch_transfer_down16(H2& h, int p, int d, const void* ypar, void* ychild, const void* addend) {
  dispatch_T16(h.T, [&](auto Tc) {
    constexpr int TT = decltype(Tc)::value;
    dispatch_prec(p, [&](auto tv, auto te) {
      using Tv = decltype(tv);
      using Te = decltype(te);
      hipLaunchKernelGGL((k_transfer16<TT, MODE_DOWN, Te, Tv>), dim3(2 << d), dim3(32 * TT), 0, h.stream,
                         static_cast<const Te*>(h.prec[p].E), (1 << (d + 1)) - 1, h.r,
                         static_cast<const Tv*>(ypar), static_cast<Tv*>(ychild), static_cast<const Tv*>(addend));
    });
  });
  check_launch("transfer_down16");
}

void launch_near_pad16(H2& h, int p, const void* x, void* xc) {
  if (p == P64)
    hipLaunchKernelGGL(k_near_pad16<double>, dim3(h.nleaf), dim3(NT), 0, h.stream, h.leaf_off,
                       h.snear.chunk_base, static_cast<const double*>(x), static_cast<double*>(xc));
  else
    hipLaunchKernelGGL(k_near_pad16<float>, dim3(h.nleaf), dim3(NT), 0, h.stream, h.leaf_off,
                       h.snear.chunk_base, static_cast<const float*>(x), static_cast<float*>(xc));
  check_launch("near_pad16");
}

void launch_dot16(H2& h, int p, int64_t nrows, const void* x, const void* y, double* part) {
  const int np = parts16(nrows);
  if (p == P64)
    hipLaunchKernelGGL(k_dot16<double>, dim3(np), dim3(NT), 0, h.stream, nrows, static_cast<const double*>(x),
                       static_cast<const double*>(y), part);
  else
    hipLaunchKernelGGL(k_dot16<float>, dim3(np), dim3(NT), 0, h.stream, nrows, static_cast<const float*>(x),
                       static_cast<const float*>(y), part);
  check_launch("dot16");
}

void launch_cg_update16(H2& h, int p, int64_t nrows, void* e, const void* pv, void* s, const void* q,
                        const double* gpart, const double* dpart, double* gnew) {
  const int np = parts16(nrows);
  if (p == P64)
    hipLaunchKernelGGL(k_cg_update16<double>, dim3(np), dim3(NT), 0, h.stream, nrows, static_cast<double*>(e),
                       static_cast<const double*>(pv), static_cast<double*>(s), static_cast<const double*>(q),
                       gpart, dpart, np, gnew, h.flags);
  else
    hipLaunchKernelGGL(k_cg_update16<float>, dim3(np), dim3(NT), 0, h.stream, nrows, static_cast<float*>(e),
                       static_cast<const float*>(pv), static_cast<float*>(s), static_cast<const float*>(q),
                       gpart, dpart, np, gnew, h.flags);
  check_launch("cg_update16");
}

void launch_cg_pupdate16(H2& h, int p, int64_t nrows, void* pv, const void* s, const double* gold,
                         const double* gnew) {
  const int np = parts16(nrows);
  if (p == P64)
    hipLaunchKernelGGL(k_cg_pupdate16<double>, dim3(np), dim3(NT), 0, h.stream, nrows, static_cast<double*>(pv),
                       static_cast<const double*>(s), gold, gnew, np);
  else
    hipLaunchKernelGGL(k_cg_pupdate16<float>, dim3(np), dim3(NT), 0, h.stream, nrows, static_cast<float*>(pv),
                       static_cast<const float*>(s), gold, gnew, np);
  check_launch("cg_pupdate16");
}

void launch_bj_apply16(H2& h, int p, int k, const void* s, void* z) {
  const bool fine = k == 1;
  const int d = h.level_depth(k);
  const int nb = fine ? h.nleaf : (1 << d);
  const int* off = fine ? h.leaf_off : nullptr;
  const int ld = fine ? h.bj_ld : h.r;
  const size_t eb = p == P64 ? 8 : 4;
  const char* base = static_cast<const char*>(fine ? h.bj_fine[p == P64 ? P64 : P32]
                                                   : h.bj_coarse[p == P64 ? P64 : P32]);
  if (!fine) base += size_t((1 << d) - 1) * h.r * h.r * eb;
  if (p == P64)
    hipLaunchKernelGGL((k_bj_apply16<double, double>), dim3(nb), dim3(NT), 0, h.stream, off, h.r,
                       reinterpret_cast<const double*>(base), ld, static_cast<const double*>(s),
                       static_cast<double*>(z));
  else
    hipLaunchKernelGGL((k_bj_apply16<float, float>), dim3(nb), dim3(NT), 0, h.stream, off, h.r,
                       reinterpret_cast<const float*>(base), ld, static_cast<const float*>(s),
                       static_cast<float*>(z));
  check_launch("bj_apply16");
}

void launch_chol_solve16(H2& h, const double* L, int64_t N, double* x) {
  for (int64_t k0 = 0; k0 < N; k0 += NB) {
    hipLaunchKernelGGL(k_trsv_fwd_diag16, dim3(1), dim3(1024), 0, h.stream, L, N, k0, x);
    const int64_t below = N - k0 - std::min<int64_t>(NB, N - k0);
    if (below > 0)
      hipLaunchKernelGGL(k_gemv_fwd16, dim3(blocks(below * NR, NT)), dim3(NT), 0, h.stream, L, N, k0, x);
  }
  const int64_t last = ((N - 1) / NB) * NB;
  for (int64_t k0 = last; k0 >= 0; k0 -= NB) {
    hipLaunchKernelGGL(k_trsv_bwd_diag16, dim3(1), dim3(1024), 0, h.stream, L, N, k0, x);
    if (k0 > 0)
      hipLaunchKernelGGL(k_gemv_bwd16, dim3(blocks(k0 * NR, NT)), dim3(NT), 0, h.stream, L, N, k0, x);
  }
  check_launch("chol_solve16");
}

}  // namespace h2mg
