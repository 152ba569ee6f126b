// Internal definition of the H2 handle and the launchers of every kernel.
//
// Numbering.  Cluster j at depth d has the global id gid = 2^d - 1 + j.
// Coefficient vectors of all depths share one buffer indexed gid * r.
// Stored r x r blocks (far couplings S and projected close blocks Pi of
// every depth) live in one array of tiles (device_common.h), upper triangle
// only (row cluster <= column cluster): the operators are symmetric, so a
// stored off-diagonal block B contributes B x_t to row s and B^T x_s to row t.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "device_common.h"
#include "h2mg.h"
#include "plan.h"

namespace h2mg {

const char* last_error_cstr();
void clear_error();

enum Prec { P64 = 0, P32 = 1, P16 = 2 };   // FP64, FP32, BF16 operator storage
constexpr int MULTI_NR = 16;               // columns of a multi-vector block
inline size_t elem_bytes(int p) { return p == P64 ? 8 : p == P32 ? 4 : 2; }

// Device allocation owned by a handle.
struct Arena {
  std::vector<std::pair<void*, size_t>> ptrs;
  size_t bytes = 0;
  void* alloc(size_t nbytes);          // throws std::bad_alloc on failure
  template <typename T> T* make(size_t n) { return static_cast<T*>(alloc(n * sizeof(T))); }
  void release(void* p);
  ~Arena();
};

// A symmetric block operator over one depth: tasks are runs of at most C
// stored blocks of one block row, processed by one wave each.
struct View {
  int depth = 0;
  int ntasks = 0;
  std::vector<int> task;               // host: 3 ints per task (row gid, b0, b1)
  int* row_task_ptr = nullptr;         // device: 2^depth + 1, offsets into this view's tasks
  int* col_ptr = nullptr;              // device: 2^depth + 1
  int* col_blk = nullptr;              // device: stored off-diagonal blocks by column
  int slot_base = 0;                   // first column-contribution slot of this view
};

// One GEMV launch over the concatenated tasks of several views.
struct Launch {
  int ntasks = 0;
  int64_t nblocks = 0;                 // stored blocks streamed by one launch
  int* task = nullptr;                 // device
  std::vector<int> base;               // task base of each view in the list
};

// Optional per-kernel timing with HIP events on the handle's stream.
enum KStatKind {
  KS_GEMV64 = 0, KS_GEMV32 = 1, KS_GEMV16 = 2, KS_NEAR64 = 3, KS_NEAR32 = 4,
  KS_NEARST64 = 5,                     // block GEMV over the stored near-field tiles
  KS_NEAR16 = 6,                       // both passes of the 16-vector product over the near tiles
  KS_COUNT = 7
};
struct KStat {
  int64_t launches = 0;
  double ms = 0.0;
  double bytes = 0.0;                  // algorithmic bytes (GEMV) or kernel evaluations (near)
  std::vector<std::pair<int, int>> pending;   // event indices not yet read
  std::vector<double> pending_bytes;
};

// Close leaf pairs (s <= t) for the on-the-fly near field.
struct NearField {
  int npairs = 0;
  int ntasks = 0;
  int* task = nullptr;                 // device: (row leaf, p0, p1)
  int* pair_col = nullptr;             // device: column leaf of each pair
  int* row_task_ptr = nullptr;         // device: nleaf + 1
  int* col_ptr = nullptr;              // device: nleaf + 1
  int* col_pair = nullptr;             // device: off-diagonal pairs by column leaf
  int ld = 0;                          // padded leaf length of partial buffers
};

// Stored near field (optional, FP64).  Every leaf is cut into chunks of at
// most 64 consecutive points (chunk k of leaf s covers local positions
// 64k .. 64k+63), and the close leaf pairs (s <= t) into 64 x 64 tiles
// between chunks: all chunk pairs of an off-diagonal leaf pair, the upper
// triangle of chunk pairs of a diagonal one (diagonal tiles stored whole,
// with the shift on their diagonal).  Padding rows and columns are zero.
// Vectors on chunks are padded: position i of leaf s is element
// chunk_base[s] * 64 + i; when every leaf holds a multiple of 64 points this
// is the tree order itself and no padding copy is made.
struct StoredNear {
  bool planned = false;                // chunks, tile lists and tasks built
  bool ready = false;                  // tiles stored
  bool identity = false;               // padded chunk order == tree order
  int nchunk = 0;
  int ntasks = 0;
  int64_t nblocks = 0;
  int nslot = 0;
  int* chunk_base = nullptr;           // device: nleaf + 1
  int* chunk_start = nullptr;          // device: first tree position of each chunk
  int* chunk_n = nullptr;              // device: points in each chunk
  int* blk_row = nullptr;              // device: row chunk of each tile
  int* blk_col = nullptr;              // device: column chunk of each tile
  int* blk_slot = nullptr;             // device: column-contribution slot (-1: diagonal)
  int* task = nullptr;                 // device: (row chunk, b0, b1), at most 16 tiles
  int* row_task_ptr = nullptr;         // device: nchunk + 1
  int* col_ptr = nullptr;              // device: nchunk + 1
  double* tiles = nullptr;             // nblocks tiles of 64 x 64 (T = 8 layout)
  float* tiles32 = nullptr;            // FP32 copy (close entries by quadrature only)
  float* xc32 = nullptr;               // nchunk * 64 padded FP32 input (zero padding; null when identity)
  double* partial = nullptr;           // ntasks * 64
  double* colpart = nullptr;           // nslot * 64
  double* xc = nullptr;                // nchunk * 64 (padded input; null when identity)
  double* yc = nullptr;                // nchunk * 64 (near-field product)
  std::vector<int> brow_h, bcol_h;     // host copies of blk_row / blk_col
  std::vector<void*> owned;            // device allocations of this structure
};

// One set of stored tiles multiplied at once with a block of MULTI_NR
// vectors: row-pass tasks (block row, i0, i1) over `rorder` (tile ids by
// block row), column-pass tasks (block column, i0, i1) over `corder` (the
// off-diagonal tile ids by block column), at most `run` tiles per task, and
// per-row task ranges for the reduce.  Rows are gids for coupling and
// projected close tiles, chunks for near-field tiles.
struct TileSet {
  int nrt = 0, nct = 0;                // row-pass and column-pass tasks
  int* rtask = nullptr;                // device: 3 ints per task
  int* rorder = nullptr;
  int* ctask = nullptr;
  int* corder = nullptr;
  int* rtp = nullptr;                  // device: rows + 1 row-pass task offsets
  int* ctp = nullptr;                  // device: rows + 1 column-pass task offsets
  const int* brow = nullptr;           // device: block row / column of every tile
  const int* bcol = nullptr;
  int row0 = 0, nrows = 0;             // rows the reduce writes
  int run = 0;                         // tiles per task
  double tuned_ms = 0.0;               // measured product + reduce time (tuned sets)
  int64_t ntiles = 0;                  // tiles in the set (each read by the row pass)
  int64_t nctiles = 0;                 // off-diagonal tiles (read again by the column pass)
  // read-once form: no column-pass tasks; each row task also writes the
  // transposed product of its off-diagonal tiles to slot rslot[i] (i: place
  // in rorder; -1 for diagonal tiles), slots ordered by block column (ctp
  // counts tiles, corder lists them)
  bool dual = false;
  int* rslot = nullptr;                // device
  int64_t nslots() const { return int64_t(nrt) + (dual ? nctiles : nct); }
};

// Buffers and task sets of the products and cycles on blocks of MULTI_NR
// vectors (built on first use).
struct BlockWork {
  bool ready = false;
  bool coarse_ready = false;
  bool near_ready = false;
  int run = 8;                         // tiles per task
  TileSet fine;                        // couplings S of every depth
  std::vector<TileSet> coarse;         // by depth d: S of depths d_top..d and Pi of depth d
  TileSet near;                        // stored near-field tiles
  void* partial = nullptr;             // max tasks x rows x NR (sized for FP64)
  int64_t partial_elems = 0;
  void* xall = nullptr;                // ngid * r x NR (FP64 size; reused by FP32)
  void* yall = nullptr;
  double* xc64 = nullptr;              // nchunk * 64 x NR (null when the chunk order is the tree order)
  float* xc32 = nullptr;
  void* yc = nullptr;                  // nchunk * 64 x NR
  double* bx = nullptr;                // n x NR staging blocks of the product entry point
  double* by = nullptr;
  std::vector<void*> owned;
};

struct PrecData {                      // operator storage in one precision
  bool ready = false;
  void* Qr = nullptr;                  // N x r row-major, tree order
  void* Qc = nullptr;                  // per leaf: r x n_leaf (column j contiguous)
  void* E = nullptr;                   // transfer tiles by child gid
  void* blk = nullptr;                 // S and Pi tiles by block id
};

struct H2 {
  Plan plan;
  KernelParams kp{};
  h2mg_kernel kernel{};                // as given to the build
  h2mg_build_opts opts{};
  int n = 0, dim = 0, r = 0, m = 0, L = 0, d_top = -1, T = 1;
  int nleaf = 0, leaf_max = 0;
  int ngid = 0;                        // 2^(L+1) - 1
  hipStream_t stream = nullptr;
  Arena arena;

  // geometry
  double* pts = nullptr;               // tree-ordered points, N x dim
  int64_t* perm = nullptr;             // tree position -> user index
  int* leaf_off = nullptr;             // nleaf + 1
  double* cbox = nullptr;              // per gid: dim centres
  double* hbox = nullptr;              // per gid: dim floored half-widths
  double* nodes1d = nullptr;           // m Chebyshev nodes
  double* scale = nullptr;             // per point s (tree order), or null: s = 1
  double* diag = nullptr;              // per point d (tree order), or null: d = shift
  double* R = nullptr;                 // per gid r x r (setup only, freed after)
  // close entries by quadrature (tree order; null: point kernel values):
  // nq sub-points per point (nq x dim) and their weights
  double* qy = nullptr;
  double* qu = nullptr;
  int nq = 0;

  // stored blocks: S of depth d in [s_first[d], s_first[d] + s_count[d]),
  // Pi of depth d in [p_first[d], p_first[d] + p_count[d])
  int nblk = 0;
  std::vector<int> blk_row_h, blk_col_h;   // gids
  std::vector<int> blk_slot_h;
  int* blk_row = nullptr;
  int* blk_col = nullptr;
  int* blk_slot = nullptr;             // column-contribution slot of each stored block
  int nslot = 0;
  std::vector<int> s_first, s_count, p_first, p_count;
  std::vector<View> sview, pview;
  NearField near;
  StoredNear snear;
  BlockWork blk16;
  PrecData prec[3];

  // launches: fine apply (S of all depths), coarse apply at depth d
  Launch fine_launch;
  std::vector<Launch> coarse_launch;   // indexed by depth
  int max_tasks = 0;

  // workspace (sized for FP64; reused by FP32 kernels)
  double* xall = nullptr;              // ngid * r
  double* yall = nullptr;
  double* partial = nullptr;           // max_tasks * r
  double* colpart = nullptr;           // nblk * r
  double* near_partial = nullptr;      // near.ntasks * ld
  double* near_colpart = nullptr;      // near.npairs * ld
  double* vtree = nullptr;             // N scratch (tree order)
  double* vtree2 = nullptr;

  // multigrid
  bool mg_built = false;
  int levels = 1;
  int64_t Nl = 0;                      // coarsest size
  double* chol = nullptr;              // Nl x Nl column-major, lower factor
  int* flags = nullptr;                // device flags (0: not SPD, 1: non-finite)
  double* dot_part = nullptr;          // reduction partials (several slots)
  std::vector<double> history;

  // block-Jacobi smoother: inverse diagonal blocks per level and precision
  bool bj_built[3] = {false, false, false};
  int bj_ld = 0;                       // padded leaf block size of the finest level
  void* bj_fine[3] = {nullptr, nullptr, nullptr};   // nleaf blocks of bj_ld^2
  void* bj_coarse[3] = {nullptr, nullptr, nullptr}; // per gid r^2 (depths d_top+1..L)

  // tile products on 16-column blocks: task run lengths chosen by timing
  // candidates when the block work is built
  bool autotune = false;

  // cycle graphs: with graphs on, the first cycle of a solve is captured
  // (on a private stream) and every cycle is one graph launch
  bool graphs = false;
  hipStream_t capture_stream = nullptr;

  // kernel timing
  bool timing = false;
  std::vector<hipEvent_t> events;
  int next_event = 0;
  KStat kstat[KS_COUNT];
  int64_t near_evals = 0;              // kernel evaluations of one near-field pass
  ~H2();
  int take_event();                    // index of a free event (creates on demand)
  void time_begin(int& ev);            // record a start event when timing
  void time_end(int kind, int ev, double bytes);
  void flush_timing();                 // synchronise and accumulate pending events

  int64_t level_size(int k) const {    // k = 1..levels
    if (k == 1) return n;
    const int d = L - k + 2;
    return (int64_t(1) << d) * r;
  }
  int level_depth(int k) const { return L - k + 2; }
};

// The per-point data of the close entries (scale, diagonal, quadrature).
inline PointScale near_scale(const H2& h) { return PointScale{h.scale, h.diag, h.qy, h.qu, h.nq}; }
// Whether the fine product in precision p reads the stored near-field tiles
// (FP64 tiles when stored; the FP32 copy exists only for quadrature).
inline bool near_stored_for(const H2& h, int p) {
  return h.snear.ready && (p == P64 || h.snear.tiles32 != nullptr);
}

// ------------------------------------------------------------ setup kernels
void launch_leaf_basis_qr(H2& h);                 // Q (FP64), R of leaves
void launch_transfer_qr(H2& h, int d);            // E of depth d+1, R of depth d
void launch_couplings(H2& h, int d);              // S tiles of depth d
void launch_pi_leaf(H2& h);                       // Pi tiles of depth L
void launch_pi_upper(H2& h, int d, const int* child_map);   // Pi tiles of depth d < L
void launch_assemble_dense(H2& h, double* A, int64_t lda);  // depth d_top blocks
void launch_assemble_kernel_dense(H2& h, double* A, int64_t lda);  // no far blocks
void launch_potrf(H2& h, double* A, int64_t N);   // blocked Cholesky, sets flags[0]
void launch_cast_precision(H2& h, int p);         // FP64 -> FP32 / BF16 copies
void launch_near_tiles(H2& h);                    // stored near-field tiles (FP64)
// Inverses of the block-Jacobi blocks: leaf blocks K_ss + shift (FP64) and the
// projected diagonal blocks of depths d_top+1..L (FP64); sets flags[0] on a
// non-positive pivot.
void launch_bj_inverse_fine(H2& h, double* out, int ld);
void launch_bj_inverse_coarse(H2& h, int d, const int* diag_blk, double* out);

// ------------------------------------------------------------ apply kernels
// All vectors are in the precision's vector type: double (P64) or float.
void launch_gemv(H2& h, int p, const Launch& l, const void* x_all);
// For every depth d in [d0, d1]: y_d = sum of the task partials and column
// contributions of views v0[d] (and v1[d] when not null) of that depth,
// written at out + offset of depth d (gid-indexed buffer) -- or, for depth
// d1 only, at out_last when it is not null.  base0/base1: task bases of the
// views in the launch that produced the partials.
void launch_reduce(H2& h, int p, int d0, int d1, const View* const* v0, const int* base0,
                   const View* const* v1, const int* base1, void* out, void* out_last);
void launch_transfer_up(H2& h, int p, int d, const void* xchild, void* xpar);
void launch_transfer_down(H2& h, int p, int d, const void* ypar, void* ychild,
                          const void* addend);
void launch_leaf_up(H2& h, int p, const void* xtree, void* xhat);
void launch_near(H2& h, int p, const void* xtree);
// Stored near field: snear.yc = D x over the chunk-padded layout, FP64
// tiles and vectors (p = P64) or the FP32 tile copy with FP32 vectors.
void launch_near_stored(H2& h, int p, const void* xtree);
// FP32 copy of the stored near-field tiles (snear.tiles32).
void launch_cast_near_tiles(H2& h);
// tree[i, :] = user[perm[i], :] for rows of `width` doubles.
void launch_gather_rows(H2& h, int width, const double* user, double* tree);
// out = alpha * Q yhat + beta * add (tree order).
void launch_leaf_down(H2& h, int p, const void* yhat, void* out, double alpha, const void* add,
                      double beta);
// out[idx] = alpha * (Q yhat + near + diag * xin) + beta * add[idx], idx = tree
// position or perm[tree position] when to_user (the diag term only with a
// per-point diagonal and the near field evaluated).  The near part comes from the stored
// near field (snear.yc) for FP64 when it is ready, else from the on-the-fly
// partials.
void launch_fine_reduce(H2& h, int p, const void* yhat, void* out, bool to_user,
                        double alpha, const void* add, double beta, const void* xin);

// ------------------------------------------------------------ blocks of 16 vectors
// Vectors of precision p: double for P64, float otherwise; tiles of the
// operator precision.  Row-major blocks (entry (i, k) at i * 16 + k).
int parts16(int64_t nrows);            // partial sums of a per-column dot
// tp: precision of the tiles (FP64 tiles with FP64 vectors, FP32 or BF16
// tiles with FP32 vectors).
void launch_tgemm(H2& h, int tp, int T, const TileSet& ts, const void* tiles, int rr, const void* x,
                  void* partial);
// Near-field tile products with the tiles evaluated from the points (near
// chunk plan of h.snear; vectors of precision p, chunk-padded).
void launch_tgemm_eval(H2& h, int p, const TileSet& ts, const void* x, void* partial);
void launch_reduce16(H2& h, int p, const TileSet& ts, int rr, const void* partial, void* out);

// Tile products of several independent problems in one launch (kernel
// arguments; member m owns blocks [start[m], start[m+1]) of the grid).
constexpr int GROUP_MAX = 16;
struct TgemmMember {
  const int* rtask;
  const int* rorder;
  const int* ctask;
  const int* corder;
  const void* tiles;
  const int* brow;
  const int* bcol;
  const void* x;
  void* partial;
  const int* rslot;
  int nrt;
  int rr;
};
struct TgemmGroup {
  int n;
  int start[GROUP_MAX + 1];
  TgemmMember m[GROUP_MAX];
};
struct TevalMember {
  const int* rtask;
  const int* rorder;
  const int* ctask;
  const int* corder;
  const int* brow;
  const int* bcol;
  const int* chunk_start;
  const int* chunk_n;
  const double* pts;
  const void* x;
  void* partial;
  const int* rslot;
  PointScale ps;
  KernelParams kp;
  int nrt;
  int dim;
};
struct TevalGroup {
  int n;
  int start[GROUP_MAX + 1];
  TevalMember m[GROUP_MAX];
};
// One problem's share of a group launch: its task set over stored tiles of
// width T (precision tp of the launch), or over near-field tiles evaluated
// from its points.
struct GroupTiles {
  int T;
  const TileSet* ts;
  const void* tiles;
  int rr;
  const void* x;
  void* partial;
};
struct GroupEval {
  const H2* h;
  const TileSet* ts;
  const void* x;
  void* partial;
};
void launch_tgemm_group(hipStream_t st, int tp, const std::vector<GroupTiles>& items);
void launch_tgemm_eval_group(hipStream_t st, int p, const std::vector<GroupEval>& items);
void launch_gather16(H2& h, int nrhs, const double* user, int ldu, double* tree);
void launch_scatter16(H2& h, int nrhs, const double* tree, double* user, int ldu);
void launch_leaf_up16(H2& h, int p, const void* x, void* xhat);
// out = alpha * (Q yhat + near) + beta * add (tree order; yhat, near may be null)
void launch_leaf_down16(H2& h, int p, const void* yhat, const void* near_y, void* out, double alpha,
                        const void* add, double beta);
void launch_transfer_up16(H2& h, int p, int d, const void* xchild, void* xpar);
void launch_transfer_down16(H2& h, int p, int d, const void* ypar, void* ychild, const void* addend);
void launch_near_pad16(H2& h, int p, const void* x, void* xc);
void launch_dot16(H2& h, int p, int64_t nrows, const void* x, const void* y, double* part);
void launch_cg_update16(H2& h, int p, int64_t nrows, void* e, const void* pv, void* s, const void* q,
                        const double* gpart, const double* dpart, double* gnew);
void launch_cg_pupdate16(H2& h, int p, int64_t nrows, void* pv, const void* s, const double* gold,
                         const double* gnew);
void launch_bj_apply16(H2& h, int p, int k, const void* s, void* z);
void launch_chol_solve16(H2& h, const double* L, int64_t N, double* x);   // in place, FP64

// ------------------------------------------------------------ boundary elements
// Per triangle (vertex rows V, index triples T): centroid y (nt x 3), scale
// s = sqrt(area), diagonal d = self-potential / (4 pi).
void launch_bem_panels(hipStream_t st, int64_t nt, const double* V, const int64_t* T, double* y,
                       double* s, double* d);
// Radon's seven-point rule per triangle: points qy (nt x 7 x 3) and weights
// qu (nt x 7) times sqrt(area), for the quadrature of the close entries.
void launch_bem_quadrature7(hipStream_t st, int64_t nt, const double* V, const int64_t* T, double* qy,
                            double* qu);
// f_i = s_i / (4 pi |y_i - x0|) (x0: 3 host doubles).
void launch_bem_rhs(hipStream_t st, int64_t n, const double* y, const double* x0, const double* s,
                    double* f);
// f_i = s_i * sum_k c_k h_k(y_i), c: 9 host doubles for the harmonic basis
// 1, x, y, z, xy, yz, zx, x^2 - y^2, x^2 + y^2 - 2 z^2.
void launch_bem_harmonic(hipStream_t st, int64_t n, const double* y, const double* coeffs, const double* s,
                         double* f);
// out_i = x_i / s_i.
void launch_div(hipStream_t st, int64_t n, const double* x, const double* s, double* out);

// ------------------------------------------------------------ vector kernels
void launch_gather(H2& h, const double* user, double* tree);     // tree[i] = user[perm[i]]
void launch_scatter(H2& h, const double* tree, double* user);    // user[perm[i]] = tree[i]
void launch_copy(H2& h, int p, const void* src, void* dst, int64_t n);
void launch_zero(H2& h, int p, void* dst, int64_t n);
void launch_cast(H2& h, int pdst, void* dst, int psrc, const void* src, int64_t n);
// y = a*x + b*y  (vector type of p)
void launch_axpby(H2& h, int p, int64_t n, double a, const void* x, double b, void* y);
// Partial sums of x.y (FP64 accumulation) into part[0 .. nparts(n)).
int dot_parts(int64_t n);
void launch_dot(H2& h, int p, int64_t n, const void* x, const void* y, double* part);
// CG step halves; scalars are read from partial-sum arrays on the device.
void launch_cg_update(H2& h, int p, int64_t n, void* e, const void* pv, void* s,
                      const void* q, const double* gamma_part, const double* delta_part,
                      double* gamma_new_part);
void launch_cg_pupdate(H2& h, int p, int64_t n, void* pv, const void* s,
                       const double* gamma_old_part, const double* gamma_new_part);
void launch_chol_solve(H2& h, const double* L, int64_t N, double* x);   // in place
void launch_check_finite(H2& h, int p, int64_t n, const void* x);      // sets flags[1]
// Gradient helpers (tree-ordered points h.pts, n x dim).
void launch_scatter_rows(H2& h, const double* tree, double* user);     // user[perm[i], :] = tree[i, :]
void launch_coord_mul(H2& h, int a, const double* x, double* w);       // w = x * p[:, a]
// grad[perm[i], a] = -2 scale x_i (p[i, a] v_i - u_i)
void launch_coord_grad(H2& h, int a, double scale, const double* x, const double* v, const double* u,
                       double* grad);
// z = M^{-1} s on one level (block-Jacobi): level 1 uses the leaf blocks,
// level k >= 2 the r x r blocks of its depth.
void launch_bj_apply(H2& h, int p, int k, const void* s, void* z);

}  // namespace h2mg
