// Internal plan state shared by the translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "common.h"

namespace bemfmm {

constexpr int NBITS = 21;        // Morton bits per axis
constexpr int MAX_LEVEL = 21;
constexpr int N_OFFSETS = 343;   // 7^3 translation-vector slots, (dx+3)*49+(dy+3)*7+(dz+3)
constexpr int NEAR_RULE = 8;     // near-singular rule: 8 x 8 collapsed Gauss points
constexpr int SELF_RULE = 64;    // self terms: Gauss points per edge angle
constexpr int MAX_DIRECT = 3;    // levels above the leaves reached by direct translations
constexpr int64_t DIRECT_BYTES = int64_t(1) << 30;  // operator memory cap per direct depth

// Multipole-to-local by rotation (point-and-shoot): pairs per tile, LDS row
// stride of a tile's expansions, largest order (its LDS holds 2 (p+1)^2 rows)
constexpr int ROT_CT = 16;
constexpr int ROT_LD = ROT_CT + 1;
constexpr int ROT_MAXP = 23;
// Table layouts: real rotation blocks of degrees 0..p one after another
// ((2n+1)^2 each, block n at rot_doff(n)); coaxial blocks of orders
// m = -p..p one after another ((p+1-|m|)^2 each, block m at rot_coff(p, m))
__host__ __device__ constexpr int rot_doff(int n) { return n * (4 * n * n - 1) / 3; }
__host__ __device__ constexpr int rot_dsz(int p) { return rot_doff(p + 1); }
__host__ __device__ constexpr int rot_s2(int x) { return x * (x + 1) * (2 * x + 1) / 6; }
__host__ __device__ constexpr int rot_csz(int p) { return (p + 1) * (p + 1) + 2 * rot_s2(p); }
__host__ __device__ constexpr int rot_coff(int p, int m) {
  return m <= 0 ? rot_s2(p + m) : 2 * rot_s2(p) + (p + 1) * (p + 1) - rot_s2(p + 1 - m);
}
// Matrix-core layout of the same blocks, as the rotation kernel reads them:
// a block of s rows and columns in 16-row tiles (rot_nmt) and 4-column
// k steps (rot_nks), each (tile, step) a chunk of 64 values in lane order
// (lane = row + 16 column-in-step), zero outside the block; block n of the
// degree tables at rot_dpoff(n), block m of the coaxial tables at
// rot_cpoff(p, m).
__host__ __device__ constexpr int rot_nmt(int s) { return (s + 15) >> 4; }
__host__ __device__ constexpr int rot_nks(int s) { return (s + 3) >> 2; }
__host__ __device__ constexpr int rot_dpoff(int n) {
  int o = 0;
  for (int j = 0; j < n; ++j) o += rot_nmt(2 * j + 1) * rot_nks(2 * j + 1) * 64;
  return o;
}
__host__ __device__ constexpr int rot_dpsz(int p) { return rot_dpoff(p + 1); }
__host__ __device__ constexpr int rot_cpoff(int p, int m) {
  int o = 0;
  for (int mm = -p; mm < m; ++mm) {
    const int s = p + 1 - (mm < 0 ? -mm : mm);
    o += rot_nmt(s) * rot_nks(s) * 64;
  }
  return o;
}
__host__ __device__ constexpr int rot_cpsz(int p) { return rot_cpoff(p, p + 1); }

// Device allocation registry: every buffer a problem owns.
struct DevArena {
  std::vector<void*> ptrs;
  int64_t bytes = 0;
  int alloc(void** p, size_t n);  // returns 0 or BEM_E_OOM
  void release();
};

// A grouped gather-GEMM-scatter job: for pair t in group g,
//   dst[pair_dst[t]] += op_g * src[pair_src[t]]
// op_g is a (rows x cols) complex matrix, row-major.  Tiles enumerate
// (group, first pair, first row) blocks of up to ct pairs x 64 rows.
template <typename R>
struct GroupedOp {
  int rows = 0, cols = 0;          // output / input coefficient counts
  int n_pairs = 0, n_tiles = 0;
  int ct = 64, ct_adj = 64;        // pairs per tile (16, 32, 64 or 128)
  int* pair_dst = nullptr;         // device, grouped by g, ascending dst within g
  int* pair_src = nullptr;
  int* tile_group = nullptr;       // device, per tile
  int* tile_pair0 = nullptr;
  int* tile_npairs = nullptr;
  int* tile_row0 = nullptr;
  int* group_slot = nullptr;       // device: group id -> matrix slot
  // device, group id -> input coefficients the forward product reads (null:
  // all); the stored operator is zero beyond them, so the adjoint (which
  // reads every row of the stored conjugate transpose) stays its transpose
  int* group_kc = nullptr;
  cplx<R>* mats = nullptr;         // device: n_slots x rows x cols
  // M2L only: the conjugate transposes (n_slots x cols x rows), so that the
  // adjoint product runs the forward kernel's operand path
  cplx<R>* mats_h = nullptr;
  int n_slots = 0;
  // adjoint: dst/src swapped, op conjugate-transposed (rows <-> cols)
  int n_tiles_adj = 0;
  int* tile_group_adj = nullptr;
  int* tile_pair0_adj = nullptr;
  int* tile_npairs_adj = nullptr;
  int* tile_row0_adj = nullptr;
  int* pair_dst_adj = nullptr;     // pairs regrouped for the adjoint (dst = old src)
  int* pair_src_adj = nullptr;
  // per-destination pair lists (CSR over destination boxes) for the
  // atomic-free two-phase product; *_adj lists pairs by source box
  int n_red = 0, n_red_adj = 0;
  int* red_ptr = nullptr;
  int* red_pairs = nullptr;
  int* red_ptr_adj = nullptr;
  int* red_pairs_adj = nullptr;
  // host: the pairs of group c are gstart_h[c] .. gstart_h[c + 1] - 1
  std::vector<int> gstart_h;
  // M2L by rotation (built on demand for orders <= ROT_MAXP; used when
  // rot_on): tiles of up to ROT_CT pairs of one group (forward and adjoint
  // alike, the adjoint pair lists keep the group order), per group the
  // rotation class (polar angle), distance class and e^{i m phi} for
  // m = 0..p (re, im); per rotation class the real blocks d_n and d_n^T
  // (matrix-core layout, rot_dpsz(p) values each); per distance class the
  // coaxial blocks and their conjugate transposes (rot_cpsz(p) each)
  bool rot_on = false, rot_ready = false;
  int rot_p = 0, rot_n_tiles = 0;
  int* rot_tile_group = nullptr;
  int* rot_tile_pair0 = nullptr;
  int* rot_tile_npairs = nullptr;
  int* rot_theta = nullptr;
  int* rot_dist = nullptr;
  R* rot_phase = nullptr;
  R* rot_dtab = nullptr;
  cplx<R>* rot_coax = nullptr;
  cplx<R>* rot_coax_h = nullptr;
};

// Buffers that one product writes, for one precision: sorted densities and
// their float64 copies, near-field sums, expansions per level and the
// per-pair M2L outputs.  A problem holds one set; batched solves give every
// further system of the same problem its own, so that their products can
// share launches.
template <typename R>
struct ExecBuf {
  std::array<cplx<R>*, MAX_LEVEL + 1> M{};   // multipole (box-major, ncoef per box)
  std::array<cplx<R>*, MAX_LEVEL + 1> Lc{};  // local
  cplx<R>* cbuf = nullptr;   // per-pair M2L products, levels below the leaf level
  cplx<R>* cbufL = nullptr;  // per-pair M2L products, leaf level
  cplx<R>* ps = nullptr;     // work vectors (sorted order)
  cplx<R>* qs = nullptr;
  cplx<R>* ys = nullptr;
  cplx<R>* ys2 = nullptr;
  c64* p64s = nullptr;       // float64 input copies for the diagonal (sorted order)
  c64* q64s = nullptr;
};

template <typename T, size_t N>
constexpr std::array<T, N> filled_array(T v) {
  std::array<T, N> a{};
  for (size_t i = 0; i < N; ++i) a[i] = v;
  return a;
}

template <typename R>
struct PrecisionData {
  // device memory of everything that depends on the expansion orders (the
  // operators, tiles, reduction lists and the product buffers X): released
  // and rebuilt when the orders or the far cut are recalibrated
  DevArena ops;
  // the P2M/L2P matrices, which depend on the leaf order alone: kept across
  // rebuilds while that order stays (leaf_order: the order they hold)
  DevArena leafops;
  int leaf_order = -1;
  // translation matrices of the last build, per operator set (key: kind and
  // level), with everything they are made from: a rebuild whose inputs match
  // (the far-cut trials of the calibration) copies them instead of
  // recomputing; released once the calibration ends
  struct TransCacheEntry {
    int ngroups = -1, sing = -1, pin = -1, pout = -1;
    std::vector<double> tv, rs, cs;
    DevArena arena;
    cplx<R>* mats = nullptr;
  };
  std::map<int, TransCacheEntry> tcache;
  void release_tcache() {
    for (auto& kv : tcache) kv.second.arena.release();
    tcache.clear();
  }
  int shift = 0;       // order shifts applied to the level rule (calibration):
  int shift_c = 0;     //   the leaf level's and the coarser levels'
  // orders dropped from the multipole side of M2L translations across three
  // boxes (Chebyshev distance 3, which converge much faster than those across
  // two): their operators read (p_l - far_cut + 1)^2 input coefficients
  int far_cut = 0;
  double err = -1.0;   // sampled relative error of the product on white-noise
                       // densities (< 0: not measured)
  double err_smooth = -1.0;  // the same on a plane-wave density
  std::array<int, MAX_LEVEL + 1> order{};   // p_l
  std::array<int, MAX_LEVEL + 1> ncoef{};   // (p_l + 1)^2
  std::array<GroupedOp<R>, MAX_LEVEL + 1> m2l{};
  std::array<GroupedOp<R>, MAX_LEVEL + 1> m2m{};  // level l -> l-1 (index l)
  std::array<GroupedOp<R>, MAX_LEVEL + 1> l2l{};  // level l-1 -> l (index l)
  // direct translations leaf <-> level L - d for d = 1 .. n_direct (index d)
  int n_direct = 0;
  std::array<GroupedOp<R>, MAX_DIRECT + 1> m2m_dir{};  // leaf -> level L - d
  std::array<GroupedOp<R>, MAX_DIRECT + 1> l2l_dir{};  // level L - d -> leaf
  std::array<int64_t, MAX_LEVEL + 1> cbuf_off{};  // offset of each level's pairs in cbuf
  int64_t cbuf_count = 0, cbufL_count = 0;        // sizes of the per-pair buffers
  cplx<R>* p2m = nullptr;   // n x ncoef_L x 2 (columns: p, q), sorted order
  cplx<R>* p2m_p = nullptr; // n x ncoef_L: the p columns alone (products with q = 0)
  cplx<R>* l2p = nullptr;   // n x ncoef_L
  // near-field corrections (accurate - 3-point rule), CSR by target and
  // CSC by source (both sorted order)
  cplx<R>* near_cp = nullptr;
  cplx<R>* near_cq = nullptr;
  cplx<R>* neart_cp = nullptr;
  cplx<R>* neart_cq = nullptr;
  // float geometry (sorted order) for the direct near field
  R* geo = nullptr;         // SoA, see GEO_* offsets
  ExecBuf<R> X;             // the problem's own product buffers
};

// SoA geometry layout offsets (multiples of n)
enum {
  GEO_CX = 0, GEO_CY, GEO_CZ, GEO_NX, GEO_NY, GEO_NZ, GEO_AREA, GEO_ELL,
  GEO_QX0, GEO_QY0, GEO_QZ0, GEO_QX1, GEO_QY1, GEO_QZ1, GEO_QX2, GEO_QY2, GEO_QZ2,
  GEO_AX, GEO_AY, GEO_AZ, GEO_BX, GEO_BY, GEO_BZ, GEO_CXV, GEO_CYV, GEO_CZV,
  GEO_COUNT
};

struct Problem {
  int64_t n = 0;
  double k = 0;
  c64 alpha{0, 0};
  double eta = 2.0;
  int leaf_cap = 64, leaf_level_req = 0, order64_req = 0, order32_req = 0;
  // target relative error of the float64 / float32 products (<= 0: the
  // level rule as it is) and the largest expansion order allowed
  double fmm_tol64 = 0, fmm_tol32 = 0;
  int p_max = 40;
  DevArena arena;
  // geometry, sorted order, float64 SoA (GEO_COUNT x n)
  double* geo = nullptr;
  int* perm = nullptr;            // sorted position -> caller index
  uint64_t* keys_orig = nullptr;  // Morton keys in caller order
  uint64_t* keys_sorted = nullptr;
  // bounding cube
  double lo[3]{}, R0 = 0, scale = 0, ell_max = 0;
  // tree
  int L = 0;
  int max_leaf = 0;  // elements in the fullest leaf
  float tuned_ms = 0.f;  // autotuner: float32 product time of the kept leaf level
  // stream schedule of the products per precision (0 float64, 1 float32),
  // chosen by timing at plan creation
  std::array<int, 2> sched{{0, 0}};
  // workgroups of the near-field kernel per precision (0: one per leaf; else
  // a grid-stride launch of that many, leaving room for the far-field chain)
  std::array<int, 2> p2p_cap{{0, 0}};
  // workgroups of the leaf-level M2L launch (0: one per tile, else that many)
  std::array<int, 2> m2l_cap{{0, 0}};
  // M2L variant: 0 dense or rotation per level by timing, 1 dense only,
  // 2 rotation wherever the order allows
  int m2l_rot_req = 0;
  // depth of the direct leaf <-> ancestor translations used (<= n_direct of
  // the precision; 0: level-by-level chains only)
  std::array<int, 2> ndir{{0, 0}};
  bool direct = false;  // leaves not wider than the near radius: direct sum, no far field
  std::array<int, MAX_LEVEL + 1> nbox{};
  std::array<uint64_t*, MAX_LEVEL + 1> box_keys{};
  std::array<int*, MAX_LEVEL + 1> box_start{};   // first sorted element (nbox+1 entries)
  std::array<int*, MAX_LEVEL + 1> box_parent{};
  std::array<double, MAX_LEVEL + 1> h{};          // box side per level
  std::array<int64_t, MAX_LEVEL + 1> n_m2l{};
  std::array<int64_t, MAX_LEVEL + 1> n_m2l_far{};  // of them across three boxes
  // V-list pairs per level (destination box, source box, offset code), built
  // once from the tree on first use (vl_n < 0: not yet)
  std::array<int*, MAX_LEVEL + 1> vl_dst{}, vl_src{}, vl_code{};
  std::array<int, MAX_LEVEL + 1> vl_n = filled_array<int, MAX_LEVEL + 1>(-1);
  int* elem_leaf = nullptr;                        // sorted element -> leaf
  int* u_ptr = nullptr;                            // leaf U lists (CSR)
  int* u_idx = nullptr;
  int64_t n_u = 0, n_p2p_pairs = 0;
  // near field (sorted order)
  int64_t n_near = 0;
  int* near_ptr = nullptr;   // n + 1
  int* near_col = nullptr;
  int* neart_ptr = nullptr;  // n + 1
  int* neart_row = nullptr;
  c64* diag_p = nullptr;     // 1/2 - alpha H_ii
  c64* diag_q = nullptr;     // S_ii + alpha/2
  PrecisionData<double> f64;
  PrecisionData<float> f32;
  // solver workspace (Krylov basis etc.) and the batched solver's cached
  // buffers, owned, see solver.hip
  void* solver_ws = nullptr;
  void* batch_cache = nullptr;
  // second stream (default priority) for the direct near field, which runs
  // concurrently with the far-field chain; fork/join events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // side streams given by the plan (shared by its problems) or created and
  // owned by this problem
  bool own_streams = false;
  // third stream: the leaf-level M2L (the largest) overlaps the coarser levels
  hipStream_t side2 = nullptr;
  hipEvent_t ev_fork2 = nullptr, ev_join2 = nullptr;
  // stage profiling with HIP events (off unless enabled): prof_on times every
  // stage with event pairs recorded on the streams; prof_leaf times only the
  // leaf-level M2L launches, with events attached to the launches themselves
  // (nothing recorded between kernels), for timing inside a timed region
  bool prof_on = false;
  bool prof_leaf = false;
  // with prof_on: every stage on the caller's stream, one after another, so
  // each stage's events time it alone on the GPU
  bool prof_serial = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_slot;   // slot of each recorded (start, end) pair
  int ev_used = 0;
};

// profiling slots: stage + 16 * precision (0: float64, 1: float32) + 32 * adjoint
enum {
  ST_GATHER = 0, ST_P2P, ST_P2M, ST_M2M, ST_M2L, ST_L2L, ST_FINISH, ST_M2L_RED,
  ST_M2L_LEAF, ST_M2L_LEAF_RED,
  // evaluation at points off the boundary: local expansions at the points,
  // direct sums over touching leaves (its translations use ST_M2L,
  // ST_M2L_LEAF and ST_L2L, its gather ST_GATHER, P2M ST_P2M)
  ST_PT_L2P, ST_PT_P2P, ST_COUNT
};
constexpr int PROF_SLOTS = 64;
constexpr int prof_slot(int stage, bool f32, bool adj) { return stage + 16 * f32 + 32 * adj; }
int prof_begin(Problem& P, hipStream_t s);                 // returns event index or -1
int prof_end(Problem& P, int idx, int slot, hipStream_t s);
int prof_pair(Problem& P, int slot);  // a (start, end) pair for a launch's own events

// Stream schedules of one product (the near field P2P always runs on the
// side stream, concurrently with the far field):
//   SCHED_CONCURRENT  leaf-level M2L on a third stream, beside the upward pass
//   SCHED_LEAF_SERIAL leaf-level M2L on the main stream before the upward pass
//   SCHED_LEAF_FIRST  as SCHED_LEAF_SERIAL, with P2P started after it
//   SCHED_P2P_AFTER_UP as SCHED_CONCURRENT, with P2P started after the
//                     upward pass (whose small launches then do not wait
//                     for compute units behind it)
//   SCHED_SERIAL      every stage on the caller's stream, one after another
//                     (no stage shares the GPU: fastest when one large
//                     launch dominates, e.g. the float64 leaf-level M2L)
//   SCHED_LEAF_THEN_P2P as SCHED_CONCURRENT, with P2P forked after the P2M,
//                     behind the leaf-level M2L (whose workgroups then take
//                     their place on the compute units first)
enum {
  SCHED_CONCURRENT = 0, SCHED_LEAF_SERIAL = 1, SCHED_LEAF_FIRST = 2, SCHED_P2P_AFTER_UP = 3,
  SCHED_LEAF_THEN_P2P = 4, SCHED_SERIAL = 5, SCHED_COUNT
};

// Every buffer of a product's ExecBuf with its element count, in one fixed
// order: f(pointer reference, count).  The plan's allocation and the
// allocation-free product's layout in static device memory both walk it.
template <typename R, typename F>
void exec_buffers(const Problem& P, const PrecisionData<R>& D, ExecBuf<R>& X, F&& f) {
  for (int l = 2; l <= P.L; ++l) {
    f(X.M[l], (int64_t)P.nbox[l] * D.ncoef[l]);
    f(X.Lc[l], (int64_t)P.nbox[l] * D.ncoef[l]);
  }
  f(X.cbuf, D.cbuf_count);
  f(X.cbufL, D.cbufL_count);
  f(X.ps, P.n);
  f(X.qs, P.n);
  f(X.ys, P.n);
  f(X.ys2, P.n);
  f(X.p64s, P.n);
  f(X.q64s, P.n);
}

// ---- host entry points implemented in the .hip translation units ----
int build_geometry_and_tree(Problem& P, const double* vert, int64_t n_vert, const int32_t* tri,
                            hipStream_t s);
int build_near_field(Problem& P, hipStream_t s);
int build_operators(Problem& P, hipStream_t s);
// Rebuild the order-dependent data of one precision with the level rule
// shifted by shift_c on the levels above the leaves and shift_l on the leaf
// level (release of the old data included).
template <typename R>
int rebuild_precision(Problem& P, PrecisionData<R>& D, int shift_c, int shift_l, hipStream_t s);
// Tables and tiles of the rotation-based M2L for every level of one
// precision whose order allows it (kept until the next rebuild; no level is
// switched on).
template <typename R>
int build_rotations(Problem& P, PrecisionData<R>& D, hipStream_t s);
// Forward tiles of a grouped op rebuilt for another pair-tile width (the
// tuner's choice for the leaf-level M2L).
template <typename R>
int retile_forward(GroupedOp<R>& op, int ct, DevArena& arena, hipStream_t s);
// Sampled relative error of one product against the exact discrete operator:
// rows spread over the mesh, seeded pseudo-random p and q, reference rows
// summed directly in float64 (rule points, near corrections, diagonal).
template <typename R>
int measure_error(Problem& P, PrecisionData<R>& D, hipStream_t s, double* err);
// Orders of both precisions chosen for the problem's tolerances (see
// bem_problem.fmm_tol), then the achieved errors measured.
int calibrate_orders(Problem& P, hipStream_t s);
template <typename R>
int alloc_exec(const Problem& P, const PrecisionData<R>& D, ExecBuf<R>& X, DevArena& arena);
template <typename R>
int fmm_apply(Problem& P, PrecisionData<R>& D, const c64* p, const c64* q, c64* y,
              hipStream_t s);
template <typename R>
int fmm_apply_adjoint(Problem& P, PrecisionData<R>& D, const c64* y, c64* u, c64* w,
                      hipStream_t s);
// The same products into the given buffers (several executions of one
// problem may be in flight with distinct buffers).
template <typename R>
int fmm_apply_x(Problem& P, PrecisionData<R>& D, ExecBuf<R>& X, const c64* p, const c64* q,
                c64* y, hipStream_t s);
template <typename R>
int fmm_apply_adjoint_x(Problem& P, PrecisionData<R>& D, ExecBuf<R>& X, const c64* y, c64* u,
                        c64* w, hipStream_t s);

// One product of a batch: forward y = A_p in + A_q q, or adjoint
// (out, out2) = (A_p^H in, A_q^H in); items of one problem need distinct X.
template <typename R>
struct BatchItem {
  Problem* P;
  PrecisionData<R>* D;
  ExecBuf<R>* X;
  const c64* in;
  const c64* q;  // forward only (may be null)
  c64* out;
  c64* out2;     // adjoint only (may be null)
};
// Streams of a batched product: the main chain on `main`; with `side` and
// `side2` set, the near field runs on `side` and the leaf-level M2L on
// `side2`, concurrently with the chain (fork/join events ev[0..3]).
struct BatchStreams {
  hipStream_t main = nullptr, side = nullptr, side2 = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};
// All items' products (same precision and direction) with every stage
// issued once for all of them.
template <typename R>
int fmm_apply_batch(const std::vector<BatchItem<R>>& items, bool adj, const BatchStreams& bs);
int sort_pairs_u64(uint64_t* keys, int* vals, int n, int nbits, DevArena& scratch,
                   hipStream_t s);
int exclusive_scan(const int* in, int* out, int n, int* total, DevArena& scratch, hipStream_t s);

// allocation-free product (scratch.hip): the product buffers in the
// library's static device array instead of the plan's
int scratch_init_current_device();
int fmm_matvec_noalloc(Problem& P, int prec, const c64* p, const c64* q, c64* y, int nrhs,
                       hipStream_t s);

// solver helpers
// coup, coup_t (device, n x n real, row-major; null: none): the coupled
// operator of an elastic body, q = coup x (adjoint: + coup_t w, coup_t the
// transpose of coup); excludes sigma
int gmres_solve(Problem& P, const c64* sigma, int adjoint, const c64* b, c64* x,
                double tol, int restart, int max_iter, int mode, double inner_tol, int use_x0,
                void* info, hipStream_t s, const double* coup = nullptr,
                const double* coup_t = nullptr);
// BEM-FEM coupling (fem.hip): C = -rho_f omega^2 Tc (K - omega^2 M)^(-1) N and
// its transpose built on the device into keep; out = M v (add: out += M v)
int coupling_build(Problem& P, const double* nodes_h, int64_t n_nodes, const int* tets_h,
                   int64_t n_tets, const int* tri_h, double lam, double mu, double rho_s,
                   double rho_f, double omega, DevArena& keep, double** C_out, double** Ct_out,
                   hipStream_t s);
int coupling_apply(const double* M, int64_t n, const c64* v, c64* out, bool add, hipStream_t s);
int plane_wave_rhs(Problem& P, const double* d, c64* b, hipStream_t s);
int point_source_rhs(Problem& P, const double* src, const c64* amp, int n_src, c64* b,
                     hipStream_t s);
int eval_field(Problem& P, const c64* p, const c64* q, const double* pts, int n_pts,
               const double* d, c64* out, hipStream_t s);
int eval_field_grad(Problem& P, const c64* p, const c64* q, const double* pts, int n_pts,
                    const double* d, const double* src, const c64* amp, int n_src, c64* out,
                    c64* grad, hipStream_t s);
// ---- evaluation points off the boundary (field_points.hip) ----
// Point boxes live on the grid of the problem's tree (same origin and box
// sides per level) and may reach PT_EXT level-2 boxes beyond its root cube
// on every side; translations into them from level-2 boxes then span up to
// PT_OFF boxes per axis (codes over a PT_W^3 table), from finer levels at
// most 3.
constexpr int PT_EXT = 8;
constexpr int PT_OFF = 3 + PT_EXT;
constexpr int PT_W = 2 * PT_OFF + 1;
constexpr int PT_CODES = PT_W * PT_W * PT_W;

// Translations of one precision into the point boxes, their locals and the
// buffers of the source tree's upward pass (multipoles and sorted densities).
template <typename R>
struct PointOps {
  std::array<GroupedOp<R>, MAX_LEVEL + 1> m2l{};  // source boxes -> point boxes, level l
  std::array<GroupedOp<R>, MAX_LEVEL + 1> l2l{};  // point boxes level l - 1 -> l (index l)
  std::array<cplx<R>*, MAX_LEVEL + 1> Lc{};       // locals of the point boxes
  ExecBuf<R> X;                                    // M[l], ps, qs, p64s, q64s only
  // float32: per-pair M2L outputs of every level (offset cbuf_off[l]),
  // summed per point box in a fixed order (float64 adds atomically: its
  // per-pair buffer would take gigabytes and its products are bound by the
  // matrix cores)
  cplx<R>* cbuf = nullptr;
  std::array<int64_t, MAX_LEVEL + 1> cbuf_off{};
};

// Host-side lists of the point octree (inputs of the operator build).
struct PointLists {
  std::array<std::vector<int>, MAX_LEVEL + 1> m2l_dst, m2l_src, m2l_code;
  std::array<std::vector<int>, MAX_LEVEL + 1> l2l_dst, l2l_src, l2l_code;
};

struct FieldPoints {
  Problem* P = nullptr;
  int prec = 0;          // 0 float64, 1 float32
  int64_t n = 0;
  DevArena arena;
  double* xyz = nullptr;  // sorted points, SoA (3 x n)
  int* perm = nullptr;    // sorted position -> caller index
  int L = 0;              // deepest point level (the problem's leaf level)
  std::array<int, MAX_LEVEL + 1> nbox{};
  std::array<int64_t, MAX_LEVEL + 1> n_m2l{};
  std::array<int64_t, MAX_LEVEL + 1> n_m2l_far{};  // of them across three boxes or more
  // leaves (boxes without children) in point order, cut into chunks of at
  // most 64 points; chunk_* describe the far-field (L2P) chunks, near_* the
  // chunks of leaves on the deepest level with their source-leaf lists
  int n_leaf = 0, n_chunk = 0, n_near_chunk = 0;
  int* leaf_box = nullptr;     // index among the point boxes of its level
  double* leaf_c = nullptr;    // centres, 3 per leaf
  int* chunk_leaf = nullptr;
  int* chunk_pt = nullptr;     // first point; count in chunk_cnt
  int* chunk_cnt = nullptr;
  int* near_pt = nullptr;      // first point, count, first / end entry of near_src
  int* near_cnt = nullptr;
  int* near_s0 = nullptr;
  int* near_s1 = nullptr;
  int* near_src = nullptr;     // source leaves (indices among the problem's leaves)
  int64_t n_near_pairs = 0;    // point x element pairs summed directly
  int max_order = 0;
  double* finv = nullptr;      // 1 / f_n per level: finv[l * (MAXP_PT + 1) + n]
  double* gcoef = nullptr;     // derivative coefficients up to max_order
  c64* acc = nullptr;          // far-field sums (field, d/dx, d/dy, d/dz) per sorted point
  c64* acc_near = nullptr;     // direct sums, the same layout (points of near chunks only)
  uint8_t* near_flag = nullptr;  // per sorted point: 1 if it has direct sums
  std::array<int, MAX_LEVEL + 2> chunk_off{};  // first far-field chunk of each level
  PointOps<float> f32;
  PointOps<double> f64;
};
constexpr int MAXP_PT = 40;    // largest expansion order (the library's)

int field_points_create(Problem& P, int prec, const double* pts, int64_t n, FieldPoints** out,
                        hipStream_t s);
void field_points_destroy(FieldPoints* F);
int eval_field_grad_fmm(FieldPoints& F, const c64* p, const c64* q, const double* d,
                        const double* src, const c64* amp, int n_src, c64* out, c64* grad,
                        hipStream_t s);
// operators.hip: translations into the point boxes and the derivative table
template <typename R>
int build_point_ops(Problem& P, PrecisionData<R>& D, const PointLists& lists, FieldPoints& F,
                    PointOps<R>& O, hipStream_t s);
// Rotation tables of the point-box M2L (see build_rotations), on the levels
// where the problem's M2L of the precision is rotation-based.
template <typename R>
int build_point_rotations(Problem& P, PrecisionData<R>& D, FieldPoints& F, PointOps<R>& O,
                          hipStream_t s);
int derivative_table(Problem& P, int p, std::vector<double>& gc, DevArena& scratch,
                     hipStream_t s);
// fmm.hip: multipoles of the problem's tree for (p, q), then the locals of
// the point boxes
// `fork` (may be null) is recorded on s once the densities are gathered
template <typename R>
int point_far_field(Problem& P, PrecisionData<R>& D, FieldPoints& F, PointOps<R>& O,
                    const c64* p, const c64* q, hipStream_t s, hipEvent_t fork);

int topological_derivative(int n, const c64* p, const c64* gp, const c64* pt, const c64* gpt,
                           double cg, double cv, double* T, hipStream_t s);
int eval_field_adjoint(Problem& P, const double* pts, int n_pts, const c64* c, c64* rp,
                       c64* rq, hipStream_t s);
void release_workspace(Problem& P);

}  // namespace bemfmm
