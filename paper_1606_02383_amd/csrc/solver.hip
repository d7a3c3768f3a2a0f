// GMRES(m) in float64 on device vectors, mixed-precision iterative
// refinement, plane-wave right-hand sides, the field representation at
// exterior points, and the objective J = sum |p(x_m)|^2 with its
// discrete-adjoint gradient.
//
// GMRES is the paper's iterative solver (Sec. 2.3 step 2; Sec. 3, tolerance
// there 1e-5).  Arnoldi uses classical Gram-Schmidt with one
// re-orthogonalisation (CGS2): two multi-dot and two multi-update kernels per
// step instead of 2(j+1) launches; reductions are deterministic two-stage
// sums.  The small Hessenberg least-squares problem (Givens rotations) is
// solved on the host from one (j+2)-entry column per step.  The exit test
// is the true relative residual ||b - A x|| / ||b|| recomputed with the
// float64 operator.
#include <cmath>
#include <complex>
#include <functional>
#include <vector>
#include <algorithm>
#include <cstring>

#include <hip/hip_ext.h>

#include "../../include/bemfmm.h"
#include "plan.h"

namespace bemfmm {

#define ARENA_ALLOC(arena, ptr, count)                                              \
  do {                                                                              \
    int _r = (arena).alloc((void**)&(ptr), sizeof(*(ptr)) * (size_t)(count));      \
    if (_r) return _r;                                                              \
  } while (0)

constexpr int RED_BLOCKS = 128;
constexpr int RED_THREADS = 256;

// Fixed-order sum over a wavefront: lane l holds v; every lane gets the total.
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block bx's partial of conj(v)^H w (complex, interleaved re/im) into
// out[0..1]; blocks stride the vector RED_BLOCKS apart.  The final sums are
// formed by the kernel that consumes them (fold_dots), so no grid-wide
// synchronisation is needed.
__device__ __forceinline__ void dot_partial(const c64* __restrict__ v, int64_t n,
                                            const c64* __restrict__ w, int bx,
                                            double* __restrict__ out) {
  __shared__ double sr[RED_THREADS / 64], si[RED_THREADS / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double ar = 0, ai = 0;
  for (int64_t i = bx * (int64_t)RED_THREADS + threadIdx.x; i < n;
       i += (int64_t)RED_BLOCKS * RED_THREADS) {
    c64 a = v[i], b = w[i];
    ar += a.re * b.re + a.im * b.im;
    ai += a.re * b.im - a.im * b.re;
  }
  ar = wave_sum(ar);
  ai = wave_sum(ai);
  if (lane == 0) {
    sr[wave] = ar;
    si[wave] = ai;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = (sr[0] + sr[1]) + (sr[2] + sr[3]);
    out[1] = (si[0] + si[1]) + (si[2] + si[3]);
  }
}

// partial[k][bx] = sum over block bx of conj(V_k[i]) w[i], k < gridDim.y
__global__ void __launch_bounds__(RED_THREADS)
    k_multidot_partial(const c64* __restrict__ V, int64_t ld, int64_t n,
                       const c64* __restrict__ w, double* __restrict__ partial) {
  const int kvec = blockIdx.y;
  dot_partial(V + kvec * ld, n, w, blockIdx.x, partial + 2 * (kvec * RED_BLOCKS + blockIdx.x));
}

// hs[k] = sum_bx partial[k][bx] for k < nk into shared memory, in a fixed
// order (every block of the caller gets bit-identical values); with out
// non-null they are also stored there (the caller passes it to one block
// only).  Wave q handles k = q, q + 4, ...
__device__ __forceinline__ void fold_dots(const double* __restrict__ partial, int nk, c64* hs,
                                          c64* __restrict__ out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = wave; k < nk; k += 4) {
    const double* pk = partial + 2 * (int64_t)k * RED_BLOCKS;
    double r = pk[2 * lane] + pk[2 * (lane + 64)];
    double m = pk[2 * lane + 1] + pk[2 * (lane + 64) + 1];
    r = wave_sum(r);
    m = wave_sum(m);
    if (lane == 0) {
      hs[k] = mk(r, m);
      if (out) out[k] = mk(r, m);
    }
  }
  __syncthreads();
}

// w -= sum_k V_k h_k with h_k folded from the dot partials (h stored to
// hout by block 0); with nrm_partial != null also the block partials of
// ||w||^2 after the update.  nk <= MAX_NK; bx is the block's index within
// the vector (256 entries per block).
constexpr int MAX_NK = 512;
__device__ __forceinline__ void update_block(const c64* __restrict__ V, int64_t ld, int64_t n,
                                             int nk, const double* __restrict__ partial,
                                             c64* __restrict__ hout, c64* __restrict__ w,
                                             double* __restrict__ nrm_partial, int bx) {
  __shared__ c64 hs[MAX_NK];
  __shared__ double sw[4];
  fold_dots(partial, nk, hs, bx == 0 ? hout : nullptr);
  int64_t i = bx * (int64_t)blockDim.x + threadIdx.x;
  double sq = 0;
  if (i < n) {
    c64 acc = w[i];
    for (int kk = 0; kk < nk; ++kk) {
      c64 v = V[kk * ld + i], c = hs[kk];
      acc.re -= v.re * c.re - v.im * c.im;
      acc.im -= v.re * c.im + v.im * c.re;
    }
    w[i] = acc;
    sq = acc.re * acc.re + acc.im * acc.im;
  }
  if (!nrm_partial) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  sq = wave_sum(sq);
  if (lane == 0) sw[wave] = sq;
  __syncthreads();
  if (threadIdx.x == 0) nrm_partial[bx] = (sw[0] + sw[1]) + (sw[2] + sw[3]);
}

__global__ void __launch_bounds__(256)
    k_multiupdate(const c64* __restrict__ V, int64_t ld, int64_t n, int nk,
                  const double* __restrict__ partial, c64* __restrict__ hout,
                  c64* __restrict__ w, double* __restrict__ nrm_partial) {
  update_block(V, ld, n, nk, partial, hout, w, nrm_partial, blockIdx.x);
}

// V_{j+1} = w / ||w||, ||w||^2 folded from the n_part block partials.
// Block 0 stores ||w||^2 to nrm_out and writes the step's Hessenberg column
// to col (host memory): col[i] = h1[i] + h2[i] for i <= j, col[j+1] = ||w||^2.
__device__ __forceinline__ void normalise_block(const c64* __restrict__ src, int64_t n,
                                                const double* __restrict__ nrm_partial,
                                                int n_part, c64* __restrict__ dst,
                                                c64* __restrict__ nrm_out,
                                                const c64* __restrict__ h1,
                                                const c64* __restrict__ h2, int j,
                                                c64* __restrict__ col, int bx) {
  __shared__ double s_nrm;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (wave == 0) {
    double t = 0;
    for (int b = lane; b < n_part; b += 64) t += nrm_partial[b];
    t = wave_sum(t);
    if (lane == 0) s_nrm = t;
  }
  __syncthreads();
  const double nrm2 = s_nrm;
  if (bx == 0) {
    if (threadIdx.x == 0 && nrm_out) *nrm_out = mk(nrm2, 0.0);
    if (col) {
      for (int t = threadIdx.x; t <= j + 1; t += blockDim.x)
        col[t] = (t <= j) ? cadd(h1[t], h2[t]) : mk(nrm2, 0.0);
      __threadfence_system();
    }
  }
  int64_t i = bx * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = sqrt(nrm2);
  double inv = (s > 0.0) ? 1.0 / s : 0.0;
  dst[i] = mk(src[i].re * inv, src[i].im * inv);
}

__global__ void __launch_bounds__(256)
    k_normalise(const c64* __restrict__ src, int64_t n, const double* __restrict__ nrm_partial,
                int n_part, c64* __restrict__ dst, c64* __restrict__ nrm_out,
                const c64* __restrict__ h1, const c64* __restrict__ h2, int j,
                c64* __restrict__ col) {
  normalise_block(src, n, nrm_partial, n_part, dst, nrm_out, h1, h2, j, col, blockIdx.x);
}

// ---------------------------------------------------------------------------
// The same CGS2 phases for several systems in one launch each (batched
// solver).  Per-system vectors and scratch are fixed for a solve and sit in
// a device table; the tick's jobs (system index and basis size) and their
// block offsets are a kernel argument.  Each block finds its job by binary
// search over the offsets and runs the single-system body on it.
// ---------------------------------------------------------------------------
constexpr int ORTH_MAX_JOBS = 64;

struct OrthSysDev {
  c64* V;  // (m + 1) x n basis, leading dimension n
  c64* w;
  int64_t n;
  double* partial;   // RED_BLOCKS x (m + 2) complex dot partials
  double* partial2;  // norm partials, one per 256-entry block
  c64* h;
  c64* h2;
  c64* hcol;  // pinned host column (slot 0)
};

struct OrthTick {
  int njobs;
  int sys[ORTH_MAX_JOBS];
  int kofs[ORTH_MAX_JOBS + 1];  // prefix sums of the basis sizes j + 1
  int bofs[ORTH_MAX_JOBS + 1];  // prefix sums of ceil(n / 256)
};

// largest job a with ofs[a] <= x (ofs ascending, ofs[0] = 0)
__device__ __forceinline__ int find_job(const int* ofs, int nj, int x) {
  int lo = 0, hi = nj - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ofs[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// grid (RED_BLOCKS, kofs[njobs]): block row y is basis vector y - kofs[a]
// of job a
__global__ void __launch_bounds__(RED_THREADS)
    k_orth_dots(const OrthSysDev* __restrict__ tab, const OrthTick t) {
  const int a = find_job(t.kofs, t.njobs, blockIdx.y);
  const OrthSysDev S = tab[t.sys[a]];
  const int kvec = blockIdx.y - t.kofs[a];
  dot_partial(S.V + kvec * S.n, S.n, S.w, blockIdx.x,
              S.partial + 2 * (kvec * RED_BLOCKS + blockIdx.x));
}

// grid (bofs[njobs]); pass 0: w -= V h1 (h1 -> h); pass 1: w -= V h2
// (h2 -> h2) and the norm partials
__global__ void __launch_bounds__(256)
    k_orth_update(const OrthSysDev* __restrict__ tab, const OrthTick t, int pass) {
  const int a = find_job(t.bofs, t.njobs, blockIdx.x);
  const OrthSysDev S = tab[t.sys[a]];
  const int nk = t.kofs[a + 1] - t.kofs[a];
  update_block(S.V, S.n, S.n, nk, S.partial, pass ? S.h2 : S.h, S.w,
               pass ? S.partial2 : nullptr, blockIdx.x - t.bofs[a]);
}

// grid (bofs[njobs]): V_{j+1} = w / ||w|| and the Hessenberg column
__global__ void __launch_bounds__(256)
    k_orth_normalise(const OrthSysDev* __restrict__ tab, const OrthTick t) {
  const int a = find_job(t.bofs, t.njobs, blockIdx.x);
  const OrthSysDev S = tab[t.sys[a]];
  const int j = t.kofs[a + 1] - t.kofs[a] - 1;
  const int nb = t.bofs[a + 1] - t.bofs[a];
  normalise_block(S.w, S.n, S.partial2, nb, S.V + (int64_t)(j + 1) * S.n, S.h2 + j + 1, S.h,
                  S.h2, j, S.hcol, blockIdx.x - t.bofs[a]);
}

// out[k] = sum_bx partial[k][bx]  (one wave per k; same order as fold_dots)
__global__ void k_multidot_final(const double* __restrict__ partial, int nk,
                                 c64* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x;
  if (k >= nk) return;
  const double* pk = partial + 2 * (int64_t)k * RED_BLOCKS;
  double r = pk[2 * lane] + pk[2 * (lane + 64)];
  double m = pk[2 * lane + 1] + pk[2 * (lane + 64) + 1];
  r = wave_sum(r);
  m = wave_sum(m);
  if (lane == 0) out[k] = mk(r, m);
}

// x += sum_k V_k y_k
__global__ void k_combine(const c64* __restrict__ V, int64_t ld, int64_t n, int nk,
                          const c64* __restrict__ y, c64* __restrict__ x) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  c64 acc = x[i];
  for (int kk = 0; kk < nk; ++kk) cfma(acc, V[kk * ld + i], y[kk]);
  x[i] = acc;
}

// r = b - a
__global__ void k_sub(const c64* __restrict__ b, const c64* __restrict__ a, int64_t n,
                      c64* __restrict__ r) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) r[i] = csub(b[i], a[i]);
}

// out = s * v (elementwise), conj_s conjugates s
__global__ void k_diag_mul(const c64* __restrict__ sg, const c64* __restrict__ v, int64_t n,
                           int conj_s, c64* __restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  c64 s = sg[i];
  if (conj_s) s.im = -s.im;
  out[i] = cmul(s, v[i]);
}

// out = a + conj(s) * b
__global__ void k_add_conj_diag(const c64* __restrict__ a, const c64* __restrict__ sg,
                                const c64* __restrict__ b, int64_t n, c64* __restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  c64 r = a[i];
  cfmac(r, sg[i], b[i]);
  out[i] = r;
}

__global__ void k_copy(const c64* __restrict__ a, int64_t n, c64* __restrict__ b) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

__global__ void k_axpy(const c64* __restrict__ a, int64_t n, c64* __restrict__ b) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = cadd(b[i], a[i]);
}

__global__ void k_set_zero(c64* __restrict__ a, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = mk(0.0, 0.0);
}

__global__ void k_scale(c64* __restrict__ a, int64_t n, double s) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = cscale(a[i], s);
}

struct Workspace {
  DevArena arena;
  int64_t n = 0;
  int m = 0;
  c64* V = nullptr;     // (m+1) x n
  c64* w = nullptr;
  c64* t1 = nullptr;
  c64* t2 = nullptr;
  c64* t3 = nullptr;
  c64* r = nullptr;
  c64* d = nullptr;
  c64* rr = nullptr;
  c64* h = nullptr;     // m+2
  c64* h2 = nullptr;
  c64* y = nullptr;
  double* partial = nullptr;   // RED_BLOCKS x (m+2) complex block partials
  double* partial2 = nullptr;  // one per 256-element block
  c64* hcol = nullptr;         // pinned host: 2 slots x (m+2) Hessenberg columns
  c64* hscal = nullptr;        // pinned host: scalars read back (norms)
  hipEvent_t ev[2] = {nullptr, nullptr};
  int ensure(int64_t n_, int m_) {
    if (n_ == n && m_ <= m) return 0;
    release();
    n = n_;
    m = m_;
    ARENA_ALLOC(arena, V, (int64_t)(m + 1) * n);
    ARENA_ALLOC(arena, w, n);
    ARENA_ALLOC(arena, t1, n);
    ARENA_ALLOC(arena, t2, n);
    ARENA_ALLOC(arena, t3, n);
    ARENA_ALLOC(arena, r, n);
    ARENA_ALLOC(arena, d, n);
    ARENA_ALLOC(arena, rr, n);
    ARENA_ALLOC(arena, h, m + 2);
    ARENA_ALLOC(arena, h2, m + 2);
    ARENA_ALLOC(arena, y, m + 2);
    ARENA_ALLOC(arena, partial, 2 * (int64_t)RED_BLOCKS * (m + 2));
    ARENA_ALLOC(arena, partial2, ceil_div(n, 256) + 1);
    BEM_HIP_TRY(hipHostMalloc((void**)&hcol, sizeof(c64) * 2 * (m + 2), hipHostMallocDefault));
    BEM_HIP_TRY(hipHostMalloc((void**)&hscal, sizeof(c64) * 4, hipHostMallocDefault));
    for (auto& e : ev) BEM_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return 0;
  }
  void release() {
    arena.release();
    if (hcol) (void)hipHostFree(hcol);
    if (hscal) (void)hipHostFree(hscal);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    hcol = hscal = nullptr;
    ev[0] = ev[1] = nullptr;
    n = 0;
    m = 0;
  }
};

static Workspace& workspace_for(Problem& P) {
  if (!P.solver_ws) P.solver_ws = new Workspace();
  return *(Workspace*)P.solver_ws;
}

// dots out[k] = V_k^H w for k < nk (partials, then one fixed-order fold)
static int multidot(Workspace& W, const c64* V, int64_t ld, int64_t n, int nk, const c64* w,
                    c64* out, hipStream_t s) {
  hipLaunchKernelGGL(k_multidot_partial, dim3(RED_BLOCKS, nk), dim3(RED_THREADS), 0, s, V, ld, n,
                     w, W.partial);
  BEM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_multidot_final, dim3(nk), dim3(64), 0, s, W.partial, nk, out);
  BEM_LAUNCH_CHECK();
  return 0;
}

// ||v|| read back to the host (synchronises the stream)
static int norm2(Workspace& W, const c64* v, int64_t n, double* out, hipStream_t s) {
  int r = multidot(W, v, n, n, 1, v, W.h2, s);
  if (r) return r;
  BEM_HIP_TRY(hipMemcpyAsync(W.hscal, W.h2, sizeof(c64), hipMemcpyDeviceToHost, s));
  BEM_HIP_TRY(hipStreamSynchronize(s));
  *out = sqrt(W.hscal[0].re);
  return 0;
}

// Orthogonalisation of one Arnoldi step (w = A V_j on entry), CGS2:
//   h1 = V^H w, w -= V h1, h2 = V^H w, w -= V h2, V_{j+1} = w / ||w||
// in five launches (each update folds the preceding dot partials itself);
// the column (h1 + h2, ||w||^2) lands in host slot `slot` of W.hcol and
// W.ev[slot] completes with the launch that writes it.
static int arnoldi_orth(Workspace& W, int64_t n, int j, int slot, hipStream_t s) {
  const int nb = ceil_div(n, 256);
  const int nk = j + 1;
  if (nk > MAX_NK) return -1;
  hipLaunchKernelGGL(k_multidot_partial, dim3(RED_BLOCKS, nk), dim3(RED_THREADS), 0, s, W.V,
                     (int64_t)n, n, W.w, W.partial);
  BEM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_multiupdate, dim3(nb), dim3(256), 0, s, W.V, (int64_t)n, n, nk,
                     W.partial, W.h, W.w, (double*)nullptr);
  BEM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_multidot_partial, dim3(RED_BLOCKS, nk), dim3(RED_THREADS), 0, s, W.V,
                     (int64_t)n, n, W.w, W.partial);
  BEM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_multiupdate, dim3(nb), dim3(256), 0, s, W.V, (int64_t)n, n, nk,
                     W.partial, W.h2, W.w, W.partial2);
  BEM_LAUNCH_CHECK();
  // W.ev[slot] is signalled by this launch's completion (no separate event
  // record, which would cost the stream a gap before the next product)
  hipExtLaunchKernelGGL(k_normalise, dim3(nb), dim3(256), 0, s, nullptr, W.ev[slot], 0, W.w, n,
                        W.partial2, nb, W.V + (int64_t)(j + 1) * n, W.h2 + j + 1, W.h, W.h2, j,
                        W.hcol + slot * (W.m + 2));
  BEM_LAUNCH_CHECK();
  return 0;
}

typedef std::function<int(const c64*, c64*)> ApplyFn;

// Relative residual reduction asked of the float32 inner solve at
// refinement step `outer` (residual rn, right-hand side norm bn): the first
// step asks for inner_tol, later ones for the reduction still needed to
// reach tol with a factor-2 margin; never below 1e-6 (the float32 operator
// is accurate to ~1e-5, so tighter inner targets only cost iterations).
static double inner_target(int outer, double inner_tol, double tol, double bn, double rn) {
  const double need = 0.5 * tol * bn / rn;
  const double t = outer == 0 ? std::max(inner_tol > 0 ? inner_tol : 1e-3, need) : need;
  return std::max(t, 1e-6);
}

struct GmresStats {
  int iters = 0, restarts = 0;
  double est = 0;
  std::vector<double> hist;
};

// GMRES(m) on apply, x in/out; stops when the (estimated, then recomputed
// with `apply`) residual <= atol or after max_iter steps.
// Returns 0, or BEM_E_NOCONV / BEM_E_NAN / BEM_E_BREAKDOWN / error.
//
// The host runs one Arnoldi step behind the device: step j + 1 is queued
// before the host waits for the Hessenberg column of step j, so the device
// does not idle while the host applies the Givens rotations.  When the
// residual trend says step j is likely the last of the cycle, the host waits
// instead of queueing a step that would be thrown away.
static int gmres_core(Workspace& W, const ApplyFn& apply, const c64* b, c64* x, int64_t n,
                      double atol, int m, int max_iter, bool x_is_zero, GmresStats& st,
                      hipStream_t s) {
  const int nb = ceil_div(n, 256);
  double beta = 0;
  int r;
  // r = b - A x
  if (x_is_zero) {
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, s, b, n, W.r);
    BEM_LAUNCH_CHECK();
  } else {
    if ((r = apply(x, W.t1))) return r;
    hipLaunchKernelGGL(k_sub, dim3(nb), dim3(256), 0, s, b, W.t1, n, W.r);
    BEM_LAUNCH_CHECK();
  }
  if ((r = norm2(W, W.r, n, &beta, s))) return r;
  st.est = beta;
  if (!std::isfinite(beta)) return -6;
  if (beta <= atol) return 0;
  std::vector<std::complex<double>> H((m + 1) * m), cs(m), sn(m), g(m + 1);
  const int ld = W.m + 2;
  // queue step j: w = A V_j, orthogonalise, column to slot j & 1
  auto issue = [&](int j) -> int {
    int rr = apply(W.V + (int64_t)j * n, W.w);
    if (rr) return rr;
    ++st.iters;
    return arnoldi_orth(W, n, j, j & 1, s);
  };
  while (st.iters < max_iter) {
    // V_0 = r / beta
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, s, W.r, n, W.V);
    BEM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scale, dim3(nb), dim3(256), 0, s, W.V, n, 1.0 / beta);
    BEM_LAUNCH_CHECK();
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jend = 0;
    if ((r = issue(0))) return r;
    bool queued_next = false;  // step j + 1 already queued
    double est_prev = beta, est_prev2 = 0.0;
    for (int j = 0; j < m; ++j) {
      // speculate on step j + 1 unless the trend predicts convergence at j
      const bool room = (j + 1 < m) && (st.iters < max_iter);
      const double pred = (est_prev2 > 0.0) ? est_prev * (est_prev / est_prev2) : est_prev;
      queued_next = false;
      if (room && pred > atol) {
        if ((r = issue(j + 1))) return r;
        queued_next = true;
      }
      BEM_HIP_TRY(hipEventSynchronize(W.ev[j & 1]));
      const c64* hc = W.hcol + (j & 1) * ld;
      std::vector<std::complex<double>> col(j + 2);
      for (int i = 0; i <= j; ++i) col[i] = std::complex<double>(hc[i].re, hc[i].im);
      double hn = sqrt(hc[j + 1].re);
      col[j + 1] = hn;
      if (!std::isfinite(hn)) {
        BEM_HIP_TRY(hipStreamSynchronize(s));
        return -6;
      }
      for (int i = 0; i < j; ++i) {
        std::complex<double> t = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -std::conj(sn[i]) * col[i] + std::conj(cs[i]) * col[i + 1];
        col[i] = t;
      }
      double den = std::sqrt(std::norm(col[j]) + std::norm(col[j + 1]));
      if (den == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        cs[j] = std::conj(col[j]) / den;
        sn[j] = std::conj(col[j + 1]) / den;
      }
      col[j] = cs[j] * col[j] + sn[j] * col[j + 1];
      col[j + 1] = 0.0;
      g[j + 1] = -std::conj(sn[j]) * g[j];
      g[j] = cs[j] * g[j];
      for (int i = 0; i <= j; ++i) H[i * m + j] = col[i];
      jend = j + 1;
      st.est = std::abs(g[j + 1]);
      st.hist.push_back(st.est);
      est_prev2 = est_prev;
      est_prev = st.est;
      if (st.est <= atol || hn == 0.0) break;
      if (!queued_next) {
        if (!room) break;
        if ((r = issue(j + 1))) return r;
        queued_next = true;
      }
    }
    // y = H^-1 g (upper triangular)
    std::vector<std::complex<double>> yv(jend);
    for (int i = jend - 1; i >= 0; --i) {
      std::complex<double> acc = g[i];
      for (int kk = i + 1; kk < jend; ++kk) acc -= H[i * m + kk] * yv[kk];
      if (std::abs(H[i * m + i]) == 0.0) {
        BEM_HIP_TRY(hipStreamSynchronize(s));
        return -5;
      }
      yv[i] = acc / H[i * m + i];
    }
    // the host column slots are reused by the next cycle: let the queued
    // (possibly speculative) step land first
    BEM_HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < jend; ++i) W.hcol[i] = mk(yv[i].real(), yv[i].imag());
    BEM_HIP_TRY(hipMemcpyAsync(W.y, W.hcol, sizeof(c64) * jend, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_combine, dim3(nb), dim3(256), 0, s, W.V, n, n, jend, W.y, x);
    BEM_LAUNCH_CHECK();
    // recompute the residual with the operator
    if ((r = apply(x, W.t1))) return r;
    hipLaunchKernelGGL(k_sub, dim3(nb), dim3(256), 0, s, b, W.t1, n, W.r);
    BEM_LAUNCH_CHECK();
    if ((r = norm2(W, W.r, n, &beta, s))) return r;
    st.est = beta;
    if (!std::isfinite(beta)) return -6;
    if (beta <= atol) return 0;
    ++st.restarts;
  }
  return -4;
}

int gmres_solve(Problem& P, const c64* sigma, int adjoint, const c64* b, c64* x, double tol,
                int restart, int max_iter, int mode, double inner_tol, int use_x0, void* info_v,
                hipStream_t s, const double* coup, const double* coup_t) {
  bem_gmres_info* info = (bem_gmres_info*)info_v;
  const int64_t n = P.n;
  const int nb = ceil_div(n, 256);
  Workspace& W = workspace_for(P);
  int r = W.ensure(n, restart);
  if (r) return r;
  int mv64 = 0, mv32 = 0;
  // operator application in a given precision, writes out = A v (or A^H v)
  auto make_apply = [&](bool f32) -> ApplyFn {
    return [&, f32](const c64* v, c64* out) -> int {
      int rr;
      if (!adjoint) {
        const c64* q = nullptr;
        if (sigma) {
          hipLaunchKernelGGL(k_diag_mul, dim3(nb), dim3(256), 0, s, sigma, v, n, 0, W.t3);
          BEM_LAUNCH_CHECK();
          q = W.t3;
        } else if (coup) {  // the elastic body's response q = C p
          if ((rr = coupling_apply(coup, n, v, W.t3, false, s))) return rr;
          q = W.t3;
        }
        rr = f32 ? fmm_apply<float>(P, P.f32, v, q, out, s) : fmm_apply<double>(P, P.f64, v, q, out, s);
        if (rr) return rr;
      } else {
        c64* wv = (sigma || coup) ? W.t3 : nullptr;
        rr = f32 ? fmm_apply_adjoint<float>(P, P.f32, v, out, wv, s)
                 : fmm_apply_adjoint<double>(P, P.f64, v, out, wv, s);
        if (rr) return rr;
        if (sigma) {
          hipLaunchKernelGGL(k_add_conj_diag, dim3(nb), dim3(256), 0, s, out, sigma, W.t3, n, out);
          BEM_LAUNCH_CHECK();
        } else if (coup) {  // (Mp + Mq C)^H = Mp^H + C^T Mq^H (C real)
          if ((rr = coupling_apply(coup_t, n, W.t3, out, true, s))) return rr;
        }
      }
      if (f32)
        ++mv32;
      else
        ++mv64;
      return 0;
    };
  };
  ApplyFn A64 = make_apply(false), A32 = make_apply(true);
  double bn = 0;
  if ((r = norm2(W, b, n, &bn, s))) return r;
  GmresStats st;
  int status = 0;
  if (!use_x0) {
    hipLaunchKernelGGL(k_set_zero, dim3(nb), dim3(256), 0, s, x, n);
    BEM_LAUNCH_CHECK();
  }
  double resid = 0;
  if (bn == 0.0) {
    hipLaunchKernelGGL(k_set_zero, dim3(nb), dim3(256), 0, s, x, n);
    BEM_LAUNCH_CHECK();
  } else if (mode == 0) {
    status = gmres_core(W, A64, b, x, n, tol * bn, restart, max_iter, !use_x0, st, s);
    resid = st.est / bn;
  } else {
    // iterative refinement: outer float64 residual, inner float32 operator
    c64* rvec = W.rr;
    c64* dvec = W.d;
    int outer = 0;
    status = -4;
    bool xzero = !use_x0;
    while (outer < 30 && st.iters < max_iter) {
      if (xzero) {
        hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, s, b, n, rvec);
        BEM_LAUNCH_CHECK();
      } else {
        if ((r = A64(x, W.t1))) return r;
        hipLaunchKernelGGL(k_sub, dim3(nb), dim3(256), 0, s, b, W.t1, n, rvec);
        BEM_LAUNCH_CHECK();
      }
      double rn = 0;
      if ((r = norm2(W, rvec, n, &rn, s))) return r;
      resid = rn / bn;
      st.hist.push_back(rn);
      if (!std::isfinite(rn)) {
        status = -6;
        break;
      }
      if (resid <= tol) {
        status = 0;
        break;
      }
      GmresStats in;
      in.iters = 0;
      hipLaunchKernelGGL(k_set_zero, dim3(nb), dim3(256), 0, s, dvec, n);
      BEM_LAUNCH_CHECK();
      const double itol = inner_target(outer, inner_tol, tol, bn, rn);
      int ist = gmres_core(W, A32, rvec, dvec, n, itol * rn, restart, max_iter - st.iters, true,
                           in, s);
      st.iters += in.iters;
      for (double h : in.hist) st.hist.push_back(h);
      if (ist && ist != -4) {
        status = ist;
        break;
      }
      hipLaunchKernelGGL(k_axpy, dim3(nb), dim3(256), 0, s, dvec, n, x);
      BEM_LAUNCH_CHECK();
      xzero = false;
      ++outer;
      st.restarts = outer;
    }
  }
  BEM_HIP_TRY(hipStreamSynchronize(s));
  if (info) {
    info->iterations = st.iters;
    info->matvec64 = mv64;
    info->matvec32 = mv32;
    info->restarts = st.restarts;
    info->resid = resid;
    info->converged = (status == 0);
    int nh = std::min((int)st.hist.size(), 512);
    info->n_hist = nh;
    for (int i = 0; i < nh; ++i) info->hist[i] = st.hist[i] / (bn > 0 ? bn : 1.0);
  }
  if (status == -4) set_error("GMRES did not reach the tolerance within max_iter");
  if (status == -5) set_error("GMRES breakdown");
  if (status == -6) set_error("NaN or Inf met in GMRES");
  return status;
}

// ---------------------------------------------------------------------------
// right-hand side, field representation, objective
// ---------------------------------------------------------------------------
__global__ void k_plane_wave(const double* __restrict__ g, int64_t n, const int* __restrict__ perm,
                             double k, double alr, double ali, double dx, double dy, double dz,
                             c64* __restrict__ b) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double ph = k * (dx * g[GEO_CX * n + i] + dy * g[GEO_CY * n + i] + dz * g[GEO_CZ * n + i]);
  double dn = dx * g[GEO_NX * n + i] + dy * g[GEO_NY * n + i] + dz * g[GEO_NZ * n + i];
  double sn, cs;
  sincos(ph, &sn, &cs);
  c64 e = mk(cs, sn);
  // 1 + alpha * i k d.n
  c64 f = mk(1.0 - ali * k * dn, alr * k * dn);
  b[perm[i]] = cmul(e, f);
}

int plane_wave_rhs(Problem& P, const double* d, c64* b, hipStream_t s) {
  double nrm = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  if (!(nrm > 0)) {
    set_error("zero incidence direction");
    return -1;
  }
  hipLaunchKernelGGL(k_plane_wave, dim3(ceil_div(P.n, 256)), dim3(256), 0, s, P.geo, P.n, P.perm,
                     P.k, P.alpha.re, P.alpha.im, d[0] / nrm, d[1] / nrm, d[2] / nrm, b);
  BEM_LAUNCH_CHECK();
  return 0;
}

constexpr double INV4PI = 0.07957747154594767;

// b_i = sum_m A_m [G(x_i - y_m) + alpha dG/dn_x(x_i - y_m)] at the collocation
// points (sorted order in, caller order out): the incident field of point
// sources of intensity A_m (the forward problem's source term, Eq. hel) and
// alpha times its normal derivative
__global__ void k_point_sources(const double* __restrict__ g, int64_t n,
                                const int* __restrict__ perm, double k, double alr, double ali,
                                const double* __restrict__ src, const c64* __restrict__ amp,
                                int nsrc, c64* __restrict__ b) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x0 = g[GEO_CX * n + i], x1 = g[GEO_CY * n + i], x2 = g[GEO_CZ * n + i];
  const double n0 = g[GEO_NX * n + i], n1 = g[GEO_NY * n + i], n2 = g[GEO_NZ * n + i];
  c64 acc = mk(0.0, 0.0), accn = mk(0.0, 0.0);
  for (int m = 0; m < nsrc; ++m) {
    const double rx = x0 - src[3 * m], ry = x1 - src[3 * m + 1], rz = x2 - src[3 * m + 2];
    const double r = sqrt(rx * rx + ry * ry + rz * rz), u = 1.0 / r;
    double sn, cs;
    sincos(k * r, &sn, &cs);
    const c64 G = mk(cs * u * INV4PI, sn * u * INV4PI);
    // dG/dn_x = G (ik - 1/r) (r.n_x) / r
    const c64 Gx = cscale(cmul(G, mk(-u, k)), (rx * n0 + ry * n1 + rz * n2) * u);
    cfma(acc, G, amp[m]);
    cfma(accn, Gx, amp[m]);
  }
  cfma(acc, mk(alr, ali), accn);
  b[perm[i]] = acc;
}

int point_source_rhs(Problem& P, const double* src, const c64* amp, int n_src, c64* b,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_point_sources, dim3(ceil_div(P.n, 256)), dim3(256), 0, s, P.geo, P.n,
                     P.perm, P.k, P.alpha.re, P.alpha.im, src, amp, n_src, b);
  BEM_LAUNCH_CHECK();
  return 0;
}

// one block per point: out_m = inc + sum_j sum_q w [G_y p_j - G q_j]
__global__ void k_eval_field(const double* __restrict__ g, int64_t n, const int* __restrict__ perm,
                             const c64* __restrict__ p, const c64* __restrict__ q,
                             const double* __restrict__ pts, double k, int has_inc, double dx,
                             double dy, double dz, c64* __restrict__ out) {
  __shared__ double sr[256], si[256];
  int m = blockIdx.x;
  double x0 = pts[3 * m], x1 = pts[3 * m + 1], x2 = pts[3 * m + 2];
  double ar = 0, ai = 0;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    int o = perm[j];
    c64 pj = p[o], qj = q ? q[o] : mk(0.0, 0.0);
    double w = g[GEO_AREA * n + j] / 3.0 * INV4PI;
    double nyx = g[GEO_NX * n + j], nyy = g[GEO_NY * n + j], nyz = g[GEO_NZ * n + j];
    for (int qq = 0; qq < 3; ++qq) {
      double rx = x0 - g[(GEO_QX0 + 3 * qq) * n + j];
      double ry = x1 - g[(GEO_QX0 + 3 * qq + 1) * n + j];
      double rz = x2 - g[(GEO_QX0 + 3 * qq + 2) * n + j];
      double r = sqrt(rx * rx + ry * ry + rz * rz), u = 1.0 / r;
      double sn, cs;
      sincos(k * r, &sn, &cs);
      c64 G = mk(cs * u * w, sn * u * w);
      // G_y = -G (ik - u) u (rv.n_y)
      double rny = rx * nyx + ry * nyy + rz * nyz;
      c64 Gy = cscale(cmul(G, mk(-u, k)), -u * rny);
      c64 v = csub(cmul(Gy, pj), cmul(G, qj));
      ar += v.re;
      ai += v.im;
    }
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      sr[threadIdx.x] += sr[threadIdx.x + st];
      si[threadIdx.x] += si[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    c64 v = mk(sr[0], si[0]);
    if (has_inc) {
      double sn, cs;
      sincos(k * (dx * x0 + dy * x1 + dz * x2), &sn, &cs);
      v = cadd(v, mk(cs, sn));
    }
    out[m] = v;
  }
}

// Total field and its gradient at points (solver step 5: the integral
// representation, 3-point rule, off the boundary), one thread per point,
// 256 points per block, source elements staged through LDS in chunks:
//   p(x) = inc(x) + sum_j [int_j dG/dn_y(x - y) p_j - int_j G(x - y) q_j]
// with rv = x - y, u = 1/|rv|, G' = G (ik - u), G'' = G ((ik - u)^2 + u^2):
//   grad G = G' u rv,  grad dG/dn_y = -(G'' - G' u)(rv.n_y) u^2 rv - G' u n_y.
// The incident part: a unit plane wave exp(i k d.x) (has_pw) plus point
// sources sum_m A_m G(x - y_m) (n_src of them).
constexpr int FG_CHUNK = 128;
__global__ void __launch_bounds__(256)
    k_field_grad(const double* __restrict__ g, int64_t n, const int* __restrict__ perm,
                 const c64* __restrict__ p, const c64* __restrict__ q,
                 const double* __restrict__ pts, int npts, double k, int has_pw, double dx,
                 double dy, double dz, const double* __restrict__ src,
                 const c64* __restrict__ amp, int nsrc, c64* __restrict__ out,
                 c64* __restrict__ grad) {
  __shared__ double s_y[9][FG_CHUNK];
  __shared__ double s_n[3][FG_CHUNK];
  __shared__ c64 s_p[FG_CHUNK], s_q[FG_CHUNK];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = t < npts;
  const double x0 = active ? pts[3 * t] : 0.0, x1 = active ? pts[3 * t + 1] : 0.0,
               x2 = active ? pts[3 * t + 2] : 0.0;
  c64 f = mk(0.0, 0.0), f0 = mk(0.0, 0.0), f1 = mk(0.0, 0.0), f2 = mk(0.0, 0.0);
  for (int64_t c0 = 0; c0 < n; c0 += FG_CHUNK) {
    const int cnt = (int)std::min<int64_t>(FG_CHUNK, n - c0);
    __syncthreads();
    for (int v = threadIdx.x; v < cnt; v += blockDim.x) {
      const int64_t j = c0 + v;
      for (int c = 0; c < 9; ++c) s_y[c][v] = g[(GEO_QX0 + c) * n + j];
      s_n[0][v] = g[GEO_NX * n + j];
      s_n[1][v] = g[GEO_NY * n + j];
      s_n[2][v] = g[GEO_NZ * n + j];
      // per-point weight (rule weight x area / (4 pi)) folded into the densities
      const double w = g[GEO_AREA * n + j] / 3.0 * INV4PI;
      const int o = perm[j];
      s_p[v] = cscale(p[o], w);
      s_q[v] = q ? cscale(q[o], w) : mk(0.0, 0.0);
    }
    __syncthreads();
    if (!active) continue;
    for (int v = 0; v < cnt; ++v) {
      const double ny0 = s_n[0][v], ny1 = s_n[1][v], ny2 = s_n[2][v];
      const c64 pv = s_p[v], qv = s_q[v];
      for (int qq = 0; qq < 3; ++qq) {
        const double r0 = x0 - s_y[3 * qq][v], r1 = x1 - s_y[3 * qq + 1][v],
                     r2 = x2 - s_y[3 * qq + 2][v];
        const double rr = r0 * r0 + r1 * r1 + r2 * r2;
        const double r = sqrt(rr), u = 1.0 / r;
        double sn, cs;
        sincos(k * r, &sn, &cs);
        const c64 G = mk(cs * u, sn * u);              // without 1/(4 pi): in the weights
        const c64 a = mk(-u, k);                        // ik - u
        const c64 g1 = cmul(G, a);                      // G'
        const c64 g2 = cmul(G, cadd(cmul(a, a), mk(u * u, 0.0)));  // G''
        const double rny = r0 * ny0 + r1 * ny1 + r2 * ny2;
        const c64 Gy = cscale(g1, -rny * u);            // dG/dn_y
        // field: Gy p - G q
        cfma(f, Gy, pv);
        cfma(f, cscale(G, -1.0), qv);
        // gradient: coefficient of rv and of n_y
        const c64 crv_p = cscale(csub(g2, cscale(g1, u)), -rny * u * u);
        const c64 cny_p = cscale(g1, -u);
        const c64 crv_q = cscale(g1, -u);               // -(grad G) = -G' u rv
        c64 cr = cmul(crv_p, pv), cn = cmul(cny_p, pv);
        cfma(cr, crv_q, qv);
        f0 = cadd(f0, cadd(cscale(cr, r0), cscale(cn, ny0)));
        f1 = cadd(f1, cadd(cscale(cr, r1), cscale(cn, ny1)));
        f2 = cadd(f2, cadd(cscale(cr, r2), cscale(cn, ny2)));
      }
    }
  }
  if (!active) return;
  if (has_pw) {
    double sn, cs;
    sincos(k * (dx * x0 + dy * x1 + dz * x2), &sn, &cs);
    const c64 e = mk(cs, sn), ike = mk(-k * sn, k * cs);
    f = cadd(f, e);
    f0 = cadd(f0, cscale(ike, dx));
    f1 = cadd(f1, cscale(ike, dy));
    f2 = cadd(f2, cscale(ike, dz));
  }
  for (int m = 0; m < nsrc; ++m) {
    const double r0 = x0 - src[3 * m], r1 = x1 - src[3 * m + 1], r2 = x2 - src[3 * m + 2];
    const double r = sqrt(r0 * r0 + r1 * r1 + r2 * r2), u = 1.0 / r;
    double sn, cs;
    sincos(k * r, &sn, &cs);
    const c64 G = cmul(mk(cs * u * INV4PI, sn * u * INV4PI), amp[m]);
    const c64 g1u = cscale(cmul(G, mk(-u, k)), u);  // A G' / r
    f = cadd(f, G);
    f0 = cadd(f0, cscale(g1u, r0));
    f1 = cadd(f1, cscale(g1u, r1));
    f2 = cadd(f2, cscale(g1u, r2));
  }
  out[t] = f;
  if (grad) {
    grad[3 * t] = f0;
    grad[3 * t + 1] = f1;
    grad[3 * t + 2] = f2;
  }
}

int eval_field_grad(Problem& P, const c64* p, const c64* q, const double* pts, int n_pts,
                    const double* d, const double* src, const c64* amp, int n_src, c64* out,
                    c64* grad, hipStream_t s) {
  if (n_pts <= 0) return 0;
  double dx = 0, dy = 0, dz = 0;
  if (d) {
    const double nrm = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (!(nrm > 0)) {
      set_error("zero incidence direction");
      return -1;
    }
    dx = d[0] / nrm;
    dy = d[1] / nrm;
    dz = d[2] / nrm;
  }
  hipLaunchKernelGGL(k_field_grad, dim3(ceil_div(n_pts, 256)), dim3(256), 0, s, P.geo, P.n,
                     P.perm, p, q, pts, n_pts, P.k, d ? 1 : 0, dx, dy, dz, src, amp,
                     src ? n_src : 0, out, grad);
  BEM_LAUNCH_CHECK();
  return 0;
}

// Topological derivative (Eq. danseitpoderi), pointwise:
//   T = Re[cg grad p . grad pt - cv p pt]
__global__ void k_topological(int n, const c64* __restrict__ p, const c64* __restrict__ gp,
                              const c64* __restrict__ pt, const c64* __restrict__ gpt, double cg,
                              double cv, double* __restrict__ T) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  c64 dot = cmul(gp[3 * t], gpt[3 * t]);
  cfma(dot, gp[3 * t + 1], gpt[3 * t + 1]);
  cfma(dot, gp[3 * t + 2], gpt[3 * t + 2]);
  const c64 pp = cmul(p[t], pt[t]);
  T[t] = cg * dot.re - cv * pp.re;
}

int topological_derivative(int n, const c64* p, const c64* gp, const c64* pt, const c64* gpt,
                           double cg, double cv, double* T, hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(k_topological, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, p, gp, pt, gpt,
                     cg, cv, T);
  BEM_LAUNCH_CHECK();
  return 0;
}

// rp_j = sum_m conj(Khat_mj) c_m,  rq_j = -sum_m conj(Shat_mj) c_m
__global__ void k_eval_field_adj(const double* __restrict__ g, int64_t n,
                                 const int* __restrict__ perm, const double* __restrict__ pts,
                                 int npts, double k, const c64* __restrict__ c,
                                 c64* __restrict__ rp, c64* __restrict__ rq) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  double w = g[GEO_AREA * n + j] / 3.0 * INV4PI;
  double nyx = g[GEO_NX * n + j], nyy = g[GEO_NY * n + j], nyz = g[GEO_NZ * n + j];
  c64 ap = mk(0.0, 0.0), aq = mk(0.0, 0.0);
  for (int m = 0; m < npts; ++m) {
    c64 K = mk(0.0, 0.0), S = mk(0.0, 0.0);
    for (int qq = 0; qq < 3; ++qq) {
      double rx = pts[3 * m] - g[(GEO_QX0 + 3 * qq) * n + j];
      double ry = pts[3 * m + 1] - g[(GEO_QX0 + 3 * qq + 1) * n + j];
      double rz = pts[3 * m + 2] - g[(GEO_QX0 + 3 * qq + 2) * n + j];
      double r = sqrt(rx * rx + ry * ry + rz * rz), u = 1.0 / r;
      double sn, cs;
      sincos(k * r, &sn, &cs);
      c64 G = mk(cs * u * w, sn * u * w);
      double rny = rx * nyx + ry * nyy + rz * nyz;
      K = cadd(K, cscale(cmul(G, mk(-u, k)), -u * rny));
      S = cadd(S, G);
    }
    cfmac(ap, K, c[m]);
    cfmac(aq, S, c[m]);
  }
  int o = perm[j];
  rp[o] = ap;
  if (rq) rq[o] = mk(-aq.re, -aq.im);
}

int eval_field(Problem& P, const c64* p, const c64* q, const double* pts, int n_pts,
               const double* d, c64* out, hipStream_t s) {
  if (n_pts <= 0) return 0;
  double dx = 0, dy = 0, dz = 0;
  if (d) {
    double nrm = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (!(nrm > 0)) {
      set_error("zero incidence direction");
      return -1;
    }
    dx = d[0] / nrm;
    dy = d[1] / nrm;
    dz = d[2] / nrm;
  }
  hipLaunchKernelGGL(k_eval_field, dim3(n_pts), dim3(256), 0, s, P.geo, P.n, P.perm, p, q, pts,
                     P.k, d ? 1 : 0, dx, dy, dz, out);
  BEM_LAUNCH_CHECK();
  return 0;
}

int eval_field_adjoint(Problem& P, const double* pts, int n_pts, const c64* c, c64* rp, c64* rq,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_eval_field_adj, dim3(ceil_div(P.n, 128)), dim3(128), 0, s, P.geo, P.n,
                     P.perm, pts, n_pts, P.k, c, rp, rq);
  BEM_LAUNCH_CHECK();
  return 0;
}

// sigma = -i k beta
__global__ void k_sigma(const c64* __restrict__ beta, int64_t n, double k, c64* __restrict__ sg) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) sg[i] = mk(k * beta[i].im, -k * beta[i].re);
}

// J = sum |p_obs|^2 (one block)
__global__ void k_objective(const c64* __restrict__ pobs, int npts, double* __restrict__ J) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0;
    for (int m = 0; m < npts; ++m) s += pobs[m].re * pobs[m].re + pobs[m].im * pobs[m].im;
    *J = s;
  }
}

// rhs = rp + conj(sigma) rq
__global__ void k_adj_rhs(const c64* __restrict__ rp, const c64* __restrict__ rq,
                          const c64* __restrict__ sg, int64_t n, c64* __restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  c64 v = rp[i];
  cfmac(v, sg[i], rq[i]);
  out[i] = v;
}

// g = -conj(w) + conj(rq);  grad = 2 Re(-i k g p) + i 2 Re(k g p)
__global__ void k_grad(const c64* __restrict__ w, const c64* __restrict__ rq,
                       const c64* __restrict__ p, int64_t n, double k, c64* __restrict__ grad) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  c64 gg = mk(-w[i].re + rq[i].re, w[i].im - rq[i].im);
  c64 gp = cmul(gg, p[i]);
  // -i k gp = k (gp.im - i gp.re) -> real part k gp.im
  grad[i] = mk(2.0 * k * gp.im, 2.0 * k * gp.re);
}

// Forward half of the objective (the state problem): sigma = -i k beta,
// A(sigma) p = b (plane wave), q = sigma p, p_obs = field at the points,
// J = sum |p_obs|^2.  p_out (n) and pobs_out (n_pts) may be null.
int objective_forward(Problem& P, const c64* beta, const double* dir, const double* pts_host,
                      int n_pts, const bem_gmres_opts* opts, double* J, c64* p_out,
                      c64* pobs_out, bem_gmres_info* info_f, hipStream_t s) {
  const int64_t n = P.n;
  const int nb = ceil_div(n, 256);
  DevArena tmp;
  struct G {
    DevArena& a;
    ~G() { a.release(); }
  } guard{tmp};
  c64 *sg, *b, *p, *q, *pobs;
  double *pts, *dJ;
  ARENA_ALLOC(tmp, sg, n);
  ARENA_ALLOC(tmp, b, n);
  ARENA_ALLOC(tmp, p, n);
  ARENA_ALLOC(tmp, q, n);
  ARENA_ALLOC(tmp, pobs, n_pts);
  ARENA_ALLOC(tmp, pts, 3 * n_pts);
  ARENA_ALLOC(tmp, dJ, 1);
  BEM_HIP_TRY(hipMemcpyAsync(pts, pts_host, sizeof(double) * 3 * n_pts, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_sigma, dim3(nb), dim3(256), 0, s, beta, n, P.k, sg);
  BEM_LAUNCH_CHECK();
  int r = plane_wave_rhs(P, dir, b, s);
  if (r) return r;
  const bem_gmres_opts o = *opts;
  r = gmres_solve(P, sg, 0, b, p, o.tol, o.restart > 0 ? o.restart : 50,
                  o.max_iter > 0 ? o.max_iter : 2000, o.mode, o.inner_tol, 0, info_f, s);
  if (r) return r;
  hipLaunchKernelGGL(k_diag_mul, dim3(nb), dim3(256), 0, s, sg, p, n, 0, q);
  BEM_LAUNCH_CHECK();
  if ((r = eval_field(P, p, q, pts, n_pts, dir, pobs, s))) return r;
  hipLaunchKernelGGL(k_objective, dim3(1), dim3(64), 0, s, pobs, n_pts, dJ);
  BEM_LAUNCH_CHECK();
  BEM_HIP_TRY(hipMemcpyAsync(J, dJ, sizeof(double), hipMemcpyDeviceToHost, s));
  if (p_out) {
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, s, p, n, p_out);
    BEM_LAUNCH_CHECK();
  }
  if (pobs_out) {
    hipLaunchKernelGGL(k_copy, dim3(ceil_div(n_pts, 256)), dim3(256), 0, s, pobs,
                       (int64_t)n_pts, pobs_out);
    BEM_LAUNCH_CHECK();
  }
  BEM_HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

// Backward half (the adjoint problem, Sec. 2.2, here in its discrete form):
// with c = p_obs (dJ/dp_obs = 2 conj(p_obs), Eq. danseideltaJ), the adjoint
// right-hand side rp + conj(sigma) rq (rp, rq: the field's adjoint), the
// conjugate-transposed solve A(sigma)^H mu = rhs, w = Mq^H mu and
// grad_e = dJ/dRe(beta_e) + i dJ/dIm(beta_e) from p, w and rq.
int objective_backward(Problem& P, const c64* beta, const c64* p, const c64* pobs,
                       const double* pts_host, int n_pts, const bem_gmres_opts* opts, c64* grad,
                       bem_gmres_info* info_a, hipStream_t s) {
  const int64_t n = P.n;
  const int nb = ceil_div(n, 256);
  DevArena tmp;
  struct G {
    DevArena& a;
    ~G() { a.release(); }
  } guard{tmp};
  c64 *sg, *rp, *rq, *rhs, *mu, *u, *w;
  double* pts;
  ARENA_ALLOC(tmp, sg, n);
  ARENA_ALLOC(tmp, rp, n);
  ARENA_ALLOC(tmp, rq, n);
  ARENA_ALLOC(tmp, rhs, n);
  ARENA_ALLOC(tmp, mu, n);
  ARENA_ALLOC(tmp, u, n);
  ARENA_ALLOC(tmp, w, n);
  ARENA_ALLOC(tmp, pts, 3 * n_pts);
  BEM_HIP_TRY(hipMemcpyAsync(pts, pts_host, sizeof(double) * 3 * n_pts, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_sigma, dim3(nb), dim3(256), 0, s, beta, n, P.k, sg);
  BEM_LAUNCH_CHECK();
  int r = eval_field_adjoint(P, pts, n_pts, pobs, rp, rq, s);
  if (r) return r;
  hipLaunchKernelGGL(k_adj_rhs, dim3(nb), dim3(256), 0, s, rp, rq, sg, n, rhs);
  BEM_LAUNCH_CHECK();
  const bem_gmres_opts o = *opts;
  r = gmres_solve(P, sg, 1, rhs, mu, o.tol, o.restart > 0 ? o.restart : 50,
                  o.max_iter > 0 ? o.max_iter : 2000, o.mode, o.inner_tol, 0, info_a, s);
  if (r) return r;
  // w = Mq^H mu (float64 adjoint product)
  if ((r = fmm_apply_adjoint<double>(P, P.f64, mu, u, w, s))) return r;
  hipLaunchKernelGGL(k_grad, dim3(nb), dim3(256), 0, s, w, rq, p, n, P.k, grad);
  BEM_LAUNCH_CHECK();
  BEM_HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

int objective_grad(Problem& P, const c64* beta, const double* dir, const double* pts_host,
                   int n_pts, const bem_gmres_opts* opts, double* J, c64* grad, c64* p_out,
                   bem_gmres_info* info_f, bem_gmres_info* info_a, hipStream_t s) {
  const int64_t n = P.n;
  DevArena tmp;
  struct G {
    DevArena& a;
    ~G() { a.release(); }
  } guard{tmp};
  c64 *p, *pobs;
  ARENA_ALLOC(tmp, p, n);
  ARENA_ALLOC(tmp, pobs, n_pts);
  int r = objective_forward(P, beta, dir, pts_host, n_pts, opts, J, p, pobs, info_f, s);
  if (r) return r;
  if (p_out) {
    hipLaunchKernelGGL(k_copy, dim3(ceil_div(n, 256)), dim3(256), 0, s, p, n, p_out);
    BEM_LAUNCH_CHECK();
  }
  if (grad && (r = objective_backward(P, beta, p, pobs, pts_host, n_pts, opts, grad, info_a, s)))
    return r;
  BEM_HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

static void release_batch_cache(Problem& P);

void release_workspace(Problem& P) {
  if (P.solver_ws) {
    Workspace* W = (Workspace*)P.solver_ws;
    W->release();
    delete W;
    P.solver_ws = nullptr;
  }
  release_batch_cache(P);
}

// ---------------------------------------------------------------------------
// batched solves: many systems (problem, sigma, direction, rhs) advance in
// lockstep.  Every tick issues, for each active system, either a float64
// residual or one Arnoldi step on its problem's stream (systems of one problem
// share that stream and its product workspaces; different problems run
// concurrently), then synchronises once and does the small host-side work
// (norms, Givens rotations, decisions) for all systems.
// ---------------------------------------------------------------------------
// CGS2 step of every listed system (sys_idx[i] with basis size nk[i] and
// length n[i]) in five launches per ORTH_MAX_JOBS systems; each column lands
// in slot 0 of its system's pinned host buffer.
static int orth_batch(const OrthSysDev* tab, const std::vector<int>& sys_idx,
                      const std::vector<int>& nk, const std::vector<int64_t>& n,
                      hipStream_t s) {
  for (size_t a0 = 0; a0 < sys_idx.size(); a0 += ORTH_MAX_JOBS) {
    OrthTick t{};
    t.njobs = (int)std::min<size_t>(ORTH_MAX_JOBS, sys_idx.size() - a0);
    for (int a = 0; a < t.njobs; ++a) {
      if (nk[a0 + a] < 1 || nk[a0 + a] > MAX_NK) return -1;
      t.sys[a] = sys_idx[a0 + a];
      t.kofs[a + 1] = t.kofs[a] + nk[a0 + a];
      t.bofs[a + 1] = t.bofs[a] + (int)ceil_div(n[a0 + a], 256);
    }
    const dim3 gd(RED_BLOCKS, t.kofs[t.njobs]), gb(t.bofs[t.njobs]);
    hipLaunchKernelGGL(k_orth_dots, gd, dim3(RED_THREADS), 0, s, tab, t);
    BEM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_orth_update, gb, dim3(256), 0, s, tab, t, 0);
    BEM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_orth_dots, gd, dim3(RED_THREADS), 0, s, tab, t);
    BEM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_orth_update, gb, dim3(256), 0, s, tab, t, 1);
    BEM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_orth_normalise, gb, dim3(256), 0, s, tab, t);
    BEM_LAUNCH_CHECK();
  }
  return 0;
}

// Per-problem cache of the batched solver's buffers, kept across calls and
// freed with the plan (allocations and frees inside a call would cost more
// than a tick): system k of a problem in a batch uses slot k; slots k >= 1
// also hold product buffers of their own.  The first problem of a batch
// keeps the device table of the orthogonalisation operands.
struct BatchSlot {
  Workspace W;
  DevArena exec_arena;
  ExecBuf<float> x32;
  ExecBuf<double> x64;
  bool has_exec = false;
};
struct BatchCache {
  std::vector<BatchSlot*> slots;
  DevArena tab_arena;
  OrthSysDev* tab = nullptr;
  int tab_cap = 0;
};

static BatchCache& batch_cache_for(Problem& P) {
  if (!P.batch_cache) P.batch_cache = new BatchCache();
  return *(BatchCache*)P.batch_cache;
}

static void release_batch_cache(Problem& P) {
  if (!P.batch_cache) return;
  BatchCache* C = (BatchCache*)P.batch_cache;
  for (BatchSlot* sl : C->slots) {
    sl->W.release();
    sl->exec_arena.release();
    delete sl;
  }
  C->tab_arena.release();
  delete C;
  P.batch_cache = nullptr;
}

struct BatchSys {
  Problem* P = nullptr;
  int adjoint = 0;
  const c64* sigma = nullptr;
  const c64* b = nullptr;
  c64* x = nullptr;
  Workspace* W = nullptr;  // from the problem's batch cache
  // product buffers: the problem's own for its first system, else the
  // cache slot's
  ExecBuf<float>* X32 = nullptr;
  ExecBuf<double>* X64 = nullptr;
  int state = 0;  // 0 outer residual, 1 Arnoldi, 2 done
  bool first = true;
  double bn = 0, rn = 0, atol = 0, beta = 0;
  int j = 0, iters = 0, mv64 = 0, mv32 = 0, outer = 0, status = -4;
  std::vector<std::complex<double>> H, cs, sn, g;
  std::vector<double> hist;
};

int gmres_solve_batch(std::vector<Problem*>& probs, const std::vector<int>& adjoint,
                      const std::vector<const c64*>& sigma, const std::vector<const c64*>& b,
                      const std::vector<c64*>& x, double tol, int m, int max_iter, int mode,
                      double inner_tol, int use_x0, bem_gmres_info* infos, hipStream_t caller) {
  const int ns = (int)probs.size();
  std::vector<BatchSys> sys(ns);
  // every stage of the tick's products is launched once for all systems (on
  // the caller's stream, near field and leaf-level M2L on the plan's two side
  // streams, which the products of its problems use too)
  BatchStreams bs;
  bs.main = caller;
  bs.side = probs[0]->side;
  bs.side2 = probs[0]->side2;
  struct StreamGuard {
    BatchStreams& b;
    ~StreamGuard() {
      for (auto& e : b.ev)
        if (e) (void)hipEventDestroy(e);
    }
  } stream_guard{bs};
  for (auto& e : bs.ev)
    BEM_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventReleaseToDevice));
  hipStream_t s = caller;
  std::vector<std::pair<Problem*, int>> used;  // systems per problem so far
  for (int i = 0; i < ns; ++i) {
    BatchSys& S = sys[i];
    S.P = probs[i];
    S.adjoint = adjoint[i];
    S.sigma = sigma[i];
    S.b = b[i];
    S.x = x[i];
    int k = 0;
    for (auto& u : used)
      if (u.first == S.P) k = ++u.second;
    if (k == 0) used.push_back({S.P, 0});
    BatchCache& C = batch_cache_for(*S.P);
    while ((int)C.slots.size() <= k) C.slots.push_back(new BatchSlot());
    BatchSlot& sl = *C.slots[k];
    int r = sl.W.ensure(S.P->n, m);
    if (r) return r;
    S.W = &sl.W;
    if (k == 0) {
      S.X32 = &S.P->f32.X;
      S.X64 = &S.P->f64.X;
    } else {  // a further system of the same problem: buffers of its own
      if (!sl.has_exec) {
        if ((r = alloc_exec<float>(*S.P, S.P->f32, sl.x32, sl.exec_arena))) return r;
        if ((r = alloc_exec<double>(*S.P, S.P->f64, sl.x64, sl.exec_arena))) return r;
        sl.has_exec = true;
      }
      S.X32 = &sl.x32;
      S.X64 = &sl.x64;
    }
    S.H.assign((size_t)(m + 1) * m, 0.0);
    S.cs.assign(m, 0.0);
    S.sn.assign(m, 0.0);
    S.g.assign(m + 1, 0.0);
    S.first = !use_x0;
  }
  // device table of the per-system orthogonalisation operands (written for
  // every call: the slots of the systems depend on the batch)
  OrthSysDev* tab = nullptr;
  {
    BatchCache& C0 = batch_cache_for(*probs[0]);
    if (C0.tab_cap < ns) {
      C0.tab_arena.release();
      C0.tab = nullptr;
      C0.tab_cap = 0;
      const int cap = std::max(ns, 64);
      int r = C0.tab_arena.alloc((void**)&C0.tab, sizeof(OrthSysDev) * cap);
      if (r) return r;
      C0.tab_cap = cap;
    }
    tab = C0.tab;
    std::vector<OrthSysDev> h(ns);
    for (int i = 0; i < ns; ++i) {
      Workspace& W = *sys[i].W;
      h[i] = OrthSysDev{W.V, W.w, W.n, W.partial, W.partial2, W.h, W.h2, W.hcol};
    }
    BEM_HIP_TRY(hipMemcpyAsync(tab, h.data(), sizeof(OrthSysDev) * ns, hipMemcpyHostToDevice, s));
    BEM_HIP_TRY(hipStreamSynchronize(s));
  }
  std::vector<int> orth_sys, orth_nk;
  std::vector<int64_t> orth_n;
  // norms of the right-hand sides
  for (auto& S : sys) {
    int r = multidot(*S.W, S.b, S.P->n, S.P->n, 1, S.b, S.W->h2, s);
    if (r) return r;
    BEM_HIP_TRY(hipMemcpyAsync(S.W->hscal, S.W->h2, sizeof(c64), hipMemcpyDeviceToHost, s));
    if (S.first) {
      hipLaunchKernelGGL(k_set_zero, dim3(ceil_div(S.P->n, 256)), dim3(256), 0, s, S.x, S.P->n);
      BEM_LAUNCH_CHECK();
    }
  }
  BEM_HIP_TRY(hipStreamSynchronize(s));
  for (auto& S : sys) {
    S.bn = sqrt(S.W->hscal[0].re);
    if (!std::isfinite(S.bn)) {
      S.status = -6;
      S.state = 2;
    } else if (S.bn == 0.0) {
      S.status = 0;
      S.state = 2;
    }
  }
  for (int tick = 0; tick < 100000; ++tick) {
    bool any = false;
    // the tick's products: outer residuals (float64, of x) and Arnoldi steps
    // (of V_j), grouped by precision and direction into batched products
    std::vector<BatchItem<float>> it32[2];
    std::vector<BatchItem<double>> it64[2];
    std::vector<char> wants(ns, 0), is32(ns, 0);
    for (int i = 0; i < ns; ++i) {
      BatchSys& S = sys[i];
      if (S.state == 2) continue;
      any = true;
      if (S.state == 0 && S.first) continue;  // r = b: no product
      const int64_t n = S.P->n;
      const int nb = ceil_div(n, 256);
      const bool f32 = S.state == 1 && mode == 1;
      const c64* vin = S.state == 0 ? S.x : S.W->V + (int64_t)S.j * n;
      c64* vout = S.state == 0 ? S.W->t1 : S.W->w;
      const c64* q = nullptr;
      c64* out2 = nullptr;
      if (!S.adjoint && S.sigma) {  // q = sigma v
        hipLaunchKernelGGL(k_diag_mul, dim3(nb), dim3(256), 0, s, S.sigma, vin, n, 0, S.W->t3);
        BEM_LAUNCH_CHECK();
        q = S.W->t3;
      }
      if (S.adjoint && S.sigma) out2 = S.W->t3;
      wants[i] = 1;
      is32[i] = f32;
      if (f32)
        it32[S.adjoint].push_back(BatchItem<float>{S.P, &S.P->f32, S.X32, vin, q, vout, out2});
      else
        it64[S.adjoint].push_back(BatchItem<double>{S.P, &S.P->f64, S.X64, vin, q, vout, out2});
    }
    if (!any) break;
    for (int a = 0; a < 2; ++a) {
      int r = 0;
      if (!it32[a].empty() && (r = fmm_apply_batch<float>(it32[a], a == 1, bs))) return r;
      if (!it64[a].empty() && (r = fmm_apply_batch<double>(it64[a], a == 1, bs))) return r;
    }
    // per system: adjoint admittance term, then residual norm; the Arnoldi
    // systems' orthogonalisation is merged into one set of launches
    orth_sys.clear();
    orth_nk.clear();
    orth_n.clear();
    for (int i = 0; i < ns; ++i) {
      BatchSys& S = sys[i];
      if (S.state == 2) continue;
      const int64_t n = S.P->n;
      const int nb = ceil_div(n, 256);
      int r = 0;
      if (wants[i]) {
        c64* vout = S.state == 0 ? S.W->t1 : S.W->w;
        if (S.adjoint && S.sigma) {
          hipLaunchKernelGGL(k_add_conj_diag, dim3(nb), dim3(256), 0, s, vout, S.sigma, S.W->t3,
                             n, vout);
          BEM_LAUNCH_CHECK();
        }
        if (is32[i])
          ++S.mv32;
        else
          ++S.mv64;
      }
      if (S.state == 0) {
        if (S.first) {
          hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, s, S.b, n, S.W->r);
        } else {
          hipLaunchKernelGGL(k_sub, dim3(nb), dim3(256), 0, s, S.b, S.W->t1, n, S.W->r);
        }
        BEM_LAUNCH_CHECK();
        if ((r = multidot(*S.W, S.W->r, n, n, 1, S.W->r, S.W->h2, s))) return r;
        BEM_HIP_TRY(hipMemcpyAsync(S.W->hscal, S.W->h2, sizeof(c64), hipMemcpyDeviceToHost, s));
      } else {
        orth_sys.push_back(i);
        orth_nk.push_back(S.j + 1);
        orth_n.push_back(n);
      }
    }
    if (!orth_sys.empty()) {
      int r = orth_batch(tab, orth_sys, orth_nk, orth_n, s);
      if (r) return r;
    }
    BEM_HIP_TRY(hipStreamSynchronize(s));
    // host decisions
    for (auto& S : sys) {
      if (S.state == 2) continue;
      const int64_t n = S.P->n;
      const int nb = ceil_div(n, 256);
      if (S.state == 0) {
        S.first = false;
        S.rn = sqrt(S.W->hscal[0].re);
        S.hist.push_back(S.rn / S.bn);
        if (!std::isfinite(S.rn)) {
          S.status = -6;
          S.state = 2;
          continue;
        }
        if (S.rn <= tol * S.bn) {
          S.status = 0;
          S.state = 2;
          continue;
        }
        if (S.iters >= max_iter || (mode == 1 && S.outer >= 30)) {
          S.status = -4;
          S.state = 2;
          continue;
        }
        const double itol = (mode == 1) ? inner_target(S.outer, inner_tol, tol, S.bn, S.rn)
                                        : tol * S.bn / S.rn;
        S.atol = itol * S.rn;
        S.beta = S.rn;
        hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, s, S.W->r, n, S.W->V);
        BEM_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_scale, dim3(nb), dim3(256), 0, s, S.W->V, n, 1.0 / S.beta);
        BEM_LAUNCH_CHECK();
        std::fill(S.g.begin(), S.g.end(), 0.0);
        S.g[0] = S.beta;
        S.j = 0;
        S.state = 1;
      } else {
        const int j = S.j;
        std::vector<std::complex<double>> col(j + 2);
        for (int i = 0; i <= j; ++i)
          col[i] = std::complex<double>(S.W->hcol[i].re, S.W->hcol[i].im);
        double hn = sqrt(S.W->hcol[j + 1].re);
        col[j + 1] = hn;
        ++S.iters;
        if (!std::isfinite(hn)) {
          S.status = -6;
          S.state = 2;
          continue;
        }
        for (int i = 0; i < j; ++i) {
          std::complex<double> t = S.cs[i] * col[i] + S.sn[i] * col[i + 1];
          col[i + 1] = -std::conj(S.sn[i]) * col[i] + std::conj(S.cs[i]) * col[i + 1];
          col[i] = t;
        }
        double den = std::sqrt(std::norm(col[j]) + std::norm(col[j + 1]));
        if (den == 0.0) {
          S.cs[j] = 1.0;
          S.sn[j] = 0.0;
        } else {
          S.cs[j] = std::conj(col[j]) / den;
          S.sn[j] = std::conj(col[j + 1]) / den;
        }
        col[j] = S.cs[j] * col[j] + S.sn[j] * col[j + 1];
        S.g[j + 1] = -std::conj(S.sn[j]) * S.g[j];
        S.g[j] = S.cs[j] * S.g[j];
        for (int i = 0; i <= j; ++i) S.H[i * m + j] = col[i];
        double est = std::abs(S.g[j + 1]);
        S.hist.push_back(est / S.bn);
        if (est <= S.atol || hn == 0.0 || j + 1 == m || S.iters >= max_iter) {
          int jend = j + 1;
          std::vector<std::complex<double>> yv(jend);
          for (int i = jend - 1; i >= 0; --i) {
            std::complex<double> acc = S.g[i];
            for (int kk = i + 1; kk < jend; ++kk) acc -= S.H[i * m + kk] * yv[kk];
            if (std::abs(S.H[i * m + i]) == 0.0) {
              acc = 0.0;
              yv[i] = 0.0;
              continue;
            }
            yv[i] = acc / S.H[i * m + i];
          }
          c64* yh = S.W->hcol + (S.W->m + 2);
          for (int i = 0; i < jend; ++i) yh[i] = mk(yv[i].real(), yv[i].imag());
          BEM_HIP_TRY(hipMemcpyAsync(S.W->y, yh, sizeof(c64) * jend,
                                     hipMemcpyHostToDevice, s));
          hipLaunchKernelGGL(k_combine, dim3(nb), dim3(256), 0, s, S.W->V, n, n, jend, S.W->y, S.x);
          BEM_LAUNCH_CHECK();
          ++S.outer;
          S.state = 0;
        } else {
          S.j = j + 1;
        }
      }
    }
  }
  BEM_HIP_TRY(hipStreamSynchronize(s));
  int worst = 0;
  for (int i = 0; i < ns; ++i) {
    BatchSys& S = sys[i];
    if (infos) {
      bem_gmres_info* info = infos + i;
      std::memset(info, 0, sizeof(*info));
      info->iterations = S.iters;
      info->matvec64 = S.mv64;
      info->matvec32 = S.mv32;
      info->restarts = S.outer;
      info->resid = (S.bn > 0) ? S.rn / S.bn : 0.0;
      info->converged = S.status == 0;
      int nh = std::min((int)S.hist.size(), 512);
      info->n_hist = nh;
      for (int t = 0; t < nh; ++t) info->hist[t] = S.hist[t];
    }
    if (S.status != 0 && worst == 0) worst = S.status;
  }
  if (worst == -4) set_error("some systems of the batch did not converge (see infos)");
  if (worst == -6) set_error("NaN or Inf met in a system of the batch");
  return worst;
}

}  // namespace bemfmm
