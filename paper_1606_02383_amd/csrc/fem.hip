// BEM-FEM coupling of an elastic scatterer (Sec. 2.3).  The body is
// discretised with linear tetrahedra (weak form Eq. fem_2): stiffness K and
// consistent mass M of an isotropic material, the boundary pressure load
// -N p with N[3a+i, j] = A_j n_{j,i} / 3 (p constant on boundary triangle j,
// n into the fluid).  Eliminating the displacement from the coupled system
// (Eq. renritupu) gives the Schur form (Eqs. kousokuu, GMRES): the normal
// derivative of the pressure on the fluid side is q = C p with
//     C = -rho_f omega^2 Tc (K - omega^2 M)^(-1) N,   Tc[j, 3a+i] = n_{j,i} / 3
// (momentum balance dp/dn = rho_f omega^2 u.n at the collocation point, where
// the linear displacement equals its mean over the triangle), and every
// product of the coupled operator is the FMM product with (p, q = C p).
//
// The paper factorises K - omega^2 M once with a multi-frontal sparse solver;
// here the plan-time step assembles it densely on the device and solves
// (K - omega^2 M) X = N by a blocked LU with partial pivoting of the
// augmented matrix [A | N] (trailing updates on the matrix cores) and
// blocked back substitution, then forms C once (n_tri^2 doubles, and its
// transpose for the adjoint); each product then costs one dense
// real-by-complex matrix-vector product besides the FMM.  Dense storage
// limits the body to BEM_FEM_MAX_DOF unknowns.
#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "../../include/bemfmm.h"
#include "plan.h"

namespace bemfmm {

#define ARENA_ALLOC(arena, ptr, count)                                              \
  do {                                                                              \
    int _r = (arena).alloc((void**)&(ptr), sizeof(*(ptr)) * (size_t)(count));      \
    if (_r) return _r;                                                              \
  } while (0)

// Element matrices of tetrahedron e added into the dense A = K - omega^2 M
// (row stride ld): K_e[(a,i),(b,j)] = V (lam d_i phi_a d_j phi_b + mu
// (delta_ij grad phi_a . grad phi_b + d_j phi_a d_i phi_b)), M_e[(a,i),(b,j)]
// = delta_ij rho V (1 + delta_ab) / 20.
__global__ void k_fem_assemble(const double* __restrict__ x, const int* __restrict__ tets,
                               int64_t ntet, double lam, double mu, double rho_w2, int64_t ld,
                               double* __restrict__ A) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= ntet) return;
  int v[4];
  double X[4][3];
  for (int a = 0; a < 4; ++a) {
    v[a] = tets[4 * e + a];
    for (int i = 0; i < 3; ++i) X[a][i] = x[3 * (int64_t)v[a] + i];
  }
  // J = [x1 - x0, x2 - x0, x3 - x0] (columns); rows of J^-1 are the gradients
  // of phi_1..phi_3, grad phi_0 = -(their sum)
  double J[3][3];
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < 3; ++i) J[i][c] = X[c + 1][i] - X[0][i];
  const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  double Ji[3][3];
  Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  double g[4][3];
  for (int i = 0; i < 3; ++i) {
    g[1][i] = Ji[0][i];
    g[2][i] = Ji[1][i];
    g[3][i] = Ji[2][i];
    g[0][i] = -(Ji[0][i] + Ji[1][i] + Ji[2][i]);
  }
  const double V = fabs(det) / 6.0;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      const double gg = g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2];
      const double m = rho_w2 * V * (a == b ? 2.0 : 1.0) / 20.0;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double k = lam * g[a][i] * g[b][j] + mu * g[a][j] * g[b][i];
          if (i == j) k += mu * gg;
          const double val = V * k - (i == j ? m : 0.0);
          atomicAdd(&A[(3 * (int64_t)v[a] + i) * ld + 3 * (int64_t)v[b] + j], val);
        }
    }
}

// Columns ndof .. ndof + ntri - 1 of the augmented matrix: N[3a+i, j] =
// A_j n_{j,i} / 3 for the vertices a of triangle j; nt[3 j + i] = n_{j,i}
// (thread j writes column ndof + j alone).
__global__ void k_fem_load(const double* __restrict__ x, const int* __restrict__ tri, int ntri,
                           int64_t ndof, int64_t ld, double* __restrict__ A,
                           double* __restrict__ nt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ntri) return;
  const int v0 = tri[3 * j], v1 = tri[3 * j + 1], v2 = tri[3 * j + 2];
  double e1[3], e2[3], c[3];
  for (int i = 0; i < 3; ++i) {
    e1[i] = x[3 * (int64_t)v1 + i] - x[3 * (int64_t)v0 + i];
    e2[i] = x[3 * (int64_t)v2 + i] - x[3 * (int64_t)v0 + i];
  }
  c[0] = e1[1] * e2[2] - e1[2] * e2[1];
  c[1] = e1[2] * e2[0] - e1[0] * e2[2];
  c[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double len = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);  // 2 A_j
  const int vs[3] = {v0, v1, v2};
  for (int i = 0; i < 3; ++i) {
    nt[3 * j + i] = c[i] / len;
    for (int a = 0; a < 3; ++a) A[(3 * (int64_t)vs[a] + i) * ld + ndof + j] += c[i] / 6.0;
  }
}

// ---------------------------------------------------------------------------
// Blocked LU with partial pivoting of the augmented matrix W = [A | N]
// (n x ncol, row stride ld; panels of LU_B columns), then blocked back
// substitution with U: the right block of W ends as X = A^-1 N.  Per panel:
// column by column one launch (k_lu_step) for the pivot, the row swap, the
// multipliers and the rank-1 update inside the panel; then the panel's swaps
// (k_lu_laswp) and the unit-lower solve L11^-1 (k_lu_trsm) on the
// columns right of it, and the update W22 -= L21 U12 on the matrix cores
// (k_lu_gemm), the trailing one once per two panels.  The multipliers of
// earlier blocks are not swapped: the right block is eliminated in place, so
// they are never read again.
// ---------------------------------------------------------------------------
constexpr int LU_B = 64;

constexpr int LU_UR = 4;  // rows (waves) per block of the in-panel update

// (|value|, row) candidates: the larger value wins, the lower row on ties
__device__ __forceinline__ void lu_better(double& bv, int& bi, double v, int i) {
  if (v > bv || (v == bv && i < bi)) {
    bv = v;
    bi = i;
  }
}

// block-wide best of one candidate per thread (blockDim = 64 * LU_UR); every
// thread returns the winner's row
__device__ __forceinline__ int lu_block_best(double bv, int bi, double* sv, int* si) {
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(bv, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    lu_better(bv, bi, ov, oi);
  }
  if ((threadIdx.x & 63) == 0) {
    sv[threadIdx.x >> 6] = bv;
    si[threadIdx.x >> 6] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int t = 1; t < LU_UR; ++t) lu_better(sv[0], si[0], sv[t], si[t]);
  }
  __syncthreads();
  return si[0];
}

// The panel (rows k0..n-1, its kb columns) is factorised in two row-major
// n x 64 buffers: step s = kk - k0 reads B[s % 2] and writes B[(s + 1) % 2],
// so the pivot row and row kk that every block reads are never written in
// the same launch.  Row k0 + s is final after step s (in B[(s + 1) % 2]);
// the other rows after the last step (in B[kb % 2]).
//
// panel load: W -> B0, and each block's best candidate for the pivot of
// column k0 (one wave per row)
__global__ void __launch_bounds__(64 * LU_UR) k_lu_panel_load(const double* __restrict__ W,
                                                              int64_t n, int64_t ld, int64_t k0,
                                                              int kb, double* __restrict__ B0,
                                                              double* __restrict__ pmax,
                                                              int* __restrict__ pidx) {
  __shared__ double sv[LU_UR];
  __shared__ int si[LU_UR];
  const int w = threadIdx.x >> 6, c = threadIdx.x & 63;
  const int64_t i = k0 + blockIdx.x * (int64_t)LU_UR + w;
  double v = 0.0;
  if (i < n && c < kb) {
    v = W[i * ld + k0 + c];
    B0[(i - k0) * 64 + c] = v;
  }
  const bool cand = (i < n && c == 0);
  const int best = lu_block_best(cand ? fabs(v) : -1.0, cand ? (int)i : INT_MAX, sv, si);
  if (threadIdx.x == 0) {
    pmax[blockIdx.x] = sv[0];
    pidx[blockIdx.x] = best;
  }
}

// step kk of the panel: every block reduces the previous step's candidates
// (npart of them) to the pivot row r, then its waves stride over the rows
// i >= kk (one wave per row at a time, lane c = panel column) and write each
// row's new state: row kk takes the pivot row, row r takes row kk's old
// values, every row below keeps its multiplier l = W[i][kk] / pivot in
// column kk and updates the columns right of kk; while column kk + 1 is in
// the panel each block leaves its best candidate (rows > kk) for it.  At
// most LU_STEP_BLOCKS blocks (two per CU: fewer candidates for every block
// to reduce; 256 and 1024 measured slower).
constexpr int LU_STEP_BLOCKS = 512;
__global__ void __launch_bounds__(64 * LU_UR) k_lu_step(
    int64_t n, int64_t k0, int kb, int64_t kk, const double* __restrict__ Pin,
    double* __restrict__ Pout, const double* __restrict__ pin_max,
    const int* __restrict__ pin_idx, int npart, double* __restrict__ pout_max,
    int* __restrict__ pout_idx, int* __restrict__ piv) {
  __shared__ double sv[LU_UR];
  __shared__ int si[LU_UR];
  __shared__ double prow[64], rowk[64];
  const int w = threadIdx.x >> 6, c = threadIdx.x & 63;
  const int ck = (int)(kk - k0);
  const double k_c = (threadIdx.x < 64 && c < kb) ? Pin[(kk - k0) * 64 + c] : 0.0;
  double bv = -1.0;
  int bi = (int)kk;
  for (int t = threadIdx.x; t < npart; t += blockDim.x) lu_better(bv, bi, pin_max[t], pin_idx[t]);
  if (threadIdx.x < 64) rowk[c] = k_c;
  const int64_t r = lu_block_best(bv, bi, sv, si);
  if (threadIdx.x < 64) prow[c] = c < kb ? Pin[(r - k0) * 64 + c] : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) piv[kk] = (int)r;
  __syncthreads();
  double cv = -1.0;
  int ci = INT_MAX;
  const int64_t stride = (int64_t)gridDim.x * LU_UR;
  for (int64_t i = kk + blockIdx.x * (int64_t)LU_UR + w; i < n; i += stride) {
    if (c >= kb) continue;
    double out;
    if (i == kk) {
      out = prow[c];
    } else {
      const double src_c = (i == r) ? rowk[c] : Pin[(i - k0) * 64 + c];
      const double src_k = (i == r) ? rowk[ck] : Pin[(i - k0) * 64 + ck];
      const double l = src_k / prow[ck];
      out = (c == ck) ? l : (c > ck ? src_c - l * prow[c] : src_c);
      lu_better(cv, ci, fabs(out), (int)i);
    }
    Pout[(i - k0) * 64 + c] = out;
  }
  if (ck + 1 < kb) {
    // the candidates sit in lane ck + 1 of each wave
    const bool cand = (c == ck + 1);
    const int best = lu_block_best(cand ? cv : -1.0, cand ? ci : INT_MAX, sv, si);
    if (threadIdx.x == 0) {
      pout_max[blockIdx.x] = sv[0];
      pout_idx[blockIdx.x] = best;
    }
  }
}

// panel store: the final rows back into W (one wave per row)
__global__ void __launch_bounds__(256) k_lu_panel_store(double* __restrict__ W, int64_t n,
                                                        int64_t ld, int64_t k0, int kb,
                                                        const double* __restrict__ B0,
                                                        const double* __restrict__ B1) {
  const int64_t i = k0 + blockIdx.x * (int64_t)4 + (threadIdx.x >> 6);
  const int c = threadIdx.x & 63;
  if (i >= n || c >= kb) return;
  const int64_t li = i - k0;
  const int b = li < kb ? (int)((li + 1) & 1) : (kb & 1);
  W[i * ld + k0 + c] = (b ? B1 : B0)[li * 64 + c];
}

// trailing columns j in [c0, ncol), one thread each: the panel's row swaps
__global__ void __launch_bounds__(256) k_lu_laswp(double* __restrict__ W, int64_t ld, int64_t k0,
                                                  int kb, int64_t c0, int64_t ncol,
                                                  const int* __restrict__ piv) {
  const int64_t j = c0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= ncol) return;
  for (int t = 0; t < kb; ++t) {
    const int64_t kk = k0 + t, r = piv[kk];
    if (r != kk) {
      const double a = W[kk * ld + j];
      W[kk * ld + j] = W[r * ld + j];
      W[r * ld + j] = a;
    }
  }
}

// columns j in [c0, ncol), one thread each, over the panel's rows k0..k0+kb-1:
// UPPER, x = U11^-1 x (U11 with its diagonal); else x = L11^-1 x (L11 unit
// lower).  The lower solve is the upper one on reversed rows and columns
// (index q = LU_B - 1 - r), so both run the same register-resident
// back substitution; the triangle is staged in LDS.
template <bool UPPER>
__global__ void __launch_bounds__(256) k_lu_trsm(double* __restrict__ W, int64_t ld, int64_t k0,
                                                 int kb, int64_t c0, int64_t ncol) {
  __shared__ double U[LU_B][LU_B + 1];
  for (int e = threadIdx.x; e < LU_B * LU_B; e += blockDim.x) {
    const int q = e / LU_B, u = e % LU_B;  // U[q][u], u >= q
    double v = (q == u) ? 1.0 : 0.0;
    if (u > q || (UPPER && u == q)) {
      const int r = UPPER ? q : LU_B - 1 - q, t = UPPER ? u : LU_B - 1 - u;
      if (r < kb && t < kb) v = W[(k0 + r) * ld + k0 + t];
    }
    U[q][u] = v;
  }
  __syncthreads();
  const int64_t j = c0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= ncol) return;
  double x[LU_B];
#pragma unroll
  for (int q = 0; q < LU_B; ++q) {
    const int r = UPPER ? q : LU_B - 1 - q;
    x[q] = (r < kb) ? W[(k0 + r) * ld + j] : 0.0;
  }
#pragma unroll
  for (int q = LU_B - 1; q >= 0; --q) {
    double s = x[q];
#pragma unroll
    for (int u = q + 1; u < LU_B; ++u) s -= U[q][u] * x[u];
    x[q] = s / U[q][q];
  }
#pragma unroll
  for (int q = 0; q < LU_B; ++q) {
    const int r = UPPER ? q : LU_B - 1 - q;
    if (r < kb) W[(k0 + r) * ld + j] = x[q];
  }
}

// W[i][j] -= sum_{t < kb} W[i][k0 + t] W[k0 + t][j] for i in [r0, r1),
// j in [c0, c1): 64 x 64 output tiles, four waves of 2 x 2 float64 MFMA
// 16x16x4 blocks; the operands staged in LDS in chunks of 32 of the inner
// dimension, zero-padded (34 KB of LDS: four workgroups per CU).
// The operand columns / rows lie outside the output range in every use (the
// updates inside a block of panels, the trailing update, the back
// substitution).
typedef double lu_v4 __attribute__((ext_vector_type(4)));
constexpr int LU_KC = 32;  // inner-dimension chunk staged in LDS
__global__ void __launch_bounds__(256) k_lu_gemm(double* __restrict__ W, int64_t ld, int64_t r0,
                                                 int64_t r1, int64_t c0, int64_t c1, int64_t k0,
                                                 int kb) {
  __shared__ double As[64][LU_KC + 1];  // [row][t]
  __shared__ double Bs[LU_KC][64 + 1];  // [t][column]
  const int64_t ib = r0 + blockIdx.y * (int64_t)64, jb = c0 + blockIdx.x * (int64_t)64;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = w >> 1, wc = w & 1, lm = lane & 15, lk = lane >> 4;
  // this lane's 16 outputs, loaded first so that their latency overlaps the
  // staging of the operands
  double cv[2][2][4];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = ib + wr * 32 + x * 16 + 4 * e + lk;
        const int64_t j = jb + wc * 32 + y * 16 + lm;
        cv[x][y][e] = (i < r1 && j < c1) ? W[i * ld + j] : 0.0;
      }
  lu_v4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = lu_v4{0.0, 0.0, 0.0, 0.0};
  for (int tc = 0; tc < kb; tc += LU_KC) {
    if (tc > 0) __syncthreads();
    for (int e = threadIdx.x; e < 64 * LU_KC; e += 256) {
      const int rr = e / LU_KC, t = e % LU_KC;  // A: row rr, inner t
      const int64_t i = ib + rr;
      As[rr][t] = (i < r1 && tc + t < kb) ? W[i * ld + k0 + tc + t] : 0.0;
      const int tb = e / 64, cb = e % 64;      // B: inner tb, column cb
      const int64_t j = jb + cb;
      Bs[tb][cb] = (tc + tb < kb && j < c1) ? W[(k0 + tc + tb) * ld + j] : 0.0;
    }
    __syncthreads();
    // MFMA 16x16x4 float64 (wave64): A[m][k] from lane m + 16 k, B[k][n] from
    // lane n + 16 k; D[m][n] in lane n + 16 j, element e, m = 4 e + j
    const int tn = min(LU_KC, kb - tc);
    for (int t0 = 0; t0 < tn; t0 += 4) {
      double a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) a[x] = As[wr * 32 + x * 16 + lm][t0 + lk];
#pragma unroll
      for (int y = 0; y < 2; ++y) b[y] = Bs[t0 + lk][wc * 32 + y * 16 + lm];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = ib + wr * 32 + x * 16 + 4 * e + lk;
        const int64_t j = jb + wc * 32 + y * 16 + lm;
        if (i < r1 && j < c1) W[i * ld + j] = cv[x][y][e] - acc[x][y][e];
      }
}

static int lu_gemm(double* W, int64_t ld, int64_t r0, int64_t r1, int64_t c0, int64_t c1,
                   int64_t k0, int kb, hipStream_t s) {
  if (r1 <= r0 || c1 <= c0) return 0;
  hipLaunchKernelGGL(k_lu_gemm, dim3(ceil_div(c1 - c0, 64), ceil_div(r1 - r0, 64)), dim3(256), 0,
                     s, W, ld, r0, r1, c0, c1, k0, kb);
  BEM_LAUNCH_CHECK();
  return 0;
}

// X = A^-1 N in the right block of W (n x ncol)
// B: two n x 64 panel buffers; pmax / pidx: two candidate arrays of
// ceil(n / LU_UR) entries each
static int lu_swaps(double* W, int64_t ld, int64_t k0, int kb, int64_t c0, int64_t c1,
                    const int* piv, hipStream_t s) {
  if (c1 <= c0) return 0;
  hipLaunchKernelGGL(k_lu_laswp, dim3(ceil_div(c1 - c0, 256)), dim3(256), 0, s, W, ld, k0, kb, c0,
                     c1, piv);
  BEM_LAUNCH_CHECK();
  return 0;
}

static int lu_trsm_lower(double* W, int64_t ld, int64_t k0, int kb, int64_t c0, int64_t c1,
                         hipStream_t s) {
  if (c1 <= c0) return 0;
  hipLaunchKernelGGL(k_lu_trsm<false>, dim3(ceil_div(c1 - c0, 256)), dim3(256), 0, s, W, ld, k0, kb,
                     c0, c1);
  BEM_LAUNCH_CHECK();
  return 0;
}

// 64-column panel k0..k0+kb-1 over rows k0..n-1 (pivots into piv)
static int lu_panel(double* W, int64_t n, int64_t ld, int64_t k0, int kb, int* piv,
                    double* const B[2], double* const pmax[2], int* const pidx[2], hipStream_t s) {
  int npart = ceil_div(n - k0, LU_UR);
  hipLaunchKernelGGL(k_lu_panel_load, dim3(npart), dim3(64 * LU_UR), 0, s, W, n, ld, k0, kb, B[0],
                     pmax[0], pidx[0]);
  for (int st = 0; st < kb; ++st) {
    const int64_t kk = k0 + st;
    const int nb = std::min(ceil_div(n - kk, LU_UR), LU_STEP_BLOCKS);
    hipLaunchKernelGGL(k_lu_step, dim3(nb), dim3(64 * LU_UR), 0, s, n, k0, kb, kk, B[st & 1],
                       B[(st + 1) & 1], pmax[st & 1], pidx[st & 1], npart, pmax[(st + 1) & 1],
                       pidx[(st + 1) & 1], piv);
    npart = nb;
  }
  hipLaunchKernelGGL(k_lu_panel_store, dim3(ceil_div(n - k0, 4)), dim3(256), 0, s, W, n, ld, k0,
                     kb, B[0], B[1]);
  BEM_LAUNCH_CHECK();
  return 0;
}

// Blocks of LU_OB = 2 panels share one trailing update with an inner
// dimension of 128, so the trailing matrix is read and written once per 128
// columns.  Inside a block each panel first updates the block's own columns
// right of it; its row swaps also reach the multipliers of the block's
// earlier panel, which the trailing update reads.
constexpr int LU_OB = 2 * LU_B;
static int lu_solve_augmented(double* W, int64_t n, int64_t ncol, int* piv, double* const B[2],
                              double* const pmax[2], int* const pidx[2], hipStream_t s) {
  const int64_t ld = ncol;
  int r;
  for (int64_t K0 = 0; K0 < n; K0 += LU_OB) {
    const int KB = (int)std::min<int64_t>(LU_OB, n - K0);
    const int64_t K1 = K0 + KB;
    for (int64_t k0 = K0; k0 < K1; k0 += LU_B) {
      const int kb = (int)std::min<int64_t>(LU_B, K1 - k0);
      if ((r = lu_panel(W, n, ld, k0, kb, piv, B, pmax, pidx, s))) return r;
      if ((r = lu_swaps(W, ld, k0, kb, K0, k0, piv, s))) return r;
      if ((r = lu_swaps(W, ld, k0, kb, k0 + kb, K1, piv, s))) return r;
      if ((r = lu_trsm_lower(W, ld, k0, kb, k0 + kb, K1, s))) return r;
      if ((r = lu_gemm(W, ld, k0 + kb, n, k0 + kb, K1, k0, kb, s))) return r;
    }
    // the block's swaps and L11^-1 on the trailing columns, then W22 -= L21 U12
    if ((r = lu_swaps(W, ld, K0, KB, K1, ncol, piv, s))) return r;
    for (int64_t k0 = K0; k0 < K1; k0 += LU_B) {
      const int kb = (int)std::min<int64_t>(LU_B, K1 - k0);
      if ((r = lu_trsm_lower(W, ld, k0, kb, K1, ncol, s))) return r;
      if ((r = lu_gemm(W, ld, k0 + kb, K1, K1, ncol, k0, kb, s))) return r;
    }
    if ((r = lu_gemm(W, ld, K1, n, K1, ncol, K0, KB, s))) return r;
  }
  for (int64_t k0 = ((n - 1) / LU_B) * LU_B; k0 >= 0; k0 -= LU_B) {
    const int kb = (int)std::min<int64_t>(LU_B, n - k0);
    hipLaunchKernelGGL(k_lu_trsm<true>, dim3(ceil_div(ncol - n, 256)), dim3(256), 0, s, W, ld,
                       k0, kb, n, ncol);
    BEM_LAUNCH_CHECK();
    if ((r = lu_gemm(W, ld, 0, k0, n, ncol, k0, kb, s))) return r;
  }
  return 0;
}

// C[j][c] = -rho_f omega^2 sum_{a in tri j} sum_i n_{j,i} / 3 X[3a + i][c],
// X the solved right block of the augmented matrix
__global__ void k_fem_schur(const double* __restrict__ A, int64_t ld, int64_t ndof,
                            const int* __restrict__ tri, const double* __restrict__ nt, int ntri,
                            double coef, double* __restrict__ C) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (c >= ntri) return;
  double s = 0.0;
  for (int a = 0; a < 3; ++a) {
    const int64_t v = tri[3 * j + a];
    for (int i = 0; i < 3; ++i) s += nt[3 * j + i] * A[(3 * v + i) * ld + ndof + c];
  }
  C[(int64_t)j * ntri + c] = coef * s / 3.0;
}

// B = A^T (n x n), through 32 x 32 tiles in LDS so that both the reads and
// the writes are coalesced
__global__ void __launch_bounds__(256) k_transpose(const double* __restrict__ A, int64_t n,
                                                   double* __restrict__ B) {
  __shared__ double t[32][33];
  const int64_t bx = (int64_t)blockIdx.x * 32, by = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int j = ty; j < 32; j += 8) {
    const int64_t r = by + j, c = bx + tx;
    if (r < n && c < n) t[j][tx] = A[r * n + c];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int64_t r = bx + j, c = by + tx;
    if (r < n && c < n) B[r * n + c] = t[tx][j];
  }
}

// out = M v (ADD: out += M v) for a real row-major n x n M and complex v: one
// workgroup of four waves per row (enough loads in flight to stream the
// matrix), 16-byte loads of the row when n is even (every row then starts
// 16-byte aligned)
template <bool ADD>
__global__ void __launch_bounds__(256) k_real_matvec(const double* __restrict__ M, int64_t n,
                                                     const c64* __restrict__ v,
                                                     c64* __restrict__ out) {
  __shared__ double red[2][4];
  const int64_t row = blockIdx.x;
  const int t = threadIdx.x;
  const double* r = M + row * n;
  double sr = 0.0, si = 0.0;
  if ((n & 1) == 0) {
    const double2* r2 = reinterpret_cast<const double2*>(r);
    for (int64_t c = t; c < n / 2; c += 256) {
      const double2 a = r2[c];
      const c64 v0 = v[2 * c], v1 = v[2 * c + 1];
      sr += a.x * v0.re + a.y * v1.re;
      si += a.x * v0.im + a.y * v1.im;
    }
  } else {
    for (int64_t c = t; c < n; c += 256) {
      const double a = r[c];
      sr += a * v[c].re;
      si += a * v[c].im;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_xor(sr, off, 64);
    si += __shfl_xor(si, off, 64);
  }
  if ((t & 63) == 0) {
    red[0][t >> 6] = sr;
    red[1][t >> 6] = si;
  }
  __syncthreads();
  if (t == 0) {
    const c64 y = mk(red[0][0] + red[0][1] + red[0][2] + red[0][3],
                     red[1][0] + red[1][1] + red[1][2] + red[1][3]);
    out[row] = ADD ? cadd(out[row], y) : y;
  }
}

// flag = 1 if any of the n values is not finite
__global__ void k_any_nonfinite(const double* __restrict__ a, int64_t n, int* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(a[i]);
  if (bad) *flag = 1;
}

int coupling_build(Problem& P, const double* nodes_h, int64_t n_nodes, const int* tets_h,
                   int64_t n_tets, const int* tri_h, double lam, double mu, double rho_s,
                   double rho_f, double omega, DevArena& keep, double** C_out, double** Ct_out,
                   hipStream_t s) {
  DevArena scratch;
  struct Guard {
    DevArena& a;
    ~Guard() { a.release(); }
  } guard{scratch};
  const int64_t ndof = 3 * n_nodes;
  const int ntri = (int)P.n;
  const int64_t ncol = ndof + ntri, ld = ncol;
  double *x, *A, *nt, *pbuf, *pmax;
  int *tets, *tri, *piv, *pidx;
  ARENA_ALLOC(scratch, x, 3 * n_nodes);
  ARENA_ALLOC(scratch, tets, 4 * n_tets);
  ARENA_ALLOC(scratch, tri, 3 * (int64_t)ntri);
  ARENA_ALLOC(scratch, A, ndof * ld);
  ARENA_ALLOC(scratch, nt, 3 * (int64_t)ntri);
  ARENA_ALLOC(scratch, piv, ndof);
  ARENA_ALLOC(scratch, pbuf, 2 * ndof * 64);
  ARENA_ALLOC(scratch, pmax, 2 * (int64_t)ceil_div(ndof, LU_UR));
  ARENA_ALLOC(scratch, pidx, 2 * (int64_t)ceil_div(ndof, LU_UR));
  ARENA_ALLOC(keep, *C_out, (int64_t)ntri * ntri);
  ARENA_ALLOC(keep, *Ct_out, (int64_t)ntri * ntri);
  BEM_HIP_TRY(hipMemcpyAsync(x, nodes_h, sizeof(double) * 3 * n_nodes, hipMemcpyHostToDevice, s));
  BEM_HIP_TRY(hipMemcpyAsync(tets, tets_h, sizeof(int) * 4 * n_tets, hipMemcpyHostToDevice, s));
  BEM_HIP_TRY(hipMemcpyAsync(tri, tri_h, sizeof(int) * 3 * ntri, hipMemcpyHostToDevice, s));
  BEM_HIP_TRY(hipMemsetAsync(A, 0, sizeof(double) * ndof * ld, s));
  hipLaunchKernelGGL(k_fem_assemble, dim3(ceil_div(n_tets, 128)), dim3(128), 0, s, x, tets,
                     n_tets, lam, mu, rho_s * omega * omega, ld, A);
  BEM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_fem_load, dim3(ceil_div(ntri, 128)), dim3(128), 0, s, x, tri, ntri, ndof,
                     ld, A, nt);
  BEM_LAUNCH_CHECK();
  double* const Bp[2] = {pbuf, pbuf + ndof * 64};
  double* const pm[2] = {pmax, pmax + ceil_div(ndof, LU_UR)};
  int* const pi[2] = {pidx, pidx + ceil_div(ndof, LU_UR)};
  int r = lu_solve_augmented(A, ndof, ncol, piv, Bp, pm, pi, s);
  if (r) return r;
  hipLaunchKernelGGL(k_fem_schur, dim3(ceil_div(ntri, 128), ntri), dim3(128), 0, s, A, ld, ndof,
                     tri, nt, ntri, -rho_f * omega * omega, *C_out);
  BEM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_transpose, dim3(ceil_div(ntri, 32), ceil_div(ntri, 32)), dim3(32, 8), 0, s,
                     *C_out, (int64_t)ntri, *Ct_out);
  BEM_LAUNCH_CHECK();
  // a singular K - omega^2 M leaves C non-finite
  int* flag;
  ARENA_ALLOC(scratch, flag, 1);
  BEM_HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_any_nonfinite, dim3(1024), dim3(256), 0, s, *C_out, (int64_t)ntri * ntri,
                     flag);
  BEM_LAUNCH_CHECK();
  int hflag = 0;
  BEM_HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  BEM_HIP_TRY(hipStreamSynchronize(s));
  if (hflag) {
    set_error("K - omega^2 M is singular (omega^2 an eigenvalue of the free body)");
    return BEM_E_NAN;
  }
  return 0;
}

int coupling_apply(const double* M, int64_t n, const c64* v, c64* out, bool add, hipStream_t s) {
  if (n <= 0) return 0;
  if (add)
    hipLaunchKernelGGL(k_real_matvec<true>, dim3(n), dim3(256), 0, s, M, n, v, out);
  else
    hipLaunchKernelGGL(k_real_matvec<false>, dim3(n), dim3(256), 0, s, M, n, v, out);
  BEM_LAUNCH_CHECK();
  return 0;
}

}  // namespace bemfmm
