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
// (K - omega^2 M) X = N by Gauss-Jordan elimination with partial pivoting
// on the augmented matrix [A | N] (one launch per step for the pivot, the
// row swap and scaling, and the elimination), then forms C once (n_tri^2
// doubles); each product then costs one dense real-by-complex matrix-vector
// product besides the FMM.  Dense storage limits the body to BEM_FEM_MAX_DOF
// unknowns.
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

// Gauss-Jordan step k on the n x (n + m) augmented matrix (row stride ld):
// pivot: the largest |A[i][k]|, i >= k (one workgroup), its row and value
__global__ void __launch_bounds__(1024) k_gj_pivot(const double* __restrict__ A, int64_t n,
                                                   int64_t ld, int64_t k, int* __restrict__ piv,
                                                   double* __restrict__ pval) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  double best = -1.0;
  int bi = (int)k;
  for (int64_t i = k + threadIdx.x; i < n; i += blockDim.x) {
    const double a = fabs(A[i * ld + k]);
    if (a > best) {
      best = a;
      bi = (int)i;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      const double o = sv[threadIdx.x + h];
      const int oi = si[threadIdx.x + h];
      if (o > sv[threadIdx.x] || (o == sv[threadIdx.x] && oi < si[threadIdx.x])) {
        sv[threadIdx.x] = o;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *piv = si[0];
    *pval = A[(int64_t)si[0] * ld + k];
  }
}

// swap rows k and piv over the columns j > k, scale row k by 1 / pivot
__global__ void k_gj_swap(double* __restrict__ A, int64_t ld, int64_t k, int64_t ncol,
                          const int* __restrict__ piv, const double* __restrict__ pval) {
  const int64_t j = k + 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= ncol) return;
  const int64_t r = *piv;
  const double a = A[k * ld + j], b = A[r * ld + j];
  if (r != k) A[r * ld + j] = a;
  A[k * ld + j] = b / *pval;
}

// A[i][j] -= A[i][k] A[k][j] for i != k, j > k, with the multipliers of the
// swapped rows (column k is not swapped: row piv takes row k's entry; the
// column is never read after this step)
__global__ void k_gj_eliminate(double* __restrict__ A, int64_t n, int64_t ld, int64_t k,
                               int64_t ncol, const int* __restrict__ piv,
                               const double* __restrict__ pval) {
  const int64_t j = k + 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j >= ncol || i == k) return;
  const int64_t r = *piv;
  // multiplier of row i after the swap (column k itself is not updated)
  const double f = (i == r) ? A[k * ld + k] : A[i * ld + k];
  A[i * ld + j] -= f * A[k * ld + j];
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

// q = C v (real n x n, complex v): one wave per row
__global__ void __launch_bounds__(256) k_real_matvec(const double* __restrict__ C, int64_t n,
                                                     const c64* __restrict__ v,
                                                     c64* __restrict__ q) {
  const int64_t row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  double sr = 0.0, si = 0.0;
  for (int64_t c = lane; c < n; c += 64) {
    const double a = C[row * n + c];
    sr += a * v[c].re;
    si += a * v[c].im;
  }
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_xor(sr, off, 64);
    si += __shfl_xor(si, off, 64);
  }
  if (lane == 0) q[row] = mk(sr, si);
}

// out += C^T w (real n x n, complex w): one thread per column
__global__ void k_real_matvec_t_add(const double* __restrict__ C, int64_t n,
                                    const c64* __restrict__ w, c64* __restrict__ out) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= n) return;
  double sr = 0.0, si = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    const double a = C[j * n + c];
    sr += a * w[j].re;
    si += a * w[j].im;
  }
  out[c] = cadd(out[c], mk(sr, si));
}

int coupling_build(Problem& P, const double* nodes_h, int64_t n_nodes, const int* tets_h,
                   int64_t n_tets, const int* tri_h, double lam, double mu, double rho_s,
                   double rho_f, double omega, DevArena& keep, double** C_out, hipStream_t s) {
  DevArena scratch;
  struct Guard {
    DevArena& a;
    ~Guard() { a.release(); }
  } guard{scratch};
  const int64_t ndof = 3 * n_nodes;
  const int ntri = (int)P.n;
  const int64_t ncol = ndof + ntri, ld = ncol;
  double *x, *A, *nt, *pval;
  int *tets, *tri, *piv;
  ARENA_ALLOC(scratch, x, 3 * n_nodes);
  ARENA_ALLOC(scratch, tets, 4 * n_tets);
  ARENA_ALLOC(scratch, tri, 3 * (int64_t)ntri);
  ARENA_ALLOC(scratch, A, ndof * ld);
  ARENA_ALLOC(scratch, nt, 3 * (int64_t)ntri);
  ARENA_ALLOC(scratch, piv, 1);
  ARENA_ALLOC(scratch, pval, 1);
  ARENA_ALLOC(keep, *C_out, (int64_t)ntri * ntri);
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
  for (int64_t k = 0; k < ndof; ++k) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(1024), 0, s, A, ndof, ld, k, piv, pval);
    const int64_t nj = ncol - k - 1;
    if (nj > 0) {
      hipLaunchKernelGGL(k_gj_swap, dim3(ceil_div(nj, 256)), dim3(256), 0, s, A, ld, k, ncol,
                         piv, pval);
      hipLaunchKernelGGL(k_gj_eliminate, dim3(ceil_div(nj, 256), ndof), dim3(256), 0, s, A,
                         ndof, ld, k, ncol, piv, pval);
    }
  }
  BEM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_fem_schur, dim3(ceil_div(ntri, 128), ntri), dim3(128), 0, s, A, ld, ndof,
                     tri, nt, ntri, -rho_f * omega * omega, *C_out);
  BEM_LAUNCH_CHECK();
  BEM_HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

int coupling_q(const double* C, int64_t n, const c64* v, c64* q, hipStream_t s) {
  hipLaunchKernelGGL(k_real_matvec, dim3(ceil_div(n, 4)), dim3(256), 0, s, C, n, v, q);
  BEM_LAUNCH_CHECK();
  return 0;
}

int coupling_qt_add(const double* C, int64_t n, const c64* w, c64* out, hipStream_t s) {
  hipLaunchKernelGGL(k_real_matvec_t_add, dim3(ceil_div(n, 256)), dim3(256), 0, s, C, n, w, out);
  BEM_LAUNCH_CHECK();
  return 0;
}

}  // namespace bemfmm
