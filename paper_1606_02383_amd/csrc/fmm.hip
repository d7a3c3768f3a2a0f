// The FMM-accelerated Burton-Miller product and its exact adjoint.
//
//   y = (I/2 - K - alpha H) p + (S + alpha K' + (alpha/2) I) q
//
// (the paper's boundary integral equation, Sec. 2.3, combined with its
// normal derivative).  Per product, in float32 or float64:
//   gather   caller order -> Morton order, split by precision (also clears
//            the expansions accumulated further down)
//   P2P      3-point-rule direct sum over neighbouring leaves (U lists),
//            j != i, plus the near-field corrections (accurate - 3-point rule)
//   P2M      leaf multipoles from per-element matrices (monopole q, dipole p)
//   M2M      child -> parent, grouped by octant
//   M2L      interaction lists, grouped by translation vector
//   L2L      parent -> child
//   finish   per leaf: the leaf-level M2L sums, L2P, the P2P sums and the
//            float64 diagonal (I/2, alpha/2 I and self integrals), scatter
// The grouped translations are gather-GEMM-scatter kernels on the matrix
// cores: every pair of one group shares one dense matrix.  M2L writes one
// result per pair, summed per destination box in a fixed order afterwards
// (deterministic); the other translations add into their destinations.  The
// adjoint applies the conjugate transpose of every stage in reverse order
// with the same lists and matrices.
//
// Pair kernel (rv = x - y, u = 1/r, G = exp(ikr)/(4 pi r)):
//   coefficient of p_j: -(G_y + alpha G_xy)
//       = G [a1 (rv.n_y + alpha n_x.n_y) + alpha a2 (rv.n_x)(rv.n_y) u^2]
//   coefficient of q_j:  G + alpha G_x = G [1 + alpha a1 rv.n_x]
// with a1 = iku - u^2 and a2 = 3u^2 - k^2 - 3iku.
#include <cmath>

#include <algorithm>
#include <vector>

#include <hip/hip_ext.h>

#include "kernel_math.h"
#include "plan.h"

namespace bemfmm {

constexpr double INV_4PI_D = 0.07957747154594767;

// Burton-Miller coefficients (sp, sq) of a target point x (normal n_x)
// against one source element, summed over the element's three rule points
// y_q, without the per-point weight (rule weight x area / (4 pi), the same
// for the three points; the callers apply it).  With r = x - y_q, u = 1/|r|,
// G = e^{ikr} u, a1 = (-u^2, k u), a2 = (3 u^2 - k^2, -3 k u):
//   p coefficient  G [a1 (r.n_y + alpha n_x.n_y) + alpha a2 (r.n_x)(r.n_y) u^2]
//                  (-dG/dn_y - alpha d2G/dn_x dn_y)
//   q coefficient  G [1 + alpha a1 (r.n_x)]       (G + alpha dG/dn_x)
// The element is flat, so r.n_y = x.n_y - d with d = y_q.n_y the same for its
// three points; n_x.n_y is shared too: both are formed once per element.
// IMAG: alpha purely imaginary (alpha = i/k, the usual coupling), which
// drops the alpha_re products.
template <typename R, bool IMAG>
__device__ __forceinline__ void bm_elem(R xx, R xy, R xz, R nxx, R nxy, R nxz, const R* yq,
                                        R nyx, R nyy, R nyz, R d, R k, R k_turns, R alr, R ali,
                                        cplx<R>& sp, cplx<R>& sq) {
  const R nn = nxx * nyx + nxy * nyy + nxz * nyz;
  const R rny = xx * nyx + xy * nyy + xz * nyz - d;
  const R c1r = rny + alr * nn, c1i = ali * nn;  // rny + alpha nn
  const R k2 = k * k, m3k = R(-3) * k;
  const R ann = ali * nn, ali3 = R(3) * ali, alik2 = ali * k2;  // IMAG only
  R spr, spi, sqr, sqi;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const R rx = xx - yq[3 * q], ry = xy - yq[3 * q + 1], rz = xz - yq[3 * q + 2];
    const R r2 = rx * rx + ry * ry + rz * rz;
    const R u = rsqrt_r<R>(r2);
    const R r = r2 * u;
    R sn, cs;
    phase<R>(r, k, k_turns, &sn, &cs);
    const R Gr = cs * u, Gi = sn * u;
    const R u2 = u * u;
    const R rnx = rx * nxx + ry * nxy + rz * nxz;
    R fr, fi, gr, gi;
    if constexpr (IMAG) {
      // alpha = i ali; with w = u^2, s = rnx rny w (terms of the general
      // branch below, multiplied out):
      //   f = (ali k u (3 s - nn) - w rny,  ali (3 w - k^2) s + k u rny - ali nn w)
      //   g = (1 - ali k u rnx,  -ali w rnx)
      const R ku = k * u, aku = ali * ku;
      const R wr = u2 * rny, sc = rnx * wr;
      fr = fma(aku, fma(R(3), sc, -nn), -wr);
      fi = fma(fma(ali3, u2, -alik2), sc, fma(ku, rny, -u2 * ann));
      gr = fma(-aku, rnx, R(1));
      gi = -(ali * u2) * rnx;
    } else {
      const R a1r = -u2, a1i = k * u;
      // a2 rnx rny u^2 = (t, v) with a2 = (3 u^2 - k^2, -3 k u)
      const R sc = rnx * rny * u2;
      const R t = (R(3) * u2 - k2) * sc, v = m3k * u * sc;
      // f = a1 (rny + alpha nn) + alpha (t, v);  g = 1 + alpha a1 rnx
      fr = a1r * c1r - a1i * c1i + alr * t - ali * v;
      fi = a1r * c1i + a1i * c1r + alr * v + ali * t;
      gr = R(1) + (alr * a1r - ali * a1i) * rnx;
      gi = (alr * a1i + ali * a1r) * rnx;
    }
    // G f and G g, the first point's as the start of the sums (no additions
    // of zero), then fused multiply-adds
    if (q == 0) {
      spr = Gr * fr;
      spi = Gr * fi;
      sqr = Gr * gr;
      sqi = Gr * gi;
    } else {
      spr = fma(Gr, fr, spr);
      spi = fma(Gr, fi, spi);
      sqr = fma(Gr, gr, sqr);
      sqi = fma(Gr, gi, sqi);
    }
    spr = fma(-Gi, fi, spr);
    spi = fma(Gi, fr, spi);
    sqr = fma(-Gi, gi, sqr);
    sqi = fma(Gi, gr, sqi);
  }
  sp = mk<R>(spr, spi);
  sq = mk<R>(sqr, sqi);
}

// A launch may cover several problems or levels ("jobs", at most MAX_JOBS):
// work item v belongs to the job q with first[q] <= v < first[q + 1].
constexpr int MAX_JOBS = 8;

// the job of a (workgroup-uniform) index, selected without dynamic indexing
// of the kernel argument
template <typename T, int N>
__device__ __forceinline__ T select_job(const T (&arr)[N], int q) {
  T v = arr[0];
#pragma unroll
  for (int i = 1; i < N; ++i)
    if (i == q) v = arr[i];
  return v;
}

template <int N>
__device__ __forceinline__ int job_of(const int (&first)[N], int njobs, int v) {
  int q = 0;
#pragma unroll
  for (int i = 1; i < N - 1; ++i)
    if (i < njobs && v >= first[i]) q = i;
  return q;
}

// Launch whose completion signals `done` (when non-null) as part of the
// dispatch itself: fork and join points between streams then need no
// separate event record (a marker that costs the stream an extra gap).
// `start` (timing events only) brackets the launch for profiling.
template <typename... KArgs, typename... Args>
static void launch_done(void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t lds,
                        hipStream_t s, hipEvent_t start, hipEvent_t done, Args... args) {
  if (done || start)
    hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, s, start, done, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

// ---------------------------------------------------------------------------
// gather / scatter
// ---------------------------------------------------------------------------
// Buffers cleared by the first kernel of a product (targets of atomic
// accumulation further down the chain), folded into it to save launches.
constexpr int MAX_ZERO = MAX_LEVEL;  // every level above the leaves
template <typename R, int NZ = MAX_ZERO>
struct ZeroList {
  int n;
  cplx<R>* ptr[NZ];
  int64_t cnt[NZ];
};

// clears the listed buffers; thread gid of gsz threads takes entries gid,
// gid + gsz, ...
template <typename R, int NZ>
__device__ __forceinline__ void zero_list(const ZeroList<R, NZ>& z, int64_t gid, int64_t gsz) {
#pragma unroll
  for (int q = 0; q < NZ; ++q) {
    if (q >= z.n) break;
    for (int64_t i = gid; i < z.cnt[q]; i += gsz) z.ptr[q][i] = mk<R>(R(0), R(0));
  }
}

__device__ __forceinline__ int64_t grid_tid() {
  return blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
}
__device__ __forceinline__ int64_t grid_threads() { return (int64_t)gridDim.x * blockDim.x; }

template <typename R>
__global__ void k_gather_in(const c64* __restrict__ p, const c64* __restrict__ q,
                            const int* __restrict__ perm, int64_t n, cplx<R>* __restrict__ ps,
                            cplx<R>* __restrict__ qs, c64* __restrict__ p64,
                            c64* __restrict__ q64, const ZeroList<R> zl) {
  zero_list(zl, grid_tid(), grid_threads());
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int o = perm[i];
  c64 a = p ? p[o] : mk(0.0, 0.0);
  c64 b = q ? q[o] : mk(0.0, 0.0);
  ps[i] = mk<R>((R)a.re, (R)a.im);
  qs[i] = mk<R>((R)b.re, (R)b.im);
  p64[i] = a;
  q64[i] = b;
}


// ---------------------------------------------------------------------------
// P2P: one block per leaf; sources of the U list staged in LDS in chunks
// ---------------------------------------------------------------------------
constexpr int P2P_THREADS = 256;
constexpr int P2P_CHUNK = 128;

// one problem's near field in a (possibly multi-problem) P2P launch; the
// forward kernel reads ps, qs and writes ys, the adjoint one reads ps (the
// sorted y) and writes ys, ys2 (u, w)
template <typename R>
struct P2PJobDev {
  const R* geo;
  int64_t n;
  const int* bstart;
  const int* u_ptr;
  const int* u_idx;
  const cplx<R>* ps;
  const cplx<R>* qs;
  cplx<R>* ys;
  cplx<R>* ys2;
  R k, alr, ali;
  int all_src;
  int q_zero;  // q = 0 (forward) or w not wanted (adjoint): the q terms are left out
  // near-field corrections (accurate minus rule integrals): CSR by target
  // element (forward) or by source element (adjoint)
  const int* nptr;
  const int* nidx;
  const cplx<R>* ncp;
  const cplx<R>* ncq;
};
template <typename R>
struct P2PBatch {
  int n;      // jobs
  int total;  // leaves of all jobs
  int leaf0[MAX_JOBS + 1];
  P2PJobDev<R> job[MAX_JOBS];
};

// QZ: q = 0 for every job of the launch; the q coefficients, densities and
// corrections are left out (they would meet zeros)
template <typename R, bool IMAG, bool QZ>
__global__ void __launch_bounds__(P2P_THREADS) k_p2p(const P2PBatch<R> batch) {
  __shared__ R s_q[9][P2P_CHUNK];
  __shared__ R s_n[4][P2P_CHUNK];  // normal and plane offset y . n
  __shared__ R s_pq[4][P2P_CHUNK];
  __shared__ int s_id[P2P_CHUNK];
  __shared__ int s_nb[28], s_pre[28];
  __shared__ cplx<R> s_red[P2P_THREADS];
  const int tid = threadIdx.x;
  // grid-stride over the leaves of all jobs (the grid may be capped)
  for (int vb = blockIdx.x; vb < batch.total; vb += gridDim.x) {
  __syncthreads();  // the previous leaf no longer reads the shared arrays
  const int qj = job_of(batch.leaf0, batch.n, vb);
  const P2PJobDev<R> J = select_job(batch.job, qj);
  const int b = vb - select_job(batch.leaf0, qj);
  const R* __restrict__ geo = J.geo;
  const int64_t n = J.n;
  const int* __restrict__ bstart = J.bstart;
  const int* __restrict__ u_ptr = J.u_ptr;
  const int* __restrict__ u_idx = J.u_idx;
  const cplx<R>* __restrict__ ps = J.ps;
  const cplx<R>* __restrict__ qs = J.qs;
  cplx<R>* __restrict__ ys = J.ys;
  const R k = J.k, alr = J.alr, ali = J.ali;
  const int all_src = J.all_src;
  const R k_turns = k * R(0.15915494309189535);  // k / (2 pi)
  const int t0 = bstart[b], nT = bstart[b + 1] - t0;
  const int u0 = u_ptr[b], nu = u_ptr[b + 1] - u0;
  if (tid == 0) {
    int acc = 0;
    if (all_src) {  // every element is a source (direct sum)
      s_nb[0] = 0;
      s_pre[0] = 0;
      acc = (int)n;
    } else {
      for (int t = 0; t < nu; ++t) {
        int nb = u_idx[u0 + t];
        s_nb[t] = bstart[nb];
        s_pre[t] = acc;
        acc += bstart[nb + 1] - bstart[nb];
      }
    }
    s_pre[all_src ? 1 : nu] = acc;
  }
  __syncthreads();
  const int total = s_pre[all_src ? 1 : nu];
  const int nseg = all_src ? 1 : nu;
  for (int tg = 0; tg < nT; tg += P2P_THREADS) {
    const int nTg = min(P2P_THREADS, nT - tg);
    const int nsl = P2P_THREADS / nTg;
    const bool active = tid < nTg * nsl;
    const int ti = tid % nTg, sl = tid / nTg;
    const int i = t0 + tg + ti;
    R xx = 0, xy = 0, xz = 0, nxx = 0, nxy = 0, nxz = 0;
    if (active) {
      xx = geo[GEO_CX * n + i];
      xy = geo[GEO_CY * n + i];
      xz = geo[GEO_CZ * n + i];
      nxx = geo[GEO_NX * n + i];
      nxy = geo[GEO_NY * n + i];
      nxz = geo[GEO_NZ * n + i];
    }
    cplx<R> acc = mk<R>(0, 0);
    for (int c0 = 0; c0 < total; c0 += P2P_CHUNK) {
      const int cnt = min(P2P_CHUNK, total - c0);
      __syncthreads();
      for (int v = tid; v < cnt; v += P2P_THREADS) {
        int gv = c0 + v, t = 0;
        while (t + 1 < nseg && s_pre[t + 1] <= gv) ++t;
        int j = s_nb[t] + (gv - s_pre[t]);
        for (int c = 0; c < 9; ++c) s_q[c][v] = geo[(GEO_QX0 + c) * n + j];
        const R nx = geo[GEO_NX * n + j], ny = geo[GEO_NY * n + j], nz = geo[GEO_NZ * n + j];
        s_n[0][v] = nx;
        s_n[1][v] = ny;
        s_n[2][v] = nz;
        s_n[3][v] = s_q[0][v] * nx + s_q[1][v] * ny + s_q[2][v] * nz;
        // densities times the per-point weight (rule weight x area / (4 pi))
        const R wj = geo[GEO_AREA * n + j] * R(1.0 / 3.0) * R(INV_4PI_D);
        const cplx<R> pv = ps[j];
        s_pq[0][v] = wj * pv.re;
        s_pq[1][v] = wj * pv.im;
        if (!QZ) {
          const cplx<R> qv = qs[j];
          s_pq[2][v] = wj * qv.re;
          s_pq[3][v] = wj * qv.im;
        }
        s_id[v] = j;
      }
      __syncthreads();
      if (active) {
        for (int v = sl; v < cnt; v += nsl) {
          if (s_id[v] == i) continue;
          R yq[9];
#pragma unroll
          for (int c = 0; c < 9; ++c) yq[c] = s_q[c][v];
          cplx<R> sp, sq;
          bm_elem<R, IMAG>(xx, xy, xz, nxx, nxy, nxz, yq, s_n[0][v], s_n[1][v], s_n[2][v],
                           s_n[3][v], k, k_turns, alr, ali, sp, sq);
          cfma(acc, sp, mk<R>(s_pq[0][v], s_pq[1][v]));
          if (!QZ) cfma(acc, sq, mk<R>(s_pq[2][v], s_pq[3][v]));
        }
      }
    }
    if (active) {  // near-field corrections of target i, split over the slices
      const int* __restrict__ nptr = J.nptr;
      for (int t = nptr[i] + sl; t < nptr[i + 1]; t += nsl) {
        const int j = J.nidx[t];
        cfma(acc, J.ncp[t], ps[j]);
        if (!QZ) cfma(acc, J.ncq[t], qs[j]);
      }
    }
    __syncthreads();
    s_red[tid] = active ? acc : mk<R>(0, 0);
    __syncthreads();
    if (tid < nTg) {
      cplx<R> s = mk<R>(0, 0);
      for (int q = 0; q < nsl; ++q) s = cadd(s, s_red[q * nTg + tid]);
      ys[t0 + tg + tid] = s;
    }
  }
  }
}

// Adjoint P2P: one block per leaf of output elements j; iterates over the
// target elements i of the U list:  u_j += conj(cp_ij) y_i,  w_j += conj(cq_ij) y_i.
// WZ: w not wanted by any job of the launch (rigid adjoint): the q
// coefficients and the w sums and corrections are left out
template <typename R, bool IMAG, bool WZ>
__global__ void __launch_bounds__(P2P_THREADS) k_p2p_adj(const P2PBatch<R> batch) {
  __shared__ R s_x[6][P2P_CHUNK];
  __shared__ R s_y[2][P2P_CHUNK];
  __shared__ int s_id[P2P_CHUNK];
  __shared__ int s_nb[28], s_pre[28];
  __shared__ cplx<R> s_red[4][P2P_THREADS];
  const int tid = threadIdx.x;
  // grid-stride over the leaves of all jobs (the grid may be capped)
  for (int vb = blockIdx.x; vb < batch.total; vb += gridDim.x) {
  __syncthreads();  // the previous leaf no longer reads the shared arrays
  const int qj = job_of(batch.leaf0, batch.n, vb);
  const P2PJobDev<R> J = select_job(batch.job, qj);
  const int b = vb - select_job(batch.leaf0, qj);
  const R* __restrict__ geo = J.geo;
  const int64_t n = J.n;
  const int* __restrict__ bstart = J.bstart;
  const int* __restrict__ u_ptr = J.u_ptr;
  const int* __restrict__ u_idx = J.u_idx;
  const cplx<R>* __restrict__ ysrt = J.ps;
  cplx<R>* __restrict__ us = J.ys;
  cplx<R>* __restrict__ ws = J.ys2;
  const R k = J.k, alr = J.alr, ali = J.ali;
  const int all_src = J.all_src;
  const R k_turns = k * R(0.15915494309189535);  // k / (2 pi)
  const int t0 = bstart[b], nT = bstart[b + 1] - t0;
  const int u0 = u_ptr[b], nu = u_ptr[b + 1] - u0;
  if (tid == 0) {
    int acc = 0;
    if (all_src) {  // every element is a source (direct sum)
      s_nb[0] = 0;
      s_pre[0] = 0;
      acc = (int)n;
    } else {
      for (int t = 0; t < nu; ++t) {
        int nb = u_idx[u0 + t];
        s_nb[t] = bstart[nb];
        s_pre[t] = acc;
        acc += bstart[nb + 1] - bstart[nb];
      }
    }
    s_pre[all_src ? 1 : nu] = acc;
  }
  __syncthreads();
  const int total = s_pre[all_src ? 1 : nu];
  const int nseg = all_src ? 1 : nu;
  for (int tg = 0; tg < nT; tg += P2P_THREADS) {
    const int nTg = min(P2P_THREADS, nT - tg);
    const int nsl = P2P_THREADS / nTg;
    const bool active = tid < nTg * nsl;
    const int ti = tid % nTg, sl = tid / nTg;
    const int j = t0 + tg + ti;
    R q[9], nyx = 0, nyy = 0, nyz = 0;
    for (int c = 0; c < 9; ++c) q[c] = active ? geo[(GEO_QX0 + c) * n + j] : R(0);
    if (active) {
      nyx = geo[GEO_NX * n + j];
      nyy = geo[GEO_NY * n + j];
      nyz = geo[GEO_NZ * n + j];
    }
    const R dj = q[0] * nyx + q[1] * nyy + q[2] * nyz;  // plane offset of element j
    cplx<R> au = mk<R>(0, 0), aw = mk<R>(0, 0);
    for (int c0 = 0; c0 < total; c0 += P2P_CHUNK) {
      const int cnt = min(P2P_CHUNK, total - c0);
      __syncthreads();
      for (int v = tid; v < cnt; v += P2P_THREADS) {
        int gv = c0 + v, t = 0;
        while (t + 1 < nseg && s_pre[t + 1] <= gv) ++t;
        int i = s_nb[t] + (gv - s_pre[t]);
        s_x[0][v] = geo[GEO_CX * n + i];
        s_x[1][v] = geo[GEO_CY * n + i];
        s_x[2][v] = geo[GEO_CZ * n + i];
        s_x[3][v] = geo[GEO_NX * n + i];
        s_x[4][v] = geo[GEO_NY * n + i];
        s_x[5][v] = geo[GEO_NZ * n + i];
        cplx<R> yv = ysrt[i];
        s_y[0][v] = yv.re;
        s_y[1][v] = yv.im;
        s_id[v] = i;
      }
      __syncthreads();
      if (active) {
        for (int v = sl; v < cnt; v += nsl) {
          if (s_id[v] == j) continue;
          cplx<R> sp, sq;
          bm_elem<R, IMAG>(s_x[0][v], s_x[1][v], s_x[2][v], s_x[3][v], s_x[4][v], s_x[5][v], q,
                           nyx, nyy, nyz, dj, k, k_turns, alr, ali, sp, sq);
          cplx<R> yv = mk<R>(s_y[0][v], s_y[1][v]);
          cfmac(au, sp, yv);
          if (!WZ) cfmac(aw, sq, yv);
        }
      }
    }
    // transposed near-field corrections of source j, split over the slices
    cplx<R> cu = mk<R>(0, 0), cw = mk<R>(0, 0);
    if (active) {
      const int* __restrict__ nptr = J.nptr;
      for (int t = nptr[j] + sl; t < nptr[j + 1]; t += nsl) {
        const cplx<R> yv = ysrt[J.nidx[t]];
        cfmac(cu, J.ncp[t], yv);
        if (!WZ) cfmac(cw, J.ncq[t], yv);
      }
    }
    __syncthreads();
    s_red[0][tid] = active ? au : mk<R>(0, 0);
    s_red[1][tid] = active ? aw : mk<R>(0, 0);
    s_red[2][tid] = cu;
    s_red[3][tid] = cw;
    __syncthreads();
    if (tid < nTg) {
      cplx<R> su = mk<R>(0, 0), sw = mk<R>(0, 0), scu = mk<R>(0, 0), scw = mk<R>(0, 0);
      for (int q2 = 0; q2 < nsl; ++q2) {
        su = cadd(su, s_red[0][q2 * nTg + tid]);
        sw = cadd(sw, s_red[1][q2 * nTg + tid]);
        scu = cadd(scu, s_red[2][q2 * nTg + tid]);
        scw = cadd(scw, s_red[3][q2 * nTg + tid]);
      }
      // per-point weight of element j (rule weight x area / (4 pi))
      const R wj = geo[GEO_AREA * n + t0 + tg + tid] * R(1.0 / 3.0) * R(INV_4PI_D);
      us[t0 + tg + tid] = cadd(cscale(su, wj), scu);
      if (!WZ) ws[t0 + tg + tid] = cadd(cscale(sw, wj), scw);
    }
  }
  }
}

// ---------------------------------------------------------------------------
// P2M (forward) and L2P^H (adjoint): per leaf, per coefficient sums over the
// leaf's elements.  mode 0: M[b][c] = sum_e A[e][c][0] p_e + A[e][c][1] q_e;
// mode 1: M[b][c] = sum_e conj(B[e][c]) y_e.
// ---------------------------------------------------------------------------
// two adjacent complex values in one wide load (16-byte aligned pair)
__device__ __forceinline__ void load_pair(const cplx<float>* p, cplx<float>& a, cplx<float>& b) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  a = mk<float>(v.x, v.y);
  b = mk<float>(v.z, v.w);
}
__device__ __forceinline__ void load_pair(const cplx<double>* p, cplx<double>& a,
                                          cplx<double>& b) {
  const double2 u = reinterpret_cast<const double2*>(p)[0];
  const double2 v = reinterpret_cast<const double2*>(p)[1];
  a = mk<double>(u.x, u.y);
  b = mk<double>(v.x, v.y);
}

// Per-leaf accumulation over the leaf's elements e:
//   mode 0 (P2M):     out[b][c] = sum_e mat[e][c][0] a_e + mat[e][c][1] bvec_e
//   mode 1 (L2P^H):   out[b][c] = sum_e conj(mat[e][c]) a_e
//   mode 2 (P2M, q = 0, mat = the p columns alone): out[b][c] = sum_e mat[e][c] a_e
// One 256-thread block per leaf: lane l of slice q handles coefficients
// l, l + 64, ... over the elements e0 + q, e0 + q + 4, ...; the four slices
// are added in a fixed order.
template <typename R>
struct LeafJobDev {
  const int* bstart;
  int ncoef;
  const cplx<R>* mat;
  const cplx<R>* a;
  const cplx<R>* bvec;
  cplx<R>* out;
};
template <typename R>
struct LeafBatch {
  int n, total;
  int leaf0[MAX_JOBS + 1];
  LeafJobDev<R> job[MAX_JOBS];
};

template <typename R>
__global__ void __launch_bounds__(256) k_leaf_accumulate(const LeafBatch<R> batch, int mode) {
  __shared__ cplx<R> part[4][64];
  __builtin_amdgcn_s_setprio(2);  // critical path: ahead of the near-field waves
  const int qj = job_of(batch.leaf0, batch.n, (int)blockIdx.x);
  const LeafJobDev<R> J = select_job(batch.job, qj);
  const int b = (int)blockIdx.x - select_job(batch.leaf0, qj);
  const int ncoef = J.ncoef;
  const cplx<R>* __restrict__ mat = J.mat;
  const cplx<R>* __restrict__ a = J.a;
  const cplx<R>* __restrict__ bvec = J.bvec;
  cplx<R>* __restrict__ out = J.out;
  const int e0 = J.bstart[b], e1 = J.bstart[b + 1];
  const int lane = threadIdx.x & 63, sl = threadIdx.x >> 6;
  for (int c0 = 0; c0 < ncoef; c0 += 64) {
    const int c = c0 + lane;
    cplx<R> acc = mk<R>(0, 0);
    if (c < ncoef) {
      for (int e = e0 + sl; e < e1; e += 4) {
        if (mode == 0) {
          cplx<R> mp, mq;
          load_pair(mat + ((int64_t)e * ncoef + c) * 2, mp, mq);
          cfma(acc, mp, a[e]);
          cfma(acc, mq, bvec[e]);
        } else if (mode == 2) {
          cfma(acc, mat[(int64_t)e * ncoef + c], a[e]);
        } else {
          cfmac(acc, mat[(int64_t)e * ncoef + c], a[e]);
        }
      }
    }
    part[sl][lane] = acc;
    __syncthreads();
    if (sl == 0 && c < ncoef)
      out[(int64_t)b * ncoef + c] =
          cadd(cadd(part[0][lane], part[1][lane]), cadd(part[2][lane], part[3][lane]));
    __syncthreads();
  }
}

// dynamic LDS of the leaf kernels (gather + leaf accumulation, leaf finish)
extern __shared__ double leaf_lds[];
constexpr size_t FUSED_LDS_MAX = 32768;  // bytes of leaf values in the fused gather

// The gather folded into the leaf accumulation (P2M, or L2P^H for the
// adjoint): block b gathers the elements of leaf b from the caller's order
// into the sorted float64 and working-precision copies (used by P2P and the
// finish) and into LDS, then forms the leaf expansion from them as
// k_leaf_accumulate does; the grid also clears the listed expansions.
// Dynamic LDS: (ADJ ? 1 : 2) * max_leaf values.
template <typename R, bool ADJ>
__global__ void __launch_bounds__(256)
    k_gather_leaf(const c64* __restrict__ p, const c64* __restrict__ q,
                  const int* __restrict__ perm, const int* __restrict__ bstart, int ncoef,
                  const cplx<R>* __restrict__ mat, cplx<R>* __restrict__ ps,
                  cplx<R>* __restrict__ qs, c64* __restrict__ p64, c64* __restrict__ q64,
                  cplx<R>* __restrict__ out, const ZeroList<R> zl) {
  __shared__ cplx<R> part[4][64];
  __builtin_amdgcn_s_setprio(2);  // critical path: ahead of the near-field waves
  cplx<R>* sa = reinterpret_cast<cplx<R>*>(leaf_lds);
  const int b = blockIdx.x;
  const int e0 = bstart[b], ne = bstart[b + 1] - e0;
  cplx<R>* sb = sa + ne;
  zero_list(zl, grid_tid(), grid_threads());
  for (int t = threadIdx.x; t < ne; t += blockDim.x) {
    const int e = e0 + t, o = perm[e];
    const c64 a = p ? p[o] : mk(0.0, 0.0);
    const cplx<R> ar = mk<R>((R)a.re, (R)a.im);
    ps[e] = ar;
    p64[e] = a;
    sa[t] = ar;
    if (!ADJ) {
      const c64 c = q ? q[o] : mk(0.0, 0.0);
      const cplx<R> cr = mk<R>((R)c.re, (R)c.im);
      qs[e] = cr;
      q64[e] = c;
      sb[t] = cr;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, sl = threadIdx.x >> 6;
  for (int c0 = 0; c0 < ncoef; c0 += 64) {
    const int c = c0 + lane;
    cplx<R> acc = mk<R>(0, 0);
    if (c < ncoef) {
      for (int t = sl; t < ne; t += 4) {
        const int64_t e = e0 + t;
        if (!ADJ && q) {
          cplx<R> mp, mq;
          load_pair(mat + (e * ncoef + c) * 2, mp, mq);
          cfma(acc, mp, sa[t]);
          cfma(acc, mq, sb[t]);
        } else if (!ADJ) {  // q = 0: mat holds the p columns alone
          cfma(acc, mat[e * ncoef + c], sa[t]);
        } else {
          cfmac(acc, mat[e * ncoef + c], sa[t]);
        }
      }
    }
    part[sl][lane] = acc;
    __syncthreads();
    if (sl == 0 && c < ncoef)
      out[(int64_t)b * ncoef + c] =
          cadd(cadd(part[0][lane], part[1][lane]), cadd(part[2][lane], part[3][lane]));
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// grouped gather-GEMM-scatter on the matrix cores:
//   dst[pair_dst] (+)= op_g src[pair_src]      (ADJ: op_g conjugate-transposed)
// Workgroup tile: 64 output rows x CT pairs (CT = 16, 32, 64 or 128; 8 waves
// for 128, else 4), operands staged through LDS in 16-wide k chunks, double
// buffered: the global loads of chunk c + 1 are in flight while chunk c runs
// on the matrix cores.  Complex products:
//   three real products per block (P1 = Ar Br, P2 = Ai Bi,
//   P3 = (Ar + Ai)(Br + Bi); C = (P1 - P2, P3 - P1 - P2)); float32 forms the
//   sums (Ar + Ai), (Br + Bi) once when staging (a third LDS plane),
//   float64 from the operands loaded from LDS.
// The output tile is staged in LDS and written as whole coefficient rows per
// pair (contiguous), either to the per-pair buffer, or added into the
// destination (plain read-modify-write where every destination of the launch
// receives one pair, else atomically).
// MFMA 16x16x4 operand layout (wave64): A[m][k] from lane m + 16 k, B[k][n]
// from lane n + 16 k.  Output D[m][n] sits in lane n + 16 j, element e, with
// m = 4 j + e for the float32 instruction and m = 4 e + j for the float64
// one (both measured on gfx950).
// ---------------------------------------------------------------------------
template <typename R>
struct MfmaOp;
template <>
struct MfmaOp<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int j, int e) { return 4 * j + e; }
};
template <>
struct MfmaOp<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int j, int e) { return 4 * e + j; }
};

constexpr int G_RT = 64, G_KC = 16, G_LD = G_KC + 1;

template <int CT>
struct TileShape {
  static constexpr int NW = (CT == 128) ? 8 : 4;         // waves
  static constexpr int WR = (NW == 8) ? 2 : (CT >= 32 ? 2 : 4);  // wave rows
  static constexpr int WC = NW / WR;                     // wave columns
  static constexpr int RB = G_RT / WR / 16;              // 16x16 blocks per wave
  static constexpr int CB = CT / WC / 16;
};

// One grouped product of a launch (a launch may cover several levels, each
// with its own operator, tiles, input and output; tiles of job q are the
// launch's tiles tile0[q] .. tile0[q + 1] - 1).
template <typename R>
struct GemmJobDev {
  int mat_rows, mat_cols;
  const int* tile_group;
  const int* tile_pair0;
  const int* tile_npairs;
  const int* tile_row0;
  const int* group_slot;
  const int* group_kc;  // input coefficients read per group (null: all)
  const int* pair_dst;
  const int* pair_src;
  const cplx<R>* mats;
  const cplx<R>* src;
  cplx<R>* dst;
  cplx<R>* cbuf;
};
template <typename R>
struct GemmBatch {
  int n;
  int ntiles;  // tile0[n]: the grid strides over them (grid <= ntiles, multiple of 8)
  int tile0[MAX_JOBS + 1];
  GemmJobDev<R> job[MAX_JOBS];
};


// KIND: 0 M2L (per-pair output), 1 M2M, 2 L2L, 3 leaf -> ancestor, 4
// ancestor -> leaf (the others add into dst)
// Two workgroups per CU: at most 128 registers for the 8-wave (128-pair)
// tiles, 256 for the 4-wave ones, so one tile's epilogue (the per-pair
// output write) overlaps the other's matrix products.
template <typename R, int CT, bool ADJ, int KIND>
__global__ void __launch_bounds__(64 * TileShape<CT>::NW)
    __attribute__((amdgpu_waves_per_eu(TileShape<CT>::NW == 8 ? 4 : 2)))
    k_grouped_gemm(const GemmBatch<R> batch) {
  typedef typename MfmaOp<R>::v4 v4;
  typedef TileShape<CT> S;
  // complex blocks as three real products (P1 = Ar Br, P2 = Ai Bi,
  // P3 = (Ar + Ai)(Br + Bi)); float32 stages the sums as a third LDS plane,
  // float64 (twice the LDS per value) forms them from the loaded operands
  constexpr bool STAGE3 = sizeof(R) == 4;
  constexpr int NP = STAGE3 ? 3 : 2;  // LDS planes: re, im (, re + im)
  constexpr int NT = 64 * S::NW;
  constexpr int PA = (G_RT * G_KC) / NT, PB = (CT * G_KC + NT - 1) / NT;
  constexpr int A_SZ = 2 * NP * G_RT * G_LD, B_SZ = 2 * NP * CT * G_LD;
  constexpr int OLD = G_RT + 1;  // staged output [pair][row], padded
  constexpr int MAIN = (A_SZ + B_SZ) * (int)sizeof(R);
  constexpr int OUTB = CT * OLD * 2 * (int)sizeof(R);
  __shared__ __attribute__((aligned(16))) char smem[MAIN > OUTB ? MAIN : OUTB];
  __shared__ int s_src[CT], s_dst[CT];
  R* As = (R*)smem;
  R* Bs = As + A_SZ;
  // XCD-aware order: workgroups go to the 8 XCDs round-robin (block b on XCD
  // b % 8), so give each XCD a contiguous range of tiles; consecutive tiles
  // share their group's matrix, which then stays in that XCD's L2.
  // Tiles are visited with a grid stride (a capped grid keeps room on the
  // compute units for work on other streams).  Virtual block vb =
  // blockIdx + i * gridDim keeps the XCD of blockIdx as the grid is a
  // multiple of 8 (or the whole tile count).
  // issue priority over the near-field waves sharing the compute unit (the
  // translations are on the product's critical path; the near field is not)
  __builtin_amdgcn_s_setprio(2);
  const int nt = batch.ntiles;
  for (int vb = blockIdx.x; vb < nt; vb += gridDim.x) {
  __syncthreads();  // the previous tile no longer reads the shared arrays
  const int xcd = vb & 7, slot_in_xcd = vb >> 3;
  const int gtile = xcd * (nt >> 3) + min(xcd, nt & 7) + slot_in_xcd;
  int q = 0;
#pragma unroll
  for (int i = 1; i < MAX_JOBS; ++i)
    if (i < batch.n && gtile >= batch.tile0[i]) q = i;
  const GemmJobDev<R> J = select_job(batch.job, q);
  const int tile = gtile - select_job(batch.tile0, q);
  const int mat_rows = J.mat_rows, mat_cols = J.mat_cols;
  const int* __restrict__ pair_src = J.pair_src;
  const cplx<R>* __restrict__ src = J.src;
  cplx<R>* __restrict__ dst = J.dst;
  cplx<R>* __restrict__ cbuf = J.cbuf;
  const int tid = threadIdx.x;
  const int grp = J.tile_group[tile], p0 = J.tile_pair0[tile], np = J.tile_npairs[tile];
  const int r0 = J.tile_row0[tile];
  const int slot = J.group_slot[grp];
  // translations across three boxes read fewer input coefficients (their
  // stored operator is zero beyond them)
  const int kc = J.group_kc ? min(mat_cols, J.group_kc[grp]) : mat_cols;
  const int out_rows = ADJ ? mat_cols : mat_rows;  // rows of the effective op
  const int in_cols = ADJ ? mat_rows : mat_cols;
  const cplx<R>* M = J.mats + (int64_t)slot * mat_rows * mat_cols;
  for (int t = tid; t < CT; t += NT) {
    s_src[t] = (t < np) ? pair_src[p0 + t] : -1;
    s_dst[t] = (t < np) ? J.pair_dst[p0 + t] : -1;
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = wave / S::WC, wc = wave % S::WC;
  const int li = lane & 15, lk = lane >> 4;
  v4 c0[S::RB][S::CB], c1[S::RB][S::CB], c2[S::RB][S::CB];
#pragma unroll
  for (int a = 0; a < S::RB; ++a)
#pragma unroll
    for (int b = 0; b < S::CB; ++b) {
      c0[a][b] = v4{0, 0, 0, 0};
      c1[a][b] = v4{0, 0, 0, 0};
      c2[a][b] = v4{0, 0, 0, 0};
    }
  cplx<R> ra[PA], rb[PB];
  // global -> registers for the chunk starting at k0
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      const int e = tid + NT * q;
      int kk, rr;
      if (ADJ) {  // consecutive threads walk a stored row (contiguous)
        rr = e % G_RT;
        kk = e / G_RT;
      } else {
        kk = e % G_KC;
        rr = e / G_KC;
      }
      const int r = r0 + rr, c = k0 + kk;
      cplx<R> v = mk<R>(0, 0);
      // (ADJ: the stored entry, conjugated when staged in LDS, so that no
      // use of the loaded value waits for the load inside this prefetch)
      if (r < out_rows && c < in_cols)
        v = ADJ ? M[(int64_t)c * mat_cols + r] : M[(int64_t)r * mat_cols + c];
      ra[q] = v;
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int e = tid + NT * q;
      const int kk = e % G_KC, cc = e / G_KC, c = k0 + kk;
      rb[q] = (cc < np && c < in_cols) ? src[(int64_t)s_src[cc] * in_cols + c] : mk<R>(0, 0);
    }
  };
  // registers -> LDS buffer buf
  auto store = [&](int buf) {
    R* A0 = As + (buf * NP) * G_RT * G_LD;
    R* B0 = Bs + (buf * NP) * CT * G_LD;
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      const int e = tid + NT * q;
      const int kk = ADJ ? e / G_RT : e % G_KC, rr = ADJ ? e % G_RT : e / G_KC;
      const R im = ADJ ? -ra[q].im : ra[q].im;  // ADJ: conjugate
      A0[rr * G_LD + kk] = ra[q].re;
      A0[G_RT * G_LD + rr * G_LD + kk] = im;
      if (STAGE3) A0[2 * G_RT * G_LD + rr * G_LD + kk] = ra[q].re + im;
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int e = tid + NT * q;
      const int kk = e % G_KC, cc = e / G_KC;
      if (cc < CT) {
        B0[cc * G_LD + kk] = rb[q].re;
        B0[CT * G_LD + cc * G_LD + kk] = rb[q].im;
        if (STAGE3) B0[2 * CT * G_LD + cc * G_LD + kk] = rb[q].re + rb[q].im;
      }
    }
  };
  const int nchunk = ((ADJ ? in_cols : kc) + G_KC - 1) / G_KC;
  load(0);
  store(0);
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nchunk) load((ch + 1) * G_KC);
    const R* A0 = As + (buf * NP) * G_RT * G_LD;
    const R* B0 = Bs + (buf * NP) * CT * G_LD;
#pragma unroll
    for (int ks = 0; ks < G_KC; ks += 4) {
      R a0[S::RB], a1[S::RB], a2[S::RB], b0[S::CB], b1[S::CB], b2[S::CB];
#pragma unroll
      for (int i = 0; i < S::RB; ++i) {
        const int o = (wr * (G_RT / S::WR) + i * 16 + li) * G_LD + ks + lk;
        a0[i] = A0[o];
        a1[i] = A0[G_RT * G_LD + o];
        a2[i] = STAGE3 ? A0[2 * G_RT * G_LD + o] : a0[i] + a1[i];
      }
#pragma unroll
      for (int j = 0; j < S::CB; ++j) {
        const int o = (wc * (CT / S::WC) + j * 16 + li) * G_LD + ks + lk;
        b0[j] = B0[o];
        b1[j] = B0[CT * G_LD + o];
        b2[j] = STAGE3 ? B0[2 * CT * G_LD + o] : b0[j] + b1[j];
      }
#pragma unroll
      for (int i = 0; i < S::RB; ++i)
#pragma unroll
        for (int j = 0; j < S::CB; ++j) {
          c0[i][j] = MfmaOp<R>::mma(a0[i], b0[j], c0[i][j]);
          c1[i][j] = MfmaOp<R>::mma(a1[i], b1[j], c1[i][j]);
          c2[i][j] = MfmaOp<R>::mma(a2[i], b2[j], c2[i][j]);
        }
    }
    if (ch + 1 < nchunk) store(buf ^ 1);
    __syncthreads();
  }
  // stage the tile [pair][row] in LDS (the operand buffers are free now)
  R* Os = (R*)smem;
#pragma unroll
  for (int i = 0; i < S::RB; ++i)
#pragma unroll
    for (int j = 0; j < S::CB; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = wr * (G_RT / S::WR) + i * 16 + MfmaOp<R>::row(lk, e);
        const int cc = wc * (CT / S::WC) + j * 16 + li;
        const R re = c0[i][j][e] - c1[i][j][e];
        const R im = c2[i][j][e] - c0[i][j][e] - c1[i][j][e];
        Os[(cc * OLD + row) * 2] = re;
        Os[(cc * OLD + row) * 2 + 1] = im;
      }
  __syncthreads();
  const int nrow = min(G_RT, out_rows - r0);
  for (int t = tid; t < CT * G_RT; t += NT) {
    const int cc = t / G_RT, row = t % G_RT;
    if (cc >= np || row >= nrow) continue;
    const cplx<R> v = mk<R>(Os[(cc * OLD + row) * 2], Os[(cc * OLD + row) * 2 + 1]);
    if (KIND == 0) {  // per-pair output, reduced per destination afterwards
      cbuf[(int64_t)(p0 + cc) * out_rows + r0 + row] = v;
    } else if ((KIND == 2 && !ADJ) || (KIND == 1 && ADJ)) {
      // parent -> child: every child is the destination of exactly one pair
      cplx<R>* d = &dst[(int64_t)s_dst[cc] * out_rows + r0 + row];
      *d = cadd(*d, v);
    } else {
      atomic_cadd(&dst[(int64_t)s_dst[cc] * out_rows + r0 + row], v);
    }
  }
  }
}

// ---------------------------------------------------------------------------
// Multipole-to-local by rotation (point-and-shoot).  With the translation
// t = |t| Q e_z, Q = R_z(phi) R_y(theta), the operator factors as
//     T(t) = Phi d T_z d^T Phi^H,
// Phi = diag(e^{-i m phi}), d the real rotation blocks of R_y(theta) (one of
// order 2n + 1 per degree n) and T_z = T(|t| e_z), which couples equal orders
// m only (one block over the degrees |m| .. p per m): about 3.3 (p+1)^3
// multiply-adds per pair instead of (p+1)^4.  A tile of up to ROT_CT pairs of
// one offset group keeps its expansions in LDS ([coefficient][pair], real and
// imaginary planes) and applies the five factors in place on the matrix
// cores: the real blocks of d act on both planes, the complex blocks of T_z
// as four real products.  Each wave owns whole blocks (degrees paired large
// with small, orders dealt in a zigzag), so within a step no wave writes what
// another reads for its own block; a block's operands sit in registers
// before it is overwritten.  The blocks are read from global memory in the
// matrix-core layout (zero-padded 64-value chunks in lane order), so a
// block product is its k steps' loads followed by its matrix instructions,
// specialised on the step count.  Rows read past a block's end hold finite
// values (other blocks', or the zeroed rows past the last one) and meet
// zero table entries.  Output: per pair, as the dense kernel's KIND 0.
// The input cut of translations across three boxes (degrees <= pf read):
// forward, the degrees above pf are loaded as zero and skipped; adjoint
// (T^H = Phi d T_z^H d^T Phi^H, cut rows), the coaxial step zeroes the
// output degrees above pf and the last rotation skips them.
// ---------------------------------------------------------------------------
constexpr int ROT_NW = 8;  // waves per tile

template <typename R>
struct RotJobDev {
  int p;
  const int* tile_group;
  const int* tile_pair0;
  const int* tile_npairs;
  const int* group_kc;  // input coefficients of the forward operator (null: all)
  const int* group_theta;
  const int* group_dist;
  const int* pair_src;
  const R* phase;
  const R* dtab;        // per rotation class: d blocks, then d^T blocks
  const cplx<R>* coax;  // adjoint: the conjugate-transposed blocks
  const cplx<R>* src;
  cplx<R>* cbuf;        // per-pair output (atomic = 0)
  cplx<R>* dst;         // atomic = 1: results added atomically into dst[pair_dst]
  const int* pair_dst;
  int atomic;
};
template <typename R>
struct RotBatch {
  int n;
  int ntiles;
  int tile0[MAX_JOBS + 1];
  RotJobDev<R> job[MAX_JOBS];
};

// Block offsets of the matrix-core tables (rot_dpoff, rot_cpoff), tabulated
// at compile time: c_rot.d[n], c_rot.c[p][m + p]
struct RotOffsets {
  int d[ROT_MAXP + 2];
  int c[ROT_MAXP + 1][2 * ROT_MAXP + 2];
};
constexpr RotOffsets make_rot_offsets() {
  RotOffsets o{};
  for (int n = 0; n <= ROT_MAXP + 1; ++n) o.d[n] = rot_dpoff(n);
  for (int p = 0; p <= ROT_MAXP; ++p)
    for (int m = -p; m <= p + 1; ++m) o.c[p][m + p] = rot_cpoff(p, m);
  return o;
}
__constant__ RotOffsets c_rot = make_rot_offsets();

__device__ __forceinline__ int isqrt_small(int c) {
  int n = (int)sqrtf((float)c);
  while (n * n > c) --n;
  while ((n + 1) * (n + 1) <= c) ++n;
  return n;
}

// One degree block (rows rb .. rb + s - 1 of both planes) times the table
// block A (matrix-core layout, NK k steps per 16-row tile; a block of NK
// steps, s in 4 NK - 3 .. 4 NK, has (NK + 3) / 4 tiles, whose table entries
// are all loaded at once).
template <typename R, int NK>
__device__ __forceinline__ void rot_deg_block(R* __restrict__ X, int PL,
                                              const R* __restrict__ A, int rb, int s, int li,
                                              int lk, int lane) {
  typedef typename MfmaOp<R>::v4 v4;
  constexpr int NMT = (NK + 3) / 4;
  R a[NMT][NK];
#pragma unroll
  for (int mt = 0; mt < NMT; ++mt)
#pragma unroll
    for (int ks = 0; ks < NK; ++ks) a[mt][ks] = A[(mt * NK + ks) * 64 + lane];
  R b0[NK], b1[NK];
#pragma unroll
  for (int ks = 0; ks < NK; ++ks) {
    const int row = rb + 4 * ks + lk;
    b0[ks] = X[row * ROT_LD + li];
    b1[ks] = X[PL + row * ROT_LD + li];
  }
#pragma unroll
  for (int mt = 0; mt < NMT; ++mt) {
    v4 c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < NK; ++ks) {
      c0 = MfmaOp<R>::mma(a[mt][ks], b0[ks], c0);
      c1 = MfmaOp<R>::mma(a[mt][ks], b1[ks], c1);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 16 * mt + MfmaOp<R>::row(lk, e);
      if (r < s) {
        X[(rb + r) * ROT_LD + li] = c0[e];
        X[PL + (rb + r) * ROT_LD + li] = c1[e];
      }
    }
  }
}

// Degrees 0 .. nmax in place, times d_n (table tb = d or d^T blocks); degree
// pairs (nmax - j, j) go to wave j % ROT_NW.  KS: k steps of the largest block.
template <typename R, int KS>
__device__ __forceinline__ void rot_degrees(R* __restrict__ X, int PL,
                                            const R* __restrict__ tb, int nmax, int wave,
                                            int li, int lk, int lane) {
  const int npair = nmax / 2 + 1;
  for (int j = wave; j < npair; j += ROT_NW) {
    for (int h = 0; h < 2; ++h) {
      const int n = h ? j : nmax - j;
      if (h && n == nmax - j) break;  // the middle degree once
      const int s = 2 * n + 1, rb = n * n;
      const R* __restrict__ A = tb + c_rot.d[n];
      switch (rot_nks(s)) {
#define ROT_DEG_CASE(K)                                            \
  case K:                                                          \
    if constexpr (K <= KS) rot_deg_block<R, K>(X, PL, A, rb, s, li, lk, lane); \
    break;
        ROT_DEG_CASE(1) ROT_DEG_CASE(2) ROT_DEG_CASE(3) ROT_DEG_CASE(4)
        ROT_DEG_CASE(5) ROT_DEG_CASE(6) ROT_DEG_CASE(7) ROT_DEG_CASE(8)
        ROT_DEG_CASE(9) ROT_DEG_CASE(10) ROT_DEG_CASE(11) ROT_DEG_CASE(12)
#undef ROT_DEG_CASE
        default: break;
      }
    }
  }
}

// One order block: rows cidx(n, m), n = am .. p, times the coaxial block T
// (matrix-core layout, nks k steps per tile, of which the first NK are read:
// the forward cut reads fewer).  Input rows past p are clamped to p (finite;
// they meet zero table entries); output degrees past kout - 1 + am are zero.
template <typename R, int NK>
__device__ __forceinline__ void rot_ord_block(R* __restrict__ X, int PL,
                                              const cplx<R>* __restrict__ T, int p, int m,
                                              int am, int s, int nks, int kout, int li, int lk,
                                              int lane) {
  typedef typename MfmaOp<R>::v4 v4;
  R yr[NK], yi[NK];
#pragma unroll
  for (int ks = 0; ks < NK; ++ks) {
    const int n = min(am + 4 * ks + lk, p), row = n * n + n + m;
    yr[ks] = X[row * ROT_LD + li];
    yi[ks] = X[PL + row * ROT_LD + li];
  }
  const int nmt = rot_nmt(s);
  for (int mt = 0; mt < nmt; ++mt) {
    cplx<R> a[NK];
#pragma unroll
    for (int ks = 0; ks < NK; ++ks) a[ks] = T[(mt * nks + ks) * 64 + lane];
    v4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < NK; ++ks) {
      cr = MfmaOp<R>::mma(a[ks].re, yr[ks], cr);
      cr = MfmaOp<R>::mma(-a[ks].im, yi[ks], cr);
      ci = MfmaOp<R>::mma(a[ks].re, yi[ks], ci);
      ci = MfmaOp<R>::mma(a[ks].im, yr[ks], ci);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 16 * mt + MfmaOp<R>::row(lk, e);
      if (r < s) {
        const int n = am + r, idx = n * n + n + m;
        const bool keep = r < kout;
        X[idx * ROT_LD + li] = keep ? cr[e] : R(0);
        X[PL + idx * ROT_LD + li] = keep ? ci[e] : R(0);
      }
    }
  }
}

// Orders m = -p .. p in place, dealt in a zigzag over the waves (order index
// i = 0, 1, 2, ... is m = 0, 1, -1, 2, ...).  Forward: the input degrees
// above pf are zero and not read; adjoint: the output degrees above pf are
// zero.  KZ: k steps of the largest block.
template <typename R, int KZ, bool ADJ>
__device__ __forceinline__ void rot_orders(R* __restrict__ X, int PL,
                                           const cplx<R>* __restrict__ cz, int p, int pf,
                                           int wave, int li, int lk, int lane) {
  for (int rnd = 0;; ++rnd) {
    const int i = rnd * ROT_NW + ((rnd & 1) ? ROT_NW - 1 - wave : wave);
    if (i > 2 * p) break;
    const int m = (i & 1) ? (i + 1) / 2 : -(i / 2);
    const int am = m < 0 ? -m : m, s = p + 1 - am;
    const int kin = ADJ ? s : min(s, pf + 1 - am);   // input degrees read
    const int kout = ADJ ? min(s, pf + 1 - am) : s;  // output degrees kept
    const cplx<R>* __restrict__ T = cz + c_rot.c[p][m + p];
    const int nks = rot_nks(s);
    switch (kin > 0 ? rot_nks(kin) : 0) {
#define ROT_ORD_CASE(K)                                                          \
  case K:                                                                        \
    if constexpr (K <= KZ) rot_ord_block<R, K>(X, PL, T, p, m, am, s, nks, kout, li, lk, lane); \
    break;
      ROT_ORD_CASE(1) ROT_ORD_CASE(2) ROT_ORD_CASE(3)
      ROT_ORD_CASE(4) ROT_ORD_CASE(5) ROT_ORD_CASE(6)
#undef ROT_ORD_CASE
      default: {  // no input degree: the block's outputs are zero
        for (int r = lane; r < s * ROT_CT; r += 64) {
          const int n = am + r / ROT_CT, cc = r % ROT_CT, idx = n * n + n + m;
          X[idx * ROT_LD + cc] = R(0);
          X[PL + idx * ROT_LD + cc] = R(0);
        }
      }
    }
  }
}

// NC: LDS rows per plane (>= (p+1)^2 of every job of the launch; 4 rows more
// hold zeros for reads past the last block).
template <typename R, int NC, bool ADJ>
__global__ void __launch_bounds__(64 * ROT_NW)
    __attribute__((amdgpu_waves_per_eu(NC <= 256 ? 4 : 2))) k_rot_m2l(const RotBatch<R> batch) {
  constexpr int NT = 64 * ROT_NW;
  constexpr int NR = NC + 4;
  constexpr int PL = NR * ROT_LD;
  constexpr int PM = NC <= 256 ? 15 : ROT_MAXP;  // largest order of the class
  constexpr int KS = rot_nks(2 * PM + 1);
  constexpr int KZ = rot_nks(PM + 1);
  constexpr int CSTR = NC <= 256 ? 256 : 512;  // coefficients per pass
  constexpr int CCS = NT / CSTR;               // pairs per pass
  __shared__ __attribute__((aligned(16))) R X[2 * PL];
  __shared__ R s_ph[2][2 * ROT_MAXP + 1];
  __shared__ int s_src[ROT_CT], s_dst[ROT_CT];
  __builtin_amdgcn_s_setprio(2);  // critical path: ahead of the near-field waves
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  for (int t = tid; t < 2 * PL; t += NT) X[t] = R(0);
  const int nt = batch.ntiles;
  for (int vb = blockIdx.x; vb < nt; vb += gridDim.x) {
    __syncthreads();  // the previous tile no longer reads the shared arrays
    // XCD-aware order, as for the dense kernel
    const int xcd = vb & 7, slot_in_xcd = vb >> 3;
    const int gtile = xcd * (nt >> 3) + min(xcd, nt & 7) + slot_in_xcd;
    int q = 0;
#pragma unroll
    for (int i = 1; i < MAX_JOBS; ++i)
      if (i < batch.n && gtile >= batch.tile0[i]) q = i;
    const RotJobDev<R> J = select_job(batch.job, q);
    const int tile = gtile - select_job(batch.tile0, q);
    const int p = J.p, nc = (p + 1) * (p + 1);
    const int grp = J.tile_group[tile], p0 = J.tile_pair0[tile], np = J.tile_npairs[tile];
    const int kc = J.group_kc ? min(nc, J.group_kc[grp]) : nc;
    int pf = 0;
    while ((pf + 2) * (pf + 2) <= kc) ++pf;
    const int th = J.group_theta[grp], di = J.group_dist[grp];
    if (tid < ROT_CT) {
      s_src[tid] = tid < np ? J.pair_src[p0 + tid] : -1;
      s_dst[tid] = (J.atomic && tid < np) ? J.pair_dst[p0 + tid] : -1;
    }
    if (tid < 2 * p + 1) {  // e^{i m phi}, m = -p .. p
      const int m = tid - p, am = m < 0 ? -m : m;
      const R* ph = J.phase + ((int64_t)grp * (p + 1) + am) * 2;
      s_ph[0][tid] = ph[0];
      s_ph[1][tid] = m < 0 ? -ph[1] : ph[1];
    }
    __syncthreads();
    // Phi^H: coefficient (n, m) times e^{i m phi} (forward: the kc
    // coefficients the cut keeps, the rest zero)
    const int kin = ADJ ? nc : kc;
    for (int c = tid % CSTR; c < nc; c += CSTR) {
      const int n = isqrt_small(c), m = c - n * n - n;
      const R er = s_ph[0][m + p], ei = s_ph[1][m + p];
      cplx<R> v[ROT_CT / CCS];
#pragma unroll
      for (int i = 0; i < ROT_CT / CCS; ++i) {
        const int cc = tid / CSTR + CCS * i;
        v[i] = (cc < np && c < kin) ? J.src[(int64_t)s_src[cc] * nc + c] : mk<R>(0, 0);
      }
#pragma unroll
      for (int i = 0; i < ROT_CT / CCS; ++i) {
        const int cc = tid / CSTR + CCS * i;
        X[c * ROT_LD + cc] = v[i].re * er - v[i].im * ei;
        X[PL + c * ROT_LD + cc] = v[i].re * ei + v[i].im * er;
      }
    }
    __syncthreads();
    const int dpsz = c_rot.d[p + 1], cpsz = c_rot.c[p][2 * p + 1];
    const R* __restrict__ dt = J.dtab + (int64_t)th * 2 * dpsz;
    const cplx<R>* __restrict__ cz = J.coax + (int64_t)di * cpsz;
    rot_degrees<R, KS>(X, PL, dt + dpsz, ADJ ? p : pf, wave, li, lk, lane);  // d^T
    __syncthreads();
    rot_orders<R, KZ, ADJ>(X, PL, cz, p, pf, wave, li, lk, lane);  // T_z (or T_z^H)
    __syncthreads();
    rot_degrees<R, KS>(X, PL, dt, ADJ ? pf : p, wave, li, lk, lane);  // d
    __syncthreads();
    // Phi: coefficient (n, m) times e^{-i m phi}, written per pair (or added
    // atomically into the destination's expansion)
    for (int c = tid % CSTR; c < nc; c += CSTR) {
      const int n = isqrt_small(c), m = c - n * n - n;
      const R er = s_ph[0][m + p], ei = s_ph[1][m + p];
#pragma unroll
      for (int i = 0; i < ROT_CT / CCS; ++i) {
        const int cc = tid / CSTR + CCS * i;
        if (cc < np) {
          const R xr = X[c * ROT_LD + cc], xi = X[PL + c * ROT_LD + cc];
          const cplx<R> v = mk<R>(xr * er + xi * ei, xi * er - xr * ei);
          if (J.atomic)
            atomic_cadd(&J.dst[(int64_t)s_dst[cc] * nc + c], v);
          else
            J.cbuf[(int64_t)(p0 + cc) * nc + c] = v;
        }
      }
    }
  }
}

// dst[b][c] (+)= sum over the pairs t of box b of cbuf[t][c]  (pairs listed
// per box in a fixed order: deterministic, no atomics)
// 256 threads per box: 4 slices of 64 coefficients, each slice sums every
// fourth pair, then the slices are added in a fixed order.
template <typename R>
struct RedJobDev {
  int ncoef;
  const int* ptr;
  const int* pairs;
  const cplx<R>* cbuf;
  cplx<R>* dst;
};
template <typename R>
struct RedBatch {
  int n;
  int box0[MAX_JOBS + 1];
  RedJobDev<R> job[MAX_JOBS];
};

// Sum over t = t0 + slice, t0 + slice + 4, ... < t1 of cbuf[pairs[t] * ncoef + c],
// added in ascending t.  Eight rows are loaded per step (out-of-range ones as
// zero, which leaves the sum unchanged) so that their latencies overlap.
template <typename R>
__device__ __forceinline__ cplx<R> slice_sum(const int* __restrict__ pairs,
                                             const cplx<R>* __restrict__ cbuf, int ncoef, int c,
                                             int t0, int t1, int slice) {
  constexpr int U = 8;
  cplx<R> acc = mk<R>(0, 0);
  for (int t = t0 + slice; t < t1; t += 4 * U) {
    int p[U];
#pragma unroll
    for (int u = 0; u < U; ++u) p[u] = t + 4 * u < t1 ? pairs[t + 4 * u] : -1;
    cplx<R> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      v[u] = p[u] >= 0 ? cbuf[(int64_t)p[u] * ncoef + c] : mk<R>(0, 0);
#pragma unroll
    for (int u = 0; u < U; ++u) acc = cadd(acc, v[u]);
  }
  return acc;
}

template <typename R>
__global__ void __launch_bounds__(256)
    k_pair_reduce(const RedBatch<R> batch, int accumulate) {
  __builtin_amdgcn_s_setprio(2);  // critical path: ahead of the near-field waves
  __shared__ cplx<R> part[4][64];
  int q = 0;
#pragma unroll
  for (int i = 1; i < MAX_JOBS; ++i)
    if (i < batch.n && (int)blockIdx.x >= batch.box0[i]) q = i;
  const RedJobDev<R> J = select_job(batch.job, q);
  const int b = blockIdx.x - select_job(batch.box0, q);
  const int ncoef = J.ncoef;
  const int t0 = J.ptr[b], t1 = J.ptr[b + 1];
  const int lane = threadIdx.x & 63, slice = threadIdx.x >> 6;
  for (int c0 = 0; c0 < ncoef; c0 += 64) {
    const int c = c0 + lane;
    const cplx<R> acc =
        c < ncoef ? slice_sum<R>(J.pairs, J.cbuf, ncoef, c, t0, t1, slice) : mk<R>(0, 0);
    part[slice][lane] = acc;
    __syncthreads();
    if (slice == 0 && c < ncoef) {
      cplx<R> s = accumulate ? J.dst[(int64_t)b * ncoef + c] : mk<R>(0, 0);
      s = cadd(s, cadd(cadd(part[0][lane], part[1][lane]), cadd(part[2][lane], part[3][lane])));
      J.dst[(int64_t)b * ncoef + c] = s;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// finish: 16 lanes per element (4 elements per wavefront).  Lane l handles
// local-expansion coefficients l, l + 16, ... and near-list entries l,
// l + 16, ...; the 16 partial sums are combined by shuffles in a fixed order.
// ---------------------------------------------------------------------------
constexpr int FIN_LANES = 16;

template <typename R>
__device__ __forceinline__ R group_sum16(R v) {
  for (int off = FIN_LANES / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, FIN_LANES);
  return v;
}

// y[perm[i]] for element i (sorted order), lane l of its 16-lane group: far
// field (L2P rows against the leaf's local expansion: Lc[elem_leaf[i]], or
// Lc itself when elem_leaf is null), near corrections when near_ptr is
// non-null (the products pass null: their P2P kernels apply them), the P2P
// sum ys and the float64 diagonal.  Every lane of a group calls it.
template <typename R>
__device__ __forceinline__ void finish_elem(
    int64_t i, int l, int64_t n, const int* __restrict__ perm, const int* __restrict__ elem_leaf,
    int ncoef, const cplx<R>* __restrict__ l2p, const cplx<R>* __restrict__ Lc,
    const int* __restrict__ near_ptr, const int* __restrict__ near_col,
    const cplx<R>* __restrict__ ncp, const cplx<R>* __restrict__ ncq,
    const cplx<R>* __restrict__ ps, const cplx<R>* __restrict__ qs,
    const cplx<R>* __restrict__ ys, const c64* __restrict__ dp, const c64* __restrict__ dq,
    const c64* __restrict__ p64, const c64* __restrict__ q64, c64* __restrict__ y) {
  cplx<R> acc = mk<R>(0, 0);
  if (i < n) {  // whole 16-lane groups are in or out: the shuffles stay inside a group
    if (ncoef > 0) {
      const cplx<R>* Bi = l2p + i * ncoef;
      const cplx<R>* Lb = elem_leaf ? Lc + (int64_t)elem_leaf[i] * ncoef : Lc;
      // four coefficients per lane per step, loads issued together (terms
      // past ncoef are zero, so the sum and its order are unchanged)
      for (int c0 = l; c0 < ncoef; c0 += 4 * FIN_LANES) {
        cplx<R> bv[4], lv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = c0 + u * FIN_LANES;
          bv[u] = c < ncoef ? Bi[c] : mk<R>(0, 0);
          lv[u] = c < ncoef ? Lb[c] : mk<R>(0, 0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) cfma(acc, bv[u], lv[u]);
      }
    }
    if (near_ptr)
      for (int t = near_ptr[i] + l; t < near_ptr[i + 1]; t += FIN_LANES) {
        const int j = near_col[t];
        cfma(acc, ncp[t], ps[j]);
        cfma(acc, ncq[t], qs[j]);
      }
  }
  acc.re = group_sum16(acc.re);
  acc.im = group_sum16(acc.im);
  if (i < n && l == 0) {
    cplx<R> s = cadd(acc, ys[i]);
    c64 out = mk((double)s.re, (double)s.im);
    cfma(out, dp[i], p64[i]);
    cfma(out, dq[i], q64[i]);
    y[perm[i]] = out;
  }
}

template <typename R>
__global__ void __launch_bounds__(256)
    k_finish(int64_t n, const int* __restrict__ perm, const int* __restrict__ elem_leaf,
             int ncoef, const cplx<R>* __restrict__ l2p, const cplx<R>* __restrict__ Lc,
             const int* __restrict__ near_ptr, const int* __restrict__ near_col,
             const cplx<R>* __restrict__ ncp, const cplx<R>* __restrict__ ncq,
             const cplx<R>* __restrict__ ps, const cplx<R>* __restrict__ qs,
             const cplx<R>* __restrict__ ys, const c64* __restrict__ dp,
             const c64* __restrict__ dq, const c64* __restrict__ p64,
             const c64* __restrict__ q64, c64* __restrict__ y) {
  finish_elem<R>(grid_tid() / FIN_LANES, threadIdx.x % FIN_LANES, n, perm, elem_leaf, ncoef, l2p,
                 Lc, near_ptr, near_col, ncp, ncq, ps, qs, ys, dp, dq, p64, q64, y);
}

// u[perm[j]], w[perm[j]] of the adjoint for source element j (sorted
// order): transposed P2M rows (against Mc[elem_leaf[j]], or Mc itself when
// elem_leaf is null), transposed near corrections when tptr is non-null (the
// products pass null: their P2P kernels apply them), the adjoint P2P sums and
// the conjugated diagonal.  Every lane of a group calls it.
// WZ: w not wanted; p2m then holds the p columns alone (n x ncoef)
template <typename R, bool WZ = false>
__device__ __forceinline__ void finish_adj_elem(
    int64_t j, int l, int64_t n, const int* __restrict__ perm, const int* __restrict__ elem_leaf,
    int ncoef, const cplx<R>* __restrict__ p2m, const cplx<R>* __restrict__ Mc,
    const int* __restrict__ tptr, const int* __restrict__ trow, const cplx<R>* __restrict__ tcp,
    const cplx<R>* __restrict__ tcq, const cplx<R>* __restrict__ ysrt,
    const cplx<R>* __restrict__ us, const cplx<R>* __restrict__ ws, const c64* __restrict__ dp,
    const c64* __restrict__ dq, const c64* __restrict__ y64, c64* __restrict__ u,
    c64* __restrict__ w) {
  cplx<R> au = mk<R>(0, 0), aw = mk<R>(0, 0);
  if (j < n) {
    if (ncoef > 0) {
      const cplx<R>* Aj = p2m + j * ncoef * (WZ ? 1 : 2);
      const cplx<R>* Mb = elem_leaf ? Mc + (int64_t)elem_leaf[j] * ncoef : Mc;
      // four coefficients per lane per step, loads issued together
      for (int c0 = l; c0 < ncoef; c0 += 4 * FIN_LANES) {
        cplx<R> ap[4], aq[4], mv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = c0 + u * FIN_LANES;
          if (c < ncoef) {
            if (WZ)
              ap[u] = Aj[c];
            else
              load_pair(Aj + 2 * c, ap[u], aq[u]);
            mv[u] = Mb[c];
          } else {
            ap[u] = aq[u] = mv[u] = mk<R>(0, 0);
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          cfmac(au, ap[u], mv[u]);
          if (!WZ) cfmac(aw, aq[u], mv[u]);
        }
      }
    }
    if (tptr)
      for (int t = tptr[j] + l; t < tptr[j + 1]; t += FIN_LANES) {
        cplx<R> yv = ysrt[trow[t]];
        cfmac(au, tcp[t], yv);
        if (!WZ) cfmac(aw, tcq[t], yv);
      }
  }
  au.re = group_sum16(au.re);
  au.im = group_sum16(au.im);
  if (!WZ) {
    aw.re = group_sum16(aw.re);
    aw.im = group_sum16(aw.im);
  }
  if (j < n && l == 0) {
    cplx<R> su = cadd(au, us[j]);
    c64 ou = mk((double)su.re, (double)su.im);
    cfmac(ou, dp[j], y64[j]);
    int o = perm[j];
    if (u) u[o] = ou;
    if (!WZ && w) {
      cplx<R> sw = cadd(aw, ws[j]);
      c64 ow = mk((double)sw.re, (double)sw.im);
      cfmac(ow, dq[j], y64[j]);
      w[o] = ow;
    }
  }
}

template <typename R>
__global__ void __launch_bounds__(256)
    k_finish_adj(int64_t n, const int* __restrict__ perm, const int* __restrict__ elem_leaf,
                 int ncoef, const cplx<R>* __restrict__ p2m, const cplx<R>* __restrict__ Mc,
                 const int* __restrict__ tptr, const int* __restrict__ trow,
                 const cplx<R>* __restrict__ tcp, const cplx<R>* __restrict__ tcq,
                 const cplx<R>* __restrict__ ysrt, const cplx<R>* __restrict__ us,
                 const cplx<R>* __restrict__ ws, const c64* __restrict__ dp,
                 const c64* __restrict__ dq, const c64* __restrict__ y64, c64* __restrict__ u,
                 c64* __restrict__ w) {
  finish_adj_elem<R>(grid_tid() / FIN_LANES, threadIdx.x % FIN_LANES, n, perm, elem_leaf, ncoef,
                     p2m, Mc, tptr, trow, tcp, tcq, ysrt, us, ws, dp, dq, y64, u, w);
}

// ---------------------------------------------------------------------------
// Leaf finish: one leaf box per block.  The leaf-level M2L reduction is
// folded into the finish: the box's expansion = its part translated from
// the level above (base, accumulated there onto a cleared buffer) + the sum
// of its per-pair M2L results, formed in LDS (same order as k_pair_reduce,
// so the values equal those of the separate reduction); then every element
// of the leaf as in k_finish / k_finish_adj.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void leaf_expansion(int b, int ncoef, const int* __restrict__ ptr,
                                               const int* __restrict__ pairs,
                                               const cplx<R>* __restrict__ cbuf,
                                               const cplx<R>* __restrict__ base, cplx<R>* out) {
  __shared__ cplx<R> part[4][64];
  const int t0 = ptr[b], t1 = ptr[b + 1];
  const int lane = threadIdx.x & 63, slice = threadIdx.x >> 6;
  for (int c0 = 0; c0 < ncoef; c0 += 64) {
    const int c = c0 + lane;
    const cplx<R> acc =
        c < ncoef ? slice_sum<R>(pairs, cbuf, ncoef, c, t0, t1, slice) : mk<R>(0, 0);
    part[slice][lane] = acc;
    __syncthreads();
    if (slice == 0 && c < ncoef)
      out[c] = cadd(base[(int64_t)b * ncoef + c],
                    cadd(cadd(part[0][lane], part[1][lane]), cadd(part[2][lane], part[3][lane])));
    __syncthreads();
  }
}

// forward: y for the elements of leaf b (L2P against the leaf's locals)
template <typename R>
__global__ void __launch_bounds__(256)
    k_leaf_finish(const int* __restrict__ bstart, int ncoef, const int* __restrict__ red_ptr,
                  const int* __restrict__ red_pairs, const cplx<R>* __restrict__ cbuf,
                  const cplx<R>* __restrict__ Lc, int64_t n, const int* __restrict__ perm,
                  const cplx<R>* __restrict__ l2p, const int* __restrict__ near_ptr,
                  const int* __restrict__ near_col, const cplx<R>* __restrict__ ncp,
                  const cplx<R>* __restrict__ ncq, const cplx<R>* __restrict__ ps,
                  const cplx<R>* __restrict__ qs, const cplx<R>* __restrict__ ys,
                  const c64* __restrict__ dp, const c64* __restrict__ dq,
                  const c64* __restrict__ p64, const c64* __restrict__ q64,
                  c64* __restrict__ y) {
  __builtin_amdgcn_s_setprio(2);  // critical path: ahead of the near-field waves
  cplx<R>* Lf = reinterpret_cast<cplx<R>*>(leaf_lds);
  const int b = blockIdx.x;
  leaf_expansion<R>(b, ncoef, red_ptr, red_pairs, cbuf, Lc, Lf);
  const int e0 = bstart[b], ne = bstart[b + 1] - e0;
  const int g = threadIdx.x / FIN_LANES, l = threadIdx.x % FIN_LANES;
  for (int e = 0; e < ne; e += 256 / FIN_LANES) {
    const int64_t i = e + g < ne ? e0 + e + g : n;  // n: group idle this pass
    finish_elem<R>(i, l, n, perm, nullptr, ncoef, l2p, Lf, near_ptr, near_col, ncp, ncq, ps, qs,
                   ys, dp, dq, p64, q64, y);
  }
}

// adjoint: u, w for the elements of leaf b (P2M^H against the leaf's
// adjoint multipoles; WZ: u alone, p2m = the p columns)
template <typename R, bool WZ>
__global__ void __launch_bounds__(256)
    k_leaf_finish_adj(const int* __restrict__ bstart, int ncoef, const int* __restrict__ red_ptr,
                      const int* __restrict__ red_pairs, const cplx<R>* __restrict__ cbuf,
                      const cplx<R>* __restrict__ Mc, int64_t n, const int* __restrict__ perm,
                      const cplx<R>* __restrict__ p2m, const int* __restrict__ tptr,
                      const int* __restrict__ trow, const cplx<R>* __restrict__ tcp,
                      const cplx<R>* __restrict__ tcq, const cplx<R>* __restrict__ ysrt,
                      const cplx<R>* __restrict__ us, const cplx<R>* __restrict__ ws,
                      const c64* __restrict__ dp, const c64* __restrict__ dq,
                      const c64* __restrict__ y64, c64* __restrict__ u, c64* __restrict__ w) {
  __builtin_amdgcn_s_setprio(2);  // critical path: ahead of the near-field waves
  cplx<R>* Mf = reinterpret_cast<cplx<R>*>(leaf_lds);
  const int b = blockIdx.x;
  leaf_expansion<R>(b, ncoef, red_ptr, red_pairs, cbuf, Mc, Mf);
  const int e0 = bstart[b], ne = bstart[b + 1] - e0;
  const int g = threadIdx.x / FIN_LANES, l = threadIdx.x % FIN_LANES;
  for (int e = 0; e < ne; e += 256 / FIN_LANES) {
    const int64_t j = e + g < ne ? e0 + e + g : n;
    finish_adj_elem<R, WZ>(j, l, n, perm, nullptr, ncoef, p2m, Mf, tptr, trow, tcp, tcq, ysrt,
                           us, ws, dp, dq, y64, u, w);
  }
}

// ---------------------------------------------------------------------------
// Gather and finish of several products in one launch each (batched
// product).  Job q owns blocks blk0[q] .. blk0[q + 1) - 1.
// ---------------------------------------------------------------------------
constexpr int BATCH_ZERO = 8;  // cleared levels per job in a batched gather

template <typename R>
struct GatherJobDev {
  const c64* p;  // forward: p (user order) | adjoint: y
  const c64* q;  // forward only, may be null
  const int* perm;
  int64_t n;
  cplx<R>* ps;
  cplx<R>* qs;
  c64* p64;
  c64* q64;
  ZeroList<R, BATCH_ZERO> zl;
};

template <typename R>
struct GatherBatch {
  int n;
  int blk0[MAX_JOBS + 1];
  GatherJobDev<R> job[MAX_JOBS];
};

template <typename R, bool ADJ>
__global__ void __launch_bounds__(256) k_gather_batch(const GatherBatch<R> batch) {
  const int qj = job_of(batch.blk0, batch.n, (int)blockIdx.x);
  const GatherJobDev<R> J = select_job(batch.job, qj);
  const int b0 = select_job(batch.blk0, qj), b1 = select_job(batch.blk0, qj + 1);
  const int64_t i = (int64_t)((int)blockIdx.x - b0) * blockDim.x + threadIdx.x;
  zero_list(J.zl, i, (int64_t)(b1 - b0) * blockDim.x);
  if (i >= J.n) return;
  const int o = J.perm[i];
  const c64 a = J.p ? J.p[o] : mk(0.0, 0.0);
  J.ps[i] = mk<R>((R)a.re, (R)a.im);
  J.p64[i] = a;
  if (!ADJ) {
    const c64 c = J.q ? J.q[o] : mk(0.0, 0.0);
    J.qs[i] = mk<R>((R)c.re, (R)c.im);
    J.q64[i] = c;
  }
}

// forward: ex = L2P rows, Mx = leaf locals, near CSR by target, a/b = sorted
// p/q, c = P2P sums, p64/q64 = float64 sorted p/q, out = y.
// adjoint: ex = P2M rows, Mx = leaf multipoles, near CSC by source, a =
// sorted y, b/c = P2P sums (u, w), p64 = float64 sorted y, out/out2 = u/w.
template <typename R>
struct FinJobDev {
  int64_t n;
  const int* perm;
  const int* elem_leaf;
  int ncoef;
  const cplx<R>* ex;
  const cplx<R>* Mx;
  const int* nptr;
  const int* nidx;
  const cplx<R>* ncp;
  const cplx<R>* ncq;
  const cplx<R>* a;
  const cplx<R>* b;
  const cplx<R>* c;
  const c64* dp;
  const c64* dq;
  const c64* p64;
  const c64* q64;
  c64* out;
  c64* out2;
};

template <typename R>
struct FinBatch {
  int n;
  int blk0[MAX_JOBS + 1];
  FinJobDev<R> job[MAX_JOBS];
};

// WZ (adjoint): no job wants w; ex holds the p columns of P2M alone
template <typename R, bool ADJ, bool WZ = false>
__global__ void __launch_bounds__(256) k_finish_batch(const FinBatch<R> batch) {
  const int qj = job_of(batch.blk0, batch.n, (int)blockIdx.x);
  const FinJobDev<R> J = select_job(batch.job, qj);
  const int64_t t = (int64_t)((int)blockIdx.x - select_job(batch.blk0, qj)) * blockDim.x +
                    threadIdx.x;
  const int l = threadIdx.x % FIN_LANES;
  if (ADJ)
    finish_adj_elem<R, WZ>(t / FIN_LANES, l, J.n, J.perm, J.elem_leaf, J.ncoef, J.ex, J.Mx,
                           J.nptr, J.nidx, J.ncp, J.ncq, J.a, J.b, J.c, J.dp, J.dq, J.p64, J.out,
                           J.out2);
  else
    finish_elem<R>(t / FIN_LANES, l, J.n, J.perm, J.elem_leaf, J.ncoef, J.ex, J.Mx, J.nptr,
                   J.nidx, J.ncp, J.ncq, J.a, J.b, J.c, J.dp, J.dq, J.p64, J.q64, J.out);
}

// ---------------------------------------------------------------------------
// stage profiling: pairs of events recorded on the stream; read by the C ABI
// ---------------------------------------------------------------------------
int prof_begin(Problem& P, hipStream_t s) {
  if (!P.prof_on) return -1;
  if ((int)P.ev_pool.size() < 2 * (P.ev_used + 1)) {
    for (int t = 0; t < 64; ++t) {
      hipEvent_t e;
      BEM_HIP_TRY(hipEventCreate(&e));
      P.ev_pool.push_back(e);
    }
  }
  int idx = P.ev_used++;
  BEM_HIP_TRY(hipEventRecord(P.ev_pool[2 * idx], s));
  return idx;
}

int prof_end(Problem& P, int idx, int slot, hipStream_t s) {
  if (idx < 0) return 0;
  BEM_HIP_TRY(hipEventRecord(P.ev_pool[2 * idx + 1], s));
  if ((int)P.ev_slot.size() <= idx) P.ev_slot.resize(idx + 1);
  P.ev_slot[idx] = slot;
  return 0;
}

// a (start, end) event pair for a launch's own events, counted in `slot`
int prof_pair(Problem& P, int slot) {
  if ((int)P.ev_pool.size() < 2 * (P.ev_used + 1)) {
    for (int t = 0; t < 64; ++t) {
      hipEvent_t e;
      BEM_HIP_TRY(hipEventCreate(&e));
      P.ev_pool.push_back(e);
    }
  }
  int idx = P.ev_used++;
  if ((int)P.ev_slot.size() <= idx) P.ev_slot.resize(idx + 1);
  P.ev_slot[idx] = slot;
  return idx;
}

// the leaf-level M2L's launch events: a timing pair when the leaf M2L alone is
// profiled, else none
template <typename R>
static void leaf_m2l_events(Problem& P, bool adj, hipEvent_t* start, hipEvent_t* done) {
  *start = nullptr;
  *done = nullptr;
  if (!P.prof_leaf) return;
  const int idx = prof_pair(P, prof_slot(ST_M2L_LEAF, sizeof(R) == 4, adj));
  if (idx < 0) return;
  *start = P.ev_pool[2 * idx];
  *done = P.ev_pool[2 * idx + 1];
}

#define PROF_BEGIN(var) int var = prof_begin(P, s)
#define PROF_END(var, stage)                                                  \
  do {                                                                        \
    int _pr = prof_end(P, var, prof_slot(stage, sizeof(R) == 4, ADJ_FLAG), s); \
    if (_pr) return _pr;                                                      \
  } while (0)

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------
// KIND: 0 M2L (per-pair output into cbuf, then reduced per destination box,
// replacing dst (accumulate = 0) or adding to it), 1 M2M, 2 L2L (added into
// dst).  One launch covers up to MAX_JOBS grouped products with the same
// pair-tile width (chosen at plan time; it selects the instantiation).
template <typename R>
struct GemmJob {
  const GroupedOp<R>* op;
  const cplx<R>* src;
  cplx<R>* dst;
  cplx<R>* cbuf;  // M2L: this job's per-pair output
};

template <typename R, int CT, bool ADJ, int KIND>
static void launch_gemm(const GemmBatch<R>& b, int nt, hipStream_t s, hipEvent_t start,
                        hipEvent_t done) {
  launch_done(k_grouped_gemm<R, CT, ADJ, KIND>, dim3(nt), dim3(64 * TileShape<CT>::NW), 0, s,
              start, done, b);
}

// grid: workgroups (0: one per tile), a multiple of 8 or all tiles
template <typename R, bool ADJ>
static int launch_rot(const RotBatch<R>& b, int maxnc, int grid, hipStream_t s, hipEvent_t done,
                      hipEvent_t start) {
  constexpr int NC_HI = (ROT_MAXP + 1) * (ROT_MAXP + 1);
  const int nt = b.ntiles;
  const int g = (grid > 0 && grid < nt) ? std::max(8, grid & ~7) : nt;
  if (maxnc <= 256)
    launch_done(k_rot_m2l<R, 256, ADJ>, dim3(g), dim3(64 * ROT_NW), 0, s, start, done, b);
  else if (maxnc <= NC_HI)
    launch_done(k_rot_m2l<R, NC_HI, ADJ>, dim3(g), dim3(64 * ROT_NW), 0, s, start, done, b);
  else {
    set_error("expansion order too high for the rotation-based translations");
    return -1;
  }
  BEM_LAUNCH_CHECK();
  return 0;
}

// launch-grouping key of an M2L product: its pair-tile width, or 1 for the
// rotation-based kernel
template <typename R>
static int tile_key(const GroupedOp<R>& op, bool adj) {
  return op.rot_on ? 1 : (adj ? op.ct_adj : op.ct);
}

template <typename R, bool ADJ, int KIND>
static int launch_gemm_ct(const GemmBatch<R>& b, int ct, int nt, hipStream_t s,
                          hipEvent_t done = nullptr, hipEvent_t start = nullptr) {
  switch (ct) {
    case 16: launch_gemm<R, 16, ADJ, KIND>(b, nt, s, start, done); break;
    case 32: launch_gemm<R, 32, ADJ, KIND>(b, nt, s, start, done); break;
    case 64: launch_gemm<R, 64, ADJ, KIND>(b, nt, s, start, done); break;
    case 128:
      if constexpr (sizeof(R) == 4) {
        launch_gemm<R, 128, ADJ, KIND>(b, nt, s, start, done);
        break;
      } else {
        set_error("128-pair tiles are float32 only");
        return -1;
      }
    default: set_error("bad pair-tile width"); return -1;
  }
  BEM_LAUNCH_CHECK();
  return 0;
}

template <typename R, int KIND>
static int launch_grouped_jobs(const GemmJob<R>* jobs, int nj, bool adj, hipStream_t s,
                               int accumulate = 0, Problem* prof = nullptr,
                               int st_gemm = ST_M2L, int grid_cap = 0,
                               bool run_reduce = true, hipEvent_t done = nullptr,
                               hipEvent_t start = nullptr) {
  // `done`: signalled by the GEMM launch (only with run_reduce = false);
  // `start`: timing event attached to the GEMM launch
  if (done && run_reduce) {
    set_error("completion event of a grouped product with its reduction");
    return -1;
  }
  if (nj <= 0) {
    if (done) BEM_HIP_TRY(hipEventRecord(done, s));
    return 0;
  }
  if (nj > MAX_JOBS) {
    set_error("too many grouped products in one launch");
    return -1;
  }
  GemmBatch<R> b{};
  RedBatch<R> rb{};
  RotBatch<R> tb{};
  b.n = rb.n = tb.n = nj;
  int nt = 0, nbox = 0, ct = 0, maxnc = 0;
  // rotation-based M2L (every job of the launch or none): per-pair outputs
  // (KIND 0) or added atomically (KIND 1, the float64 translations into
  // point boxes; forward only)
  const bool rot = (KIND == 0 || KIND == 1) && jobs[0].op->rot_on;
  if (rot && KIND == 1 && adj) {
    set_error("atomic rotation-based translations are forward only");
    return -1;
  }
  // adjoint M2L: the stored conjugate transposes through the forward
  // operand path (the transposed load path is slower)
  bool via_fwd = adj && KIND == 0;
  for (int q = 0; q < nj; ++q) via_fwd = via_fwd && jobs[q].op->mats_h;
  for (int q = 0; q < nj; ++q) {
    const GroupedOp<R>& op = *jobs[q].op;
    if (KIND == 0 && !jobs[q].cbuf) {
      set_error("multipole-to-local product without its per-pair buffer");
      return -1;
    }
    const int jct = adj ? op.ct_adj : op.ct;
    if (q > 0 && jct != ct && !rot) {
      set_error("grouped products of one launch differ in tile width");
      return -1;
    }
    ct = jct;
    if (op.rot_on != rot || (rot && (!op.rot_ready || op.rot_p > ROT_MAXP ||
                                     (op.rot_p + 1) * (op.rot_p + 1) != op.rows))) {
      set_error("rotation-based and dense translations in one launch, or rotation tables missing");
      return -1;
    }
    if (rot) {
      RotJobDev<R>& T = tb.job[q];
      T.p = op.rot_p;
      T.tile_group = op.rot_tile_group;
      T.tile_pair0 = op.rot_tile_pair0;
      T.tile_npairs = op.rot_tile_npairs;
      T.group_kc = op.group_kc;
      T.group_theta = op.rot_theta;
      T.group_dist = op.rot_dist;
      T.pair_src = adj ? op.pair_src_adj : op.pair_src;
      T.phase = op.rot_phase;
      T.dtab = op.rot_dtab;
      T.coax = adj ? op.rot_coax_h : op.rot_coax;
      T.src = jobs[q].src;
      T.cbuf = jobs[q].cbuf;
      T.dst = jobs[q].dst;
      T.pair_dst = op.pair_dst;
      T.atomic = KIND == 1 ? 1 : 0;
      tb.tile0[q] = nt;
      nt += op.rot_n_tiles;
      maxnc = std::max(maxnc, op.rows);
    }
    GemmJobDev<R>& J = b.job[q];
    J.mat_rows = via_fwd ? op.cols : op.rows;
    J.mat_cols = via_fwd ? op.rows : op.cols;
    J.tile_group = adj ? op.tile_group_adj : op.tile_group;
    J.tile_pair0 = adj ? op.tile_pair0_adj : op.tile_pair0;
    J.tile_npairs = adj ? op.tile_npairs_adj : op.tile_npairs;
    J.tile_row0 = adj ? op.tile_row0_adj : op.tile_row0;
    J.group_slot = op.group_slot;
    J.group_kc = adj ? nullptr : op.group_kc;
    J.pair_dst = adj ? op.pair_dst_adj : op.pair_dst;
    J.pair_src = adj ? op.pair_src_adj : op.pair_src;
    J.mats = via_fwd ? op.mats_h : op.mats;
    J.src = jobs[q].src;
    J.dst = jobs[q].dst;
    J.cbuf = jobs[q].cbuf;
    if (!rot) {
      b.tile0[q] = nt;
      nt += adj ? op.n_tiles_adj : op.n_tiles;
    }
    RedJobDev<R>& RJ = rb.job[q];
    RJ.ncoef = adj ? op.cols : op.rows;
    RJ.ptr = adj ? op.red_ptr_adj : op.red_ptr;
    RJ.pairs = adj ? op.red_pairs_adj : op.red_pairs;
    RJ.cbuf = jobs[q].cbuf;
    RJ.dst = jobs[q].dst;
    rb.box0[q] = nbox;
    nbox += adj ? op.n_red_adj : op.n_red;
  }
  b.tile0[nj] = tb.tile0[nj] = nt;
  b.ntiles = tb.ntiles = nt;
  rb.box0[nj] = nbox;
  if (nt == 0 && start) BEM_HIP_TRY(hipEventRecord(start, s));
  if (nt == 0 && done) BEM_HIP_TRY(hipEventRecord(done, s));
  if (nt > 0) {
    int evg = prof ? prof_begin(*prof, s) : -1;
    const int grid = (grid_cap > 0 && grid_cap < nt) ? (grid_cap & ~7) : nt;
    const int g = grid > 0 ? grid : nt;
    int r = rot ? (adj ? launch_rot<R, true>(tb, maxnc, grid, s, done, start)
                       : launch_rot<R, false>(tb, maxnc, grid, s, done, start))
            : (adj && !via_fwd) ? launch_gemm_ct<R, true, KIND>(b, ct, g, s, done, start)
                                : launch_gemm_ct<R, false, KIND>(b, ct, g, s, done, start);
    if (r) return r;
    if (prof) {
      int pr = prof_end(*prof, evg, prof_slot(st_gemm, sizeof(R) == 4, adj), s);
      if (pr) return pr;
    }
  }
  // the reduction also runs with no tiles: it then clears the destinations
  if (KIND == 0 && nbox > 0 && run_reduce) {
    int ev = prof ? prof_begin(*prof, s) : -1;
    hipLaunchKernelGGL(k_pair_reduce<R>, dim3(nbox), dim3(256), 0, s, rb, accumulate);
    BEM_LAUNCH_CHECK();
    if (prof) {
      const int st_red = st_gemm == ST_M2L_LEAF ? ST_M2L_LEAF_RED : ST_M2L_RED;
      int pr = prof_end(*prof, ev, prof_slot(st_red, sizeof(R) == 4, adj), s);
      if (pr) return pr;
    }
  }
  return 0;
}

template <typename R, int KIND>
static int launch_grouped(const GroupedOp<R>& op, bool adj, const cplx<R>* src, cplx<R>* dst,
                          hipStream_t s, cplx<R>* cbuf = nullptr, int accumulate = 0,
                          Problem* prof = nullptr, int st_gemm = ST_M2L, int grid_cap = 0,
                          bool run_reduce = true, hipEvent_t done = nullptr,
                          hipEvent_t start = nullptr) {
  GemmJob<R> j{&op, src, dst, cbuf};
  return launch_grouped_jobs<R, KIND>(&j, 1, adj, s, accumulate, prof, st_gemm, grid_cap,
                                      run_reduce, done, start);
}

// The per-destination reductions of several M2L products (their GEMMs
// launched with run_reduce = false), up to MAX_JOBS per launch.
template <typename R>
static int launch_reduce_jobs(const std::vector<GemmJob<R>>& jobs, bool adj, hipStream_t s,
                              Problem* prof = nullptr, int st_red = ST_M2L_RED) {
  for (size_t a = 0; a < jobs.size(); a += MAX_JOBS) {
    const int nj = (int)std::min<size_t>(MAX_JOBS, jobs.size() - a);
    RedBatch<R> rb{};
    rb.n = nj;
    int nbox = 0;
    for (int q = 0; q < nj; ++q) {
      const GroupedOp<R>& op = *jobs[a + q].op;
      RedJobDev<R>& RJ = rb.job[q];
      RJ.ncoef = adj ? op.cols : op.rows;
      RJ.ptr = adj ? op.red_ptr_adj : op.red_ptr;
      RJ.pairs = adj ? op.red_pairs_adj : op.red_pairs;
      RJ.cbuf = jobs[a + q].cbuf;
      RJ.dst = jobs[a + q].dst;
      rb.box0[q] = nbox;
      nbox += adj ? op.n_red_adj : op.n_red;
    }
    rb.box0[nj] = nbox;
    if (nbox == 0) continue;
    int ev = prof ? prof_begin(*prof, s) : -1;
    hipLaunchKernelGGL(k_pair_reduce<R>, dim3(nbox), dim3(256), 0, s, rb, 0);
    BEM_LAUNCH_CHECK();
    if (prof) {
      int pr = prof_end(*prof, ev, prof_slot(st_red, sizeof(R) == 4, adj), s);
      if (pr) return pr;
    }
  }
  return 0;
}

// near-field job of one problem (buffers X)
template <typename R>
static P2PJobDev<R> p2p_job(Problem& P, PrecisionData<R>& D, ExecBuf<R>& X, bool adj) {
  P2PJobDev<R> j{};
  j.geo = D.geo;
  j.n = P.n;
  j.bstart = P.box_start[P.L];
  j.u_ptr = P.u_ptr;
  j.u_idx = P.u_idx;
  j.ps = X.ps;
  j.qs = X.qs;
  j.ys = X.ys;
  j.ys2 = X.ys2;
  j.k = (R)P.k;
  j.alr = (R)P.alpha.re;
  j.ali = (R)P.alpha.im;
  j.all_src = P.direct ? 1 : 0;
  j.nptr = adj ? P.neart_ptr : P.near_ptr;
  j.nidx = adj ? P.neart_row : P.near_col;
  j.ncp = adj ? D.neart_cp : D.near_cp;
  j.ncq = adj ? D.neart_cq : D.near_cq;
  return j;
}

// one P2P launch over up to MAX_JOBS problems (imag: all with alpha_re = 0);
// grid_cap > 0 caps the grid (grid-stride over the leaves)
template <typename R>
static int launch_p2p_jobs(const P2PJobDev<R>* jobs, const int* nleaf, int nj, bool adj,
                           bool imag, int grid_cap, hipStream_t s, hipEvent_t done = nullptr) {
  if (nj <= 0) {
    if (done) BEM_HIP_TRY(hipEventRecord(done, s));
    return 0;
  }
  if (nj > MAX_JOBS) {
    set_error("too many near-field jobs in one launch");
    return -1;
  }
  P2PBatch<R> b{};
  b.n = nj;
  int tot = 0;
  for (int q = 0; q < nj; ++q) {
    b.leaf0[q] = tot;
    b.job[q] = jobs[q];
    tot += nleaf[q];
  }
  b.leaf0[nj] = tot;
  b.total = tot;
  if (tot == 0) {
    if (done) BEM_HIP_TRY(hipEventRecord(done, s));
    return 0;
  }
  const int grid = (grid_cap > 0 && grid_cap < tot) ? grid_cap : tot;
  if (adj) {
    bool wz = true;
    for (int q = 0; q < nj; ++q) wz = wz && jobs[q].q_zero;
    if (imag && wz)
      launch_done(k_p2p_adj<R, true, true>, dim3(grid), dim3(P2P_THREADS), 0, s, nullptr, done, b);
    else if (imag)
      launch_done(k_p2p_adj<R, true, false>, dim3(grid), dim3(P2P_THREADS), 0, s, nullptr, done,
                  b);
    else if (wz)
      launch_done(k_p2p_adj<R, false, true>, dim3(grid), dim3(P2P_THREADS), 0, s, nullptr, done,
                  b);
    else
      launch_done(k_p2p_adj<R, false, false>, dim3(grid), dim3(P2P_THREADS), 0, s, nullptr, done,
                  b);
  } else {
    bool qz = true;
    for (int q = 0; q < nj; ++q) qz = qz && jobs[q].q_zero;
    if (imag && qz)
      launch_done(k_p2p<R, true, true>, dim3(grid), dim3(P2P_THREADS), 0, s, nullptr, done, b);
    else if (imag)
      launch_done(k_p2p<R, true, false>, dim3(grid), dim3(P2P_THREADS), 0, s, nullptr, done, b);
    else if (qz)
      launch_done(k_p2p<R, false, true>, dim3(grid), dim3(P2P_THREADS), 0, s, nullptr, done, b);
    else
      launch_done(k_p2p<R, false, false>, dim3(grid), dim3(P2P_THREADS), 0, s, nullptr, done, b);
  }
  BEM_LAUNCH_CHECK();
  return 0;
}

// one leaf-accumulation launch (mode 0 P2M, 2 P2M with q = 0, 1 L2P^H) over up to
// MAX_JOBS problems
template <typename R>
static int launch_leaf_jobs(const LeafJobDev<R>* jobs, const int* nleaf, int nj, int mode,
                            hipStream_t s, hipEvent_t done = nullptr) {
  if (nj <= 0) {
    if (done) BEM_HIP_TRY(hipEventRecord(done, s));
    return 0;
  }
  if (nj > MAX_JOBS) {
    set_error("too many leaf jobs in one launch");
    return -1;
  }
  LeafBatch<R> b{};
  b.n = nj;
  int tot = 0;
  for (int q = 0; q < nj; ++q) {
    b.leaf0[q] = tot;
    b.job[q] = jobs[q];
    tot += nleaf[q];
  }
  b.leaf0[nj] = tot;
  b.total = tot;
  if (tot == 0) {
    if (done) BEM_HIP_TRY(hipEventRecord(done, s));
    return 0;
  }
  launch_done(k_leaf_accumulate<R>, dim3(tot), dim3(256), 0, s, nullptr, done, b, mode);
  BEM_LAUNCH_CHECK();
  return 0;
}

// M2L of the levels 2 .. L-1 (all inputs ready once the upward pass is done):
// consecutive levels with the same pair-tile width share a launch (up to
// MAX_JOBS levels), each level keeping the width chosen for it
template <typename R>
static int launch_coarse_m2l(Problem& P, PrecisionData<R>& D, ExecBuf<R>& X, bool adj,
                             hipStream_t s) {
  const int L = P.L;
  std::vector<GemmJob<R>> all;
  int l = 2;
  while (l < L) {
    GemmJob<R> jobs[MAX_JOBS];
    int nj = 0;
    const int key = tile_key(D.m2l[l], adj);
    for (; l < L && nj < MAX_JOBS && tile_key(D.m2l[l], adj) == key; ++l, ++nj) {
      jobs[nj].op = &D.m2l[l];
      jobs[nj].src = adj ? X.Lc[l] : X.M[l];
      jobs[nj].dst = adj ? X.M[l] : X.Lc[l];
      jobs[nj].cbuf = X.cbuf + D.cbuf_off[l];
      all.push_back(jobs[nj]);
    }
    int r = launch_grouped_jobs<R, 0>(jobs, nj, adj, s, 0, P.prof_on ? &P : nullptr, ST_M2L, 0,
                                      false);
    if (r) return r;
  }
  return launch_reduce_jobs<R>(all, adj, s, P.prof_on ? &P : nullptr);
}

// Upward pass: leaf multipoles to the n_direct levels above in one launch
// (KIND 3), then the level-by-level chain above them.  Adjoint: the mirror
// image for the adjoint locals (direct L2L^H, then the L2L^H chain).
template <typename R>
static int upward_pass(Problem& P, PrecisionData<R>& D, ExecBuf<R>& X, bool adj,
                       hipStream_t s) {
  const int L = P.L, nd = std::min(D.n_direct, P.ndir[sizeof(R) == 4]);
  GemmJob<R> jobs[MAX_JOBS];
  for (int d = 1; d <= nd; ++d) {
    if (adj)
      jobs[d - 1] = GemmJob<R>{&D.l2l_dir[d], X.Lc[L], X.Lc[L - d], nullptr};
    else
      jobs[d - 1] = GemmJob<R>{&D.m2m_dir[d], X.M[L], X.M[L - d], nullptr};
  }
  int r = 0;
  if (nd > 0) {
    r = adj ? launch_grouped_jobs<R, 4>(jobs, nd, true, s) : launch_grouped_jobs<R, 3>(jobs, nd, false, s);
    if (r) return r;
  }
  for (int l = L - nd; l >= 3; --l) {
    cplx<R>* par = adj ? X.Lc[l - 1] : X.M[l - 1];  // cleared by the gather kernel
    r = adj ? launch_grouped<R, 2>(D.l2l[l], true, X.Lc[l], par, s)
            : launch_grouped<R, 1>(D.m2m[l], false, X.M[l], par, s);
    if (r) return r;
  }
  return 0;
}

// Downward pass: the level-by-level chain down to level L - n_direct (totals
// there), then all n_direct levels to the leaves in one launch (KIND 4).
// The leaf level receives only the translated part (onto a cleared buffer);
// the leaf finish adds the leaf-level M2L.  Adjoint: the mirror image (M2M^H
// chain, direct M2M^H).
template <typename R>
static int downward_pass(Problem& P, PrecisionData<R>& D, ExecBuf<R>& X, bool adj,
                         hipStream_t s) {
  const int L = P.L, nd = std::min(D.n_direct, P.ndir[sizeof(R) == 4]);
  int r = 0;
  for (int l = 3; l <= L - nd; ++l) {
    r = adj ? launch_grouped<R, 1>(D.m2m[l], true, X.M[l - 1], X.M[l], s)
            : launch_grouped<R, 2>(D.l2l[l], false, X.Lc[l - 1], X.Lc[l], s);
    if (r) return r;
  }
  if (nd > 0) {
    GemmJob<R> jobs[MAX_JOBS];
    for (int d = 1; d <= nd; ++d) {
      if (adj)
        jobs[d - 1] = GemmJob<R>{&D.m2m_dir[d], X.M[L - d], X.M[L], nullptr};
      else
        jobs[d - 1] = GemmJob<R>{&D.l2l_dir[d], X.Lc[L - d], X.Lc[L], nullptr};
    }
    r = adj ? launch_grouped_jobs<R, 3>(jobs, nd, true, s) : launch_grouped_jobs<R, 4>(jobs, nd, false, s);
    if (r) return r;
  }
  return 0;
}

// the parent-level expansions accumulated atomically in the chain (M for the
// forward upward pass, L for the adjoint one), cleared by the gather kernel;
// with leaf, also the leaf-level target of the downward pass (L forward, M
// adjoint), whose M2L part the leaf finish adds
template <typename R>
static ZeroList<R> chain_zero_list(Problem& P, PrecisionData<R>& D, ExecBuf<R>& X, bool adj,
                                   bool leaf = false) {
  ZeroList<R> z{};
  z.n = 0;
  if (P.direct) return z;
  if (leaf) {
    z.ptr[z.n] = adj ? X.M[P.L] : X.Lc[P.L];
    z.cnt[z.n] = (int64_t)P.nbox[P.L] * D.ncoef[P.L];
    ++z.n;
  }
  for (int l = P.L - 1; l >= 2 && z.n < MAX_ZERO; --l) {
    z.ptr[z.n] = adj ? X.Lc[l] : X.M[l];
    z.cnt[z.n] = (int64_t)P.nbox[l] * D.ncoef[l];
    ++z.n;
  }
  return z;
}


// Join before the finish.  With the leaf-level M2L on the third stream (the
// later of the two side paths to finish), that stream first waits for the
// near field's completion event, so the caller's stream waits on one event
// (each wait there costs it several microseconds).
static int join_side_streams(Problem& P, hipStream_t s, bool leaf_side) {
  if (leaf_side) {
    BEM_HIP_TRY(hipStreamWaitEvent(P.side2, P.ev_join, 0));
    BEM_HIP_TRY(hipEventRecord(P.ev_join2, P.side2));
    BEM_HIP_TRY(hipStreamWaitEvent(s, P.ev_join2, 0));
  } else {
    BEM_HIP_TRY(hipStreamWaitEvent(s, P.ev_join, 0));
  }
  return 0;
}

template <typename R>
int fmm_apply_x(Problem& P, PrecisionData<R>& D, ExecBuf<R>& X, const c64* p, const c64* q,
                c64* y, hipStream_t s) {
  const int64_t n = P.n;
  const int L = P.L;
  const R k = (R)P.k, alr = (R)P.alpha.re, ali = (R)P.alpha.im;
  constexpr int ADJ_FLAG = 0;
  int nb = ceil_div(n, 256);
  const int nleaf = P.nbox[L];
  const int sched = P.direct ? 0 : P.sched[sizeof(R) == 4];
  const int cap = P.direct ? 0 : P.p2p_cap[sizeof(R) == 4];
  const bool p2p_first = sched == SCHED_CONCURRENT || sched == SCHED_LEAF_SERIAL ||
                         sched == SCHED_SERIAL || P.direct;
  // every stage on this stream (direct sum, serial schedule or serial stage
  // profile)
  const bool one_stream = P.direct || sched == SCHED_SERIAL || (P.prof_on && P.prof_serial);
  // gather and P2M in one launch when a leaf's values fit in LDS and the
  // near field does not start right after the gather (it would start later:
  // measured slower); its completion (event ev_fork2) forks the leaf M2L
  const size_t lds_fused = 2 * (size_t)P.max_leaf * sizeof(cplx<R>);
  const bool fused = !P.direct && !p2p_first && lds_fused <= FUSED_LDS_MAX;
  // else the gather's completion forks the near field when it follows directly
  const bool fork_at_gather = p2p_first && !one_stream;
  int r = 0;
  PROF_BEGIN(e0);
  if (fused) {
    launch_done(k_gather_leaf<R, false>, dim3(nleaf), dim3(256), lds_fused, s, nullptr,
                P.ev_fork2, p, q, P.perm, P.box_start[L], D.ncoef[L], q ? D.p2m : D.p2m_p, X.ps,
                X.qs, X.p64s,
                X.q64s, X.M[L], chain_zero_list(P, D, X, false, true));
  } else {
    launch_done(k_gather_in<R>, dim3(nb), dim3(256), 0, s, nullptr,
                fork_at_gather ? P.ev_fork : nullptr, p, q, P.perm, n, X.ps, X.qs, X.p64s,
                X.q64s, chain_zero_list(P, D, X, false, true));
  }
  BEM_LAUNCH_CHECK();
  PROF_END(e0, fused ? ST_P2M : ST_GATHER);
  // the near field runs on the side stream, concurrently with the far field
  auto launch_p2p = [&]() -> int {
    hipStream_t sn = one_stream ? s : P.side;
    if (!one_stream) {
      hipEvent_t fork = P.ev_fork;
      if (sched == SCHED_LEAF_THEN_P2P)
        fork = P.ev_fork2;  // completion of the P2M (or gather + P2M)
      else if (!fork_at_gather)
        BEM_HIP_TRY(hipEventRecord(P.ev_fork, s));
      BEM_HIP_TRY(hipStreamWaitEvent(sn, fork, 0));
    }
    int e1 = prof_begin(P, sn);
    P2PJobDev<R> job = p2p_job(P, D, X, false);
    job.q_zero = q ? 0 : 1;
    int rr = launch_p2p_jobs<R>(&job, &nleaf, 1, false, P.alpha.re == 0.0, cap, sn,
                                one_stream ? nullptr : P.ev_join);
    if (rr) return rr;
    int pr = prof_end(P, e1, prof_slot(ST_P2P, sizeof(R) == 4, false), sn);
    if (pr) return pr;
    return 0;
  };
  if (p2p_first && (r = launch_p2p())) return r;
  if (P.direct) {
    hipLaunchKernelGGL(k_finish<R>, dim3(ceil_div(n * FIN_LANES, 256)), dim3(256), 0, s, n, P.perm,
                       P.elem_leaf, 0, D.l2p, X.Lc[L], nullptr, nullptr, nullptr,
                       nullptr, X.ps, X.qs, X.ys, P.diag_p, P.diag_q, X.p64s, X.q64s, y);
    BEM_LAUNCH_CHECK();
    return 0;
  }
  // leaf-level M2L (needs only the leaf multipoles): on its own stream
  // (SCHED_CONCURRENT), or on this stream before the upward pass; the fork
  // is signalled by the P2M launch
  const bool leaf_side = !one_stream && (sched == SCHED_CONCURRENT ||
                                         sched == SCHED_P2P_AFTER_UP ||
                                         sched == SCHED_LEAF_THEN_P2P);
  hipStream_t sl = leaf_side ? P.side2 : s;
  if (!fused) {
    PROF_BEGIN(e2);
    // with q = 0 the q columns meet zeros: the p columns alone are read
    const LeafJobDev<R> lj{P.box_start[L], D.ncoef[L], q ? D.p2m : D.p2m_p, X.ps, X.qs, X.M[L]};
    if ((r = launch_leaf_jobs<R>(&lj, &nleaf, 1, q ? 0 : 2, s, leaf_side ? P.ev_fork2 : nullptr)))
      return r;
    PROF_END(e2, ST_P2M);
  }
  if (leaf_side) BEM_HIP_TRY(hipStreamWaitEvent(P.side2, P.ev_fork2, 0));
  // (its per-destination sums are formed by the leaf finish)
  hipEvent_t m2l_start, m2l_done;
  leaf_m2l_events<R>(P, false, &m2l_start, &m2l_done);
  if ((r = launch_grouped<R, 0>(D.m2l[L], false, X.M[L], X.Lc[L], sl, X.cbufL, 0,
                                P.prof_on ? &P : nullptr, ST_M2L_LEAF,
                                P.m2l_cap[sizeof(R) == 4], false, m2l_done, m2l_start)))
    return r;
  if ((sched == SCHED_LEAF_FIRST || sched == SCHED_LEAF_THEN_P2P) && (r = launch_p2p()))
    return r;
  PROF_BEGIN(e3);
  if ((r = upward_pass<R>(P, D, X, false, s))) return r;
  PROF_END(e3, ST_M2M);
  if (sched == SCHED_P2P_AFTER_UP && (r = launch_p2p())) return r;
  if ((r = launch_coarse_m2l<R>(P, D, X, false, s))) return r;
  PROF_BEGIN(e5);
  if ((r = downward_pass<R>(P, D, X, false, s))) return r;
  PROF_END(e5, ST_L2L);
  if (!one_stream && (r = join_side_streams(P, s, leaf_side))) return r;
  PROF_BEGIN(e6);
  {
    const GroupedOp<R>& op = D.m2l[L];
    hipLaunchKernelGGL(k_leaf_finish<R>, dim3(nleaf), dim3(256), sizeof(cplx<R>) * D.ncoef[L], s,
                       P.box_start[L], D.ncoef[L], op.red_ptr, op.red_pairs, X.cbufL, X.Lc[L], n,
                       P.perm, D.l2p, nullptr, nullptr, nullptr, nullptr, X.ps, X.qs,
                       X.ys, P.diag_p, P.diag_q, X.p64s, X.q64s, y);
    BEM_LAUNCH_CHECK();
  }
  PROF_END(e6, ST_FINISH);
  return 0;
}

template <typename R>
__global__ void k_gather_adj(const c64* __restrict__ y, const int* __restrict__ perm, int64_t n,
                             cplx<R>* __restrict__ ys, c64* __restrict__ y64,
                             const ZeroList<R> zl) {
  zero_list(zl, grid_tid(), grid_threads());
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  c64 a = y[perm[i]];
  ys[i] = mk<R>((R)a.re, (R)a.im);
  y64[i] = a;
}

template <typename R>
int fmm_apply_adjoint_x(Problem& P, PrecisionData<R>& D, ExecBuf<R>& X, const c64* y, c64* u,
                        c64* w, hipStream_t s) {
  const int64_t n = P.n;
  const int L = P.L;
  const R k = (R)P.k, alr = (R)P.alpha.re, ali = (R)P.alpha.im;
  constexpr int ADJ_FLAG = 1;
  int nb = ceil_div(n, 256);
  // sorted input in X.ps, X.p64s; P2P results in X.ys (u) and X.ys2 (w)
  const int nleaf = P.nbox[L];
  const int sched = P.direct ? 0 : P.sched[sizeof(R) == 4];
  const int cap = P.direct ? 0 : P.p2p_cap[sizeof(R) == 4];
  const bool p2p_first = sched == SCHED_CONCURRENT || sched == SCHED_LEAF_SERIAL ||
                         sched == SCHED_SERIAL || P.direct;
  // every stage on this stream (direct sum, serial schedule or serial stage
  // profile)
  const bool one_stream = P.direct || sched == SCHED_SERIAL || (P.prof_on && P.prof_serial);
  // gather and L2P^H in one launch under the forward product's conditions
  const size_t lds_fused = (size_t)P.max_leaf * sizeof(cplx<R>);
  const bool fused = !P.direct && !p2p_first && lds_fused <= FUSED_LDS_MAX;
  const bool fork_at_gather = p2p_first && !one_stream;
  int r = 0;
  PROF_BEGIN(e0);
  if (fused) {
    launch_done(k_gather_leaf<R, true>, dim3(nleaf), dim3(256), lds_fused, s, nullptr,
                P.ev_fork2, y, (const c64*)nullptr, P.perm, P.box_start[L], D.ncoef[L], D.l2p,
                X.ps, (cplx<R>*)nullptr, X.p64s, (c64*)nullptr, X.Lc[L],
                chain_zero_list(P, D, X, true, true));
  } else {
    launch_done(k_gather_adj<R>, dim3(nb), dim3(256), 0, s, nullptr,
                fork_at_gather ? P.ev_fork : nullptr, y, P.perm, n, X.ps, X.p64s,
                chain_zero_list(P, D, X, true, true));
  }
  BEM_LAUNCH_CHECK();
  PROF_END(e0, fused ? ST_P2M : ST_GATHER);
  auto launch_p2p = [&]() -> int {
    hipStream_t sn = one_stream ? s : P.side;
    if (!one_stream) {
      hipEvent_t fork = P.ev_fork;
      if (sched == SCHED_LEAF_THEN_P2P)
        fork = P.ev_fork2;  // completion of the L2P^H (or gather + L2P^H)
      else if (!fork_at_gather)
        BEM_HIP_TRY(hipEventRecord(P.ev_fork, s));
      BEM_HIP_TRY(hipStreamWaitEvent(sn, fork, 0));
    }
    int e1 = prof_begin(P, sn);
    P2PJobDev<R> job = p2p_job(P, D, X, true);
    job.q_zero = w ? 0 : 1;
    int rr = launch_p2p_jobs<R>(&job, &nleaf, 1, true, P.alpha.re == 0.0, cap, sn,
                                one_stream ? nullptr : P.ev_join);
    if (rr) return rr;
    int pr = prof_end(P, e1, prof_slot(ST_P2P, sizeof(R) == 4, true), sn);
    if (pr) return pr;
    return 0;
  };
  if (p2p_first && (r = launch_p2p())) return r;
  if (P.direct) {
    hipLaunchKernelGGL(k_finish_adj<R>, dim3(ceil_div(n * FIN_LANES, 256)), dim3(256), 0, s, n, P.perm,
                       P.elem_leaf, 0, D.p2m, X.M[L], nullptr, nullptr, nullptr,
                       nullptr, X.ps, X.ys, X.ys2, P.diag_p, P.diag_q, X.p64s, u, w);
    BEM_LAUNCH_CHECK();
    return 0;
  }
  // adjoint locals (L2P^H) in Lc, adjoint multipoles in M
  // leaf-level M2L^H (needs only the leaf adjoint locals): own stream or
  // this one, as in the forward product
  const bool leaf_side = !one_stream && (sched == SCHED_CONCURRENT ||
                                         sched == SCHED_P2P_AFTER_UP ||
                                         sched == SCHED_LEAF_THEN_P2P);
  hipStream_t sl = leaf_side ? P.side2 : s;
  if (!fused) {
    PROF_BEGIN(e2);
    const LeafJobDev<R> lj{P.box_start[L], D.ncoef[L], D.l2p, X.ps, nullptr, X.Lc[L]};
    if ((r = launch_leaf_jobs<R>(&lj, &nleaf, 1, 1, s, leaf_side ? P.ev_fork2 : nullptr)))
      return r;
    PROF_END(e2, ST_P2M);
  }
  if (leaf_side) BEM_HIP_TRY(hipStreamWaitEvent(P.side2, P.ev_fork2, 0));
  hipEvent_t m2l_start, m2l_done;
  leaf_m2l_events<R>(P, true, &m2l_start, &m2l_done);
  if ((r = launch_grouped<R, 0>(D.m2l[L], true, X.Lc[L], X.M[L], sl, X.cbufL, 0,
                                P.prof_on ? &P : nullptr, ST_M2L_LEAF,
                                P.m2l_cap[sizeof(R) == 4], false, m2l_done, m2l_start)))
    return r;
  if ((sched == SCHED_LEAF_FIRST || sched == SCHED_LEAF_THEN_P2P) && (r = launch_p2p()))
    return r;
  PROF_BEGIN(e5);
  if ((r = upward_pass<R>(P, D, X, true, s))) return r;
  PROF_END(e5, ST_L2L);
  if (sched == SCHED_P2P_AFTER_UP && (r = launch_p2p())) return r;
  if ((r = launch_coarse_m2l<R>(P, D, X, true, s))) return r;
  PROF_BEGIN(e3);
  if ((r = downward_pass<R>(P, D, X, true, s))) return r;
  PROF_END(e3, ST_M2M);
  if (!one_stream && (r = join_side_streams(P, s, leaf_side))) return r;
  PROF_BEGIN(e6);
  {
    const GroupedOp<R>& op = D.m2l[L];
    // w not wanted (rigid adjoint): the p columns of P2M^H alone
    if (w)
      hipLaunchKernelGGL((k_leaf_finish_adj<R, false>), dim3(nleaf), dim3(256),
                         sizeof(cplx<R>) * D.ncoef[L], s, P.box_start[L], D.ncoef[L],
                         op.red_ptr_adj, op.red_pairs_adj, X.cbufL, X.M[L], n, P.perm, D.p2m,
                         nullptr, nullptr, nullptr, nullptr, X.ps, X.ys, X.ys2, P.diag_p,
                         P.diag_q, X.p64s, u, w);
    else
      hipLaunchKernelGGL((k_leaf_finish_adj<R, true>), dim3(nleaf), dim3(256),
                         sizeof(cplx<R>) * D.ncoef[L], s, P.box_start[L], D.ncoef[L],
                         op.red_ptr_adj, op.red_pairs_adj, X.cbufL, X.M[L], n, P.perm, D.p2m_p,
                         nullptr, nullptr, nullptr, nullptr, X.ps, X.ys, X.ys2, P.diag_p,
                         P.diag_q, X.p64s, u, w);
    BEM_LAUNCH_CHECK();
  }
  PROF_END(e6, ST_FINISH);
  return 0;
}

// grouped launches of any number of jobs: by pair-tile width, MAX_JOBS at a time
template <typename R, int KIND>
static int launch_grouped_any(const std::vector<GemmJob<R>>& jobs, bool adj, hipStream_t s) {
  for (int key : {1, 16, 32, 64, 128}) {
    std::vector<GemmJob<R>> g;
    for (const GemmJob<R>& j : jobs)
      if ((KIND == 0 ? tile_key(*j.op, adj) : (adj ? j.op->ct_adj : j.op->ct)) == key)
        g.push_back(j);
    for (size_t a = 0; a < g.size(); a += MAX_JOBS) {
      const int nj = (int)std::min<size_t>(MAX_JOBS, g.size() - a);
      int r = launch_grouped_jobs<R, KIND>(&g[a], nj, adj, s, 0, nullptr, ST_M2L, 0, false);
      if (r) return r;
    }
  }
  // M2L: the per-destination reductions of every tile width in one pass
  return KIND == 0 ? launch_reduce_jobs<R>(jobs, adj, s) : 0;
}

// The batched product: every stage is one launch (or one per tile width and
// MAX_JOBS items) over all items, in the order of the single product (near
// field and leaf-level M2L on the side streams when given); the gathers and
// finishes take MAX_JOBS items per launch.  Level chains of problems with
// different depths are merged step by step from the leaves.  The leaf-level
// M2L is reduced by its own pass here (the finish is per element).
template <typename R>
int fmm_apply_batch(const std::vector<BatchItem<R>>& items, bool adj, const BatchStreams& bs) {
  int r = 0;
  hipStream_t s = bs.main;
  const bool sides = bs.side && bs.side2;
  hipStream_t sn = sides ? bs.side : s, sl = sides ? bs.side2 : s;
  // gathers (and the clears of the atomically accumulated expansions), up
  // to MAX_JOBS items per launch; an item with more cleared levels than a
  // batched job holds gets a launch of its own
  {
    GatherBatch<R> gb{};
    auto flush = [&]() -> int {
      if (gb.n == 0) return 0;
      if (adj)
        hipLaunchKernelGGL((k_gather_batch<R, true>), dim3(gb.blk0[gb.n]), dim3(256), 0, s, gb);
      else
        hipLaunchKernelGGL((k_gather_batch<R, false>), dim3(gb.blk0[gb.n]), dim3(256), 0, s, gb);
      BEM_LAUNCH_CHECK();
      gb = GatherBatch<R>{};
      return 0;
    };
    for (const BatchItem<R>& it : items) {
      Problem& P = *it.P;
      PrecisionData<R>& D = *it.D;
      ExecBuf<R>& X = *it.X;
      const int nb = ceil_div(P.n, 256);
      const ZeroList<R> z = chain_zero_list(P, D, X, adj);
      if (z.n > BATCH_ZERO) {
        if (adj)
          hipLaunchKernelGGL(k_gather_adj<R>, dim3(nb), dim3(256), 0, s, it.in, P.perm, P.n, X.ps,
                             X.p64s, z);
        else
          hipLaunchKernelGGL(k_gather_in<R>, dim3(nb), dim3(256), 0, s, it.in, it.q, P.perm, P.n,
                             X.ps, X.qs, X.p64s, X.q64s, z);
        BEM_LAUNCH_CHECK();
        continue;
      }
      GatherJobDev<R>& J = gb.job[gb.n];
      J = GatherJobDev<R>{it.in, adj ? nullptr : it.q, P.perm, P.n, X.ps, X.qs, X.p64s, X.q64s, {}};
      J.zl.n = z.n;
      for (int e = 0; e < z.n; ++e) {
        J.zl.ptr[e] = z.ptr[e];
        J.zl.cnt[e] = z.cnt[e];
      }
      gb.blk0[gb.n + 1] = gb.blk0[gb.n] + nb;
      if (++gb.n == MAX_JOBS && (r = flush())) return r;
    }
    if ((r = flush())) return r;
  }
  // near field, by kind of alpha
  if (sides) {
    BEM_HIP_TRY(hipEventRecord(bs.ev[0], s));
    BEM_HIP_TRY(hipStreamWaitEvent(sn, bs.ev[0], 0));
  }
  for (int imag = 0; imag < 2; ++imag) {
    std::vector<P2PJobDev<R>> jobs;
    std::vector<int> nl;
    for (const BatchItem<R>& it : items)
      if ((it.P->alpha.re == 0.0) == (imag == 1)) {
        P2PJobDev<R> job = p2p_job(*it.P, *it.D, *it.X, adj);
        job.q_zero = adj ? (it.out2 ? 0 : 1) : (it.q ? 0 : 1);
        jobs.push_back(job);
        nl.push_back(it.P->nbox[it.P->L]);
      }
    for (size_t a = 0; a < jobs.size(); a += MAX_JOBS) {
      const int nj = (int)std::min<size_t>(MAX_JOBS, jobs.size() - a);
      if ((r = launch_p2p_jobs<R>(&jobs[a], &nl[a], nj, adj, imag == 1, 0, sn))) return r;
    }
  }
  if (sides) BEM_HIP_TRY(hipEventRecord(bs.ev[1], sn));
  // far field of the items that have one
  std::vector<const BatchItem<R>*> far;
  for (const BatchItem<R>& it : items)
    if (!it.P->direct) far.push_back(&it);
  // (forward items with q = 0 read the p columns alone: mode 2, launched
  // apart from those with q)
  for (int pass = 0; pass < (adj ? 1 : 2); ++pass) {
    std::vector<LeafJobDev<R>> jobs;
    std::vector<int> nl;
    for (const BatchItem<R>* it : far) {
      Problem& P = *it->P;
      PrecisionData<R>& D = *it->D;
      ExecBuf<R>& X = *it->X;
      const int L = P.L;
      if (adj)
        jobs.push_back(LeafJobDev<R>{P.box_start[L], D.ncoef[L], D.l2p, X.ps, nullptr, X.Lc[L]});
      else if (pass == 0 && it->q)
        jobs.push_back(LeafJobDev<R>{P.box_start[L], D.ncoef[L], D.p2m, X.ps, X.qs, X.M[L]});
      else if (pass == 1 && !it->q)
        jobs.push_back(LeafJobDev<R>{P.box_start[L], D.ncoef[L], D.p2m_p, X.ps, nullptr, X.M[L]});
      else
        continue;
      nl.push_back(P.nbox[L]);
    }
    const int mode = adj ? 1 : (pass == 0 ? 0 : 2);
    for (size_t a = 0; a < jobs.size(); a += MAX_JOBS) {
      const int nj = (int)std::min<size_t>(MAX_JOBS, jobs.size() - a);
      if ((r = launch_leaf_jobs<R>(&jobs[a], &nl[a], nj, mode, s))) return r;
    }
  }
  // level chains only: merged across problems step by step they need few
  // launches, while the direct operators (8^d per depth, mostly sparse
  // groups) cost more than they save once launches are shared
  auto nd_of = [](const BatchItem<R>*) { return 0; };
  // leaf-level M2L
  if (sides) {
    BEM_HIP_TRY(hipEventRecord(bs.ev[2], s));
    BEM_HIP_TRY(hipStreamWaitEvent(sl, bs.ev[2], 0));
  }
  {
    std::vector<GemmJob<R>> jobs;
    for (const BatchItem<R>* it : far) {
      const int L = it->P->L;
      ExecBuf<R>& X = *it->X;
      jobs.push_back(GemmJob<R>{&it->D->m2l[L], adj ? X.Lc[L] : X.M[L], adj ? X.M[L] : X.Lc[L],
                                X.cbufL});
    }
    if ((r = launch_grouped_any<R, 0>(jobs, adj, sl))) return r;
  }
  if (sides) BEM_HIP_TRY(hipEventRecord(bs.ev[3], sl));
  // upward pass: direct translations, then the chains step by step
  {
    std::vector<GemmJob<R>> jobs;
    int max_steps = 0;
    for (const BatchItem<R>* it : far) {
      const int L = it->P->L, nd = nd_of(it);
      ExecBuf<R>& X = *it->X;
      for (int d = 1; d <= nd; ++d)
        jobs.push_back(adj ? GemmJob<R>{&it->D->l2l_dir[d], X.Lc[L], X.Lc[L - d], nullptr}
                           : GemmJob<R>{&it->D->m2m_dir[d], X.M[L], X.M[L - d], nullptr});
      max_steps = std::max(max_steps, L - nd - 2);
    }
    if (adj) {
      if ((r = launch_grouped_any<R, 4>(jobs, true, s))) return r;
    } else {
      if ((r = launch_grouped_any<R, 3>(jobs, false, s))) return r;
    }
    for (int t = 0; t < max_steps; ++t) {
      jobs.clear();
      for (const BatchItem<R>* it : far) {
        const int l = it->P->L - nd_of(it) - t;  // level l -> l - 1
        if (l < 3) continue;
        ExecBuf<R>& X = *it->X;
        jobs.push_back(adj ? GemmJob<R>{&it->D->l2l[l], X.Lc[l], X.Lc[l - 1], nullptr}
                           : GemmJob<R>{&it->D->m2m[l], X.M[l], X.M[l - 1], nullptr});
      }
      if (adj) {
        if ((r = launch_grouped_any<R, 2>(jobs, true, s))) return r;
      } else {
        if ((r = launch_grouped_any<R, 1>(jobs, false, s))) return r;
      }
    }
  }
  // M2L of the levels above the leaves
  {
    std::vector<GemmJob<R>> jobs;
    for (const BatchItem<R>* it : far) {
      ExecBuf<R>& X = *it->X;
      for (int l = 2; l < it->P->L; ++l)
        jobs.push_back(GemmJob<R>{&it->D->m2l[l], adj ? X.Lc[l] : X.M[l],
                                  adj ? X.M[l] : X.Lc[l], X.cbuf + it->D->cbuf_off[l]});
    }
    if ((r = launch_grouped_any<R, 0>(jobs, adj, s))) return r;
  }
  // downward pass (its last step writes the leaf level): the chains step
  // by step, then the direct translations
  if (sides) BEM_HIP_TRY(hipStreamWaitEvent(s, bs.ev[3], 0));
  {
    std::vector<GemmJob<R>> jobs;
    int max_steps = 0;
    for (const BatchItem<R>* it : far) max_steps = std::max(max_steps, it->P->L - nd_of(it) - 2);
    for (int t = 0; t < max_steps; ++t) {
      jobs.clear();
      for (const BatchItem<R>* it : far) {
        const int l = 3 + t;  // level l - 1 -> l
        if (l > it->P->L - nd_of(it)) continue;
        ExecBuf<R>& X = *it->X;
        jobs.push_back(adj ? GemmJob<R>{&it->D->m2m[l], X.M[l - 1], X.M[l], nullptr}
                           : GemmJob<R>{&it->D->l2l[l], X.Lc[l - 1], X.Lc[l], nullptr});
      }
      if (adj) {
        if ((r = launch_grouped_any<R, 1>(jobs, true, s))) return r;
      } else {
        if ((r = launch_grouped_any<R, 2>(jobs, false, s))) return r;
      }
    }
    jobs.clear();
    for (const BatchItem<R>* it : far) {
      const int L = it->P->L, nd = nd_of(it);
      ExecBuf<R>& X = *it->X;
      for (int d = 1; d <= nd; ++d)
        jobs.push_back(adj ? GemmJob<R>{&it->D->m2m_dir[d], X.M[L - d], X.M[L], nullptr}
                           : GemmJob<R>{&it->D->l2l_dir[d], X.Lc[L - d], X.Lc[L], nullptr});
    }
    if (adj) {
      if ((r = launch_grouped_any<R, 3>(jobs, true, s))) return r;
    } else {
      if ((r = launch_grouped_any<R, 4>(jobs, false, s))) return r;
    }
  }
  // finish, up to MAX_JOBS items per launch
  if (sides) BEM_HIP_TRY(hipStreamWaitEvent(s, bs.ev[1], 0));
  {
    FinBatch<R> fb{};
    bool fb_wz = false;  // the adjoint jobs of fb want no w (P2M^H p columns alone)
    auto flush = [&]() -> int {
      if (fb.n == 0) return 0;
      if (adj && fb_wz)
        hipLaunchKernelGGL((k_finish_batch<R, true, true>), dim3(fb.blk0[fb.n]), dim3(256), 0, s,
                           fb);
      else if (adj)
        hipLaunchKernelGGL((k_finish_batch<R, true>), dim3(fb.blk0[fb.n]), dim3(256), 0, s, fb);
      else
        hipLaunchKernelGGL((k_finish_batch<R, false>), dim3(fb.blk0[fb.n]), dim3(256), 0, s, fb);
      BEM_LAUNCH_CHECK();
      fb = FinBatch<R>{};
      return 0;
    };
    for (const BatchItem<R>& it : items) {
      Problem& P = *it.P;
      PrecisionData<R>& D = *it.D;
      ExecBuf<R>& X = *it.X;
      const int L = P.L;
      const int ncoef = P.direct ? 0 : D.ncoef[L];
      const bool wz = adj && !it.out2 && !P.direct;
      if (fb.n > 0 && wz != fb_wz && (r = flush())) return r;
      fb_wz = wz;
      if (adj)
        fb.job[fb.n] = FinJobDev<R>{P.n, P.perm, P.elem_leaf, ncoef, wz ? D.p2m_p : D.p2m, X.M[L],
                                    nullptr, nullptr, nullptr, nullptr, X.ps,
                                    X.ys, X.ys2, P.diag_p, P.diag_q, X.p64s, nullptr, it.out,
                                    it.out2};
      else
        fb.job[fb.n] = FinJobDev<R>{P.n, P.perm, P.elem_leaf, ncoef, D.l2p, X.Lc[L],
                                    nullptr, nullptr, nullptr, nullptr, X.ps,
                                    X.qs, X.ys, P.diag_p, P.diag_q, X.p64s, X.q64s, it.out,
                                    nullptr};
      fb.blk0[fb.n + 1] = fb.blk0[fb.n] + ceil_div(P.n * FIN_LANES, 256);
      if (++fb.n == MAX_JOBS && (r = flush())) return r;
    }
    if ((r = flush())) return r;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Accuracy of a built problem: the product on seeded pseudo-random (white)
// densities and on a plane-wave density against the exact discrete operator
// on sampled rows.  The two differ: white noise mostly cancels in the far
// field, where a smooth density adds up coherently, so the same truncation
// gives the smooth density a larger error relative to the product.
// ---------------------------------------------------------------------------
// Re and Im uniform in [-1, 1) from a 64-bit mix of (seed, index)
// (splitmix64's finaliser)
__device__ __forceinline__ double unit_from_hash(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// p = exp(i k d.x), q = dp/dn = i k (d.n) p at the collocation points (caller
// order): a smooth density, whose far field adds up coherently
__global__ void k_fill_plane(const double* __restrict__ geo, int64_t n,
                             const int* __restrict__ perm, double k, double dx, double dy,
                             double dz, c64* __restrict__ p, c64* __restrict__ q) {
  const int64_t i = grid_tid();
  if (i >= n) return;
  const double ph = k * (dx * geo[GEO_CX * n + i] + dy * geo[GEO_CY * n + i] +
                         dz * geo[GEO_CZ * n + i]);
  const double dn = dx * geo[GEO_NX * n + i] + dy * geo[GEO_NY * n + i] + dz * geo[GEO_NZ * n + i];
  double sn, cs;
  sincos(ph, &sn, &cs);
  const int o = perm[i];
  p[o] = mk(cs, sn);
  q[o] = mk(-k * dn * sn, k * dn * cs);
}

__global__ void k_fill_random(c64* __restrict__ v, int64_t n, uint64_t seed) {
  const int64_t i = grid_tid();
  if (i < n)
    v[i] = mk(unit_from_hash(seed * 0x100000000ull + 2 * (uint64_t)i),
              unit_from_hash(seed * 0x100000000ull + 2 * (uint64_t)i + 1));
}

// One block per sampled row (sorted target index rows[t]): the exact row of
// the discrete operator applied to p, q (caller order), in float64: the
// 3-point rule over every other element, the near-field corrections of the
// row and the diagonal (I/2, alpha/2, self integrals).
__global__ void __launch_bounds__(256)
    k_exact_rows(const double* __restrict__ geo, int64_t n, const int* __restrict__ perm,
                 const int* __restrict__ rows, const c64* __restrict__ p,
                 const c64* __restrict__ q, double k, double alr, double ali,
                 const int* __restrict__ nptr, const int* __restrict__ ncol,
                 const c64* __restrict__ ncp, const c64* __restrict__ ncq,
                 const c64* __restrict__ dp, const c64* __restrict__ dq, c64* __restrict__ out) {
  __shared__ double sr[256], si[256];
  const int i = rows[blockIdx.x];
  const double xx = geo[GEO_CX * n + i], xy = geo[GEO_CY * n + i], xz = geo[GEO_CZ * n + i];
  const double nxx = geo[GEO_NX * n + i], nxy = geo[GEO_NY * n + i],
               nxz = geo[GEO_NZ * n + i];
  c64 acc = mk(0.0, 0.0);
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    if (j == i) continue;
    double yq[9];
    for (int c = 0; c < 9; ++c) yq[c] = geo[(GEO_QX0 + c) * n + j];
    const double nyx = geo[GEO_NX * n + j], nyy = geo[GEO_NY * n + j],
                 nyz = geo[GEO_NZ * n + j];
    const double d = yq[0] * nyx + yq[1] * nyy + yq[2] * nyz;
    c64 sp, sq;
    bm_elem<double, false>(xx, xy, xz, nxx, nxy, nxz, yq, nyx, nyy, nyz, d, k, 0.0, alr, ali, sp,
                           sq);
    const double w = geo[GEO_AREA * n + j] * (1.0 / 3.0) * INV_4PI_D;
    const int o = perm[j];
    cfma(acc, cscale(sp, w), p[o]);
    cfma(acc, cscale(sq, w), q[o]);
  }
  for (int t = nptr[i] + threadIdx.x; t < nptr[i + 1]; t += blockDim.x) {
    const int o = perm[ncol[t]];
    cfma(acc, ncp[t], p[o]);
    cfma(acc, ncq[t], q[o]);
  }
  sr[threadIdx.x] = acc.re;
  si[threadIdx.x] = acc.im;
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
    const int o = perm[i];
    cfma(v, dp[i], p[o]);
    cfma(v, dq[i], q[o]);
    out[blockIdx.x] = v;
  }
}

__global__ void k_gather_rows(const c64* __restrict__ y, const int* __restrict__ perm,
                              const int* __restrict__ rows, int m, c64* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) out[t] = y[perm[rows[t]]];
}

template <typename R>
int measure_error(Problem& P, PrecisionData<R>& D, hipStream_t s, double* err) {
  const int64_t n = P.n;
  const int m = (int)std::min<int64_t>(128, n);
  DevArena tmp;
  struct G {
    DevArena& a;
    ~G() { a.release(); }
  } guard{tmp};
  c64 *p, *q, *y, *yr, *ys;
  int* rows;
  if (tmp.alloc((void**)&p, sizeof(c64) * n) || tmp.alloc((void**)&q, sizeof(c64) * n) ||
      tmp.alloc((void**)&y, sizeof(c64) * n) || tmp.alloc((void**)&yr, sizeof(c64) * m) ||
      tmp.alloc((void**)&ys, sizeof(c64) * m) || tmp.alloc((void**)&rows, sizeof(int) * m))
    return -2;
  // rows spread evenly over the sorted (space-filling) order
  std::vector<int> hr(m);
  for (int t = 0; t < m; ++t) hr[t] = (int)(((int64_t)t * n + n / (2 * m)) / m);
  BEM_HIP_TRY(hipMemcpyAsync(rows, hr.data(), sizeof(int) * m, hipMemcpyHostToDevice, s));
  double e[2] = {0, 0};
  for (int kind = 0; kind < 2; ++kind) {
    if (kind == 0) {  // white noise
      hipLaunchKernelGGL(k_fill_random, dim3(ceil_div(n, 256)), dim3(256), 0, s, p, n, 1ull);
      hipLaunchKernelGGL(k_fill_random, dim3(ceil_div(n, 256)), dim3(256), 0, s, q, n, 2ull);
    } else {  // plane wave along (1, 2, 3) / sqrt(14)
      const double c = 1.0 / std::sqrt(14.0);
      hipLaunchKernelGGL(k_fill_plane, dim3(ceil_div(n, 256)), dim3(256), 0, s, P.geo, n, P.perm,
                         P.k, c, 2.0 * c, 3.0 * c, p, q);
    }
    BEM_LAUNCH_CHECK();
    int r = fmm_apply_x<R>(P, D, D.X, p, q, y, s);
    if (r) return r;
    hipLaunchKernelGGL(k_exact_rows, dim3(m), dim3(256), 0, s, P.geo, n, P.perm, rows, p, q,
                       P.k, P.alpha.re, P.alpha.im, P.near_ptr, P.near_col, P.f64.near_cp,
                       P.f64.near_cq, P.diag_p, P.diag_q, yr);
    hipLaunchKernelGGL(k_gather_rows, dim3(ceil_div(m, 64)), dim3(64), 0, s, y, P.perm, rows, m,
                       ys);
    BEM_LAUNCH_CHECK();
    std::vector<c64> a(m), b(m);
    BEM_HIP_TRY(hipMemcpyAsync(a.data(), ys, sizeof(c64) * m, hipMemcpyDeviceToHost, s));
    BEM_HIP_TRY(hipMemcpyAsync(b.data(), yr, sizeof(c64) * m, hipMemcpyDeviceToHost, s));
    BEM_HIP_TRY(hipStreamSynchronize(s));
    double num = 0, den = 0;
    for (int t = 0; t < m; ++t) {
      const double dr = a[t].re - b[t].re, di = a[t].im - b[t].im;
      num += dr * dr + di * di;
      den += b[t].re * b[t].re + b[t].im * b[t].im;
    }
    e[kind] = den > 0 ? std::sqrt(num / den) : 0.0;
  }
  D.err = e[0];
  D.err_smooth = e[1];
  *err = std::max(e[0], e[1]);
  return 0;
}
template int measure_error<float>(Problem&, PrecisionData<float>&, hipStream_t, double*);
template int measure_error<double>(Problem&, PrecisionData<double>&, hipStream_t, double*);

template <typename R>
int fmm_apply(Problem& P, PrecisionData<R>& D, const c64* p, const c64* q, c64* y,
              hipStream_t s) {
  return fmm_apply_x<R>(P, D, D.X, p, q, y, s);
}
template <typename R>
int fmm_apply_adjoint(Problem& P, PrecisionData<R>& D, const c64* y, c64* u, c64* w,
                      hipStream_t s) {
  return fmm_apply_adjoint_x<R>(P, D, D.X, y, u, w, s);
}

// Far field at evaluation points off the boundary: the problem's multipoles
// for (p, q) (gather, P2M, upward pass, as in a product), then the locals of
// the point boxes level by level: L2L from the parent point box onto the
// cleared locals (one pair per child), then the M2L from the source boxes
// (a point box receives several of them in one launch): float32 writes
// per-pair outputs and sums them per box in a fixed order, float64 adds
// atomically.
template <typename R>
int point_far_field(Problem& P, PrecisionData<R>& D, FieldPoints& F, PointOps<R>& O,
                    const c64* p, const c64* q, hipStream_t s, hipEvent_t fork) {
  const int L = P.L;
  ExecBuf<R>& X = O.X;
  ZeroList<R> z = chain_zero_list(P, D, X, false, false);
  for (int l = 2; l <= L; ++l) {
    if (z.n >= MAX_ZERO) {
      set_error("too many levels for the point-box clear");
      return -1;
    }
    z.ptr[z.n] = O.Lc[l];
    z.cnt[z.n] = (int64_t)F.nbox[l] * D.ncoef[l];
    ++z.n;
  }
  constexpr int ADJ_FLAG = 0;
  Problem* prof = P.prof_on ? &P : nullptr;
  PROF_BEGIN(e0);
  hipLaunchKernelGGL(k_gather_in<R>, dim3(ceil_div(P.n, 256)), dim3(256), 0, s, p, q, P.perm,
                     P.n, X.ps, X.qs, X.p64s, X.q64s, z);
  BEM_LAUNCH_CHECK();
  PROF_END(e0, ST_GATHER);
  if (fork) BEM_HIP_TRY(hipEventRecord(fork, s));
  const int nleaf = P.nbox[L];
  const LeafJobDev<R> lj{P.box_start[L], D.ncoef[L], q ? D.p2m : D.p2m_p, X.ps, X.qs, X.M[L]};
  PROF_BEGIN(e1);
  int r = launch_leaf_jobs<R>(&lj, &nleaf, 1, q ? 0 : 2, s);
  if (r) return r;
  PROF_END(e1, ST_P2M);
  PROF_BEGIN(e2);
  if ((r = upward_pass(P, D, X, false, s))) return r;
  PROF_END(e2, ST_M2M);
  for (int l = 2; l <= L && !r; ++l) {
    if (l >= 3) r = launch_grouped<R, 2>(O.l2l[l], false, O.Lc[l - 1], O.Lc[l], s, nullptr, 0,
                                         prof, ST_L2L);
    if (!r && O.cbuf)  // per-pair outputs, then the fixed-order sums
      r = launch_grouped<R, 0>(O.m2l[l], false, X.M[l], O.Lc[l], s, O.cbuf + O.cbuf_off[l], 1,
                               prof, l == L ? ST_M2L_LEAF : ST_M2L);
    else if (!r)
      r = launch_grouped<R, 1>(O.m2l[l], false, X.M[l], O.Lc[l], s, nullptr, 0, prof,
                               l == L ? ST_M2L_LEAF : ST_M2L);
  }
  return r;
}
template int point_far_field<float>(Problem&, PrecisionData<float>&, FieldPoints&,
                                    PointOps<float>&, const c64*, const c64*, hipStream_t,
                                    hipEvent_t);
template int point_far_field<double>(Problem&, PrecisionData<double>&, FieldPoints&,
                                     PointOps<double>&, const c64*, const c64*, hipStream_t,
                                     hipEvent_t);

template int fmm_apply_x<float>(Problem&, PrecisionData<float>&, ExecBuf<float>&, const c64*,
                                const c64*, c64*, hipStream_t);
template int fmm_apply_x<double>(Problem&, PrecisionData<double>&, ExecBuf<double>&, const c64*,
                                 const c64*, c64*, hipStream_t);
template int fmm_apply_adjoint_x<float>(Problem&, PrecisionData<float>&, ExecBuf<float>&,
                                        const c64*, c64*, c64*, hipStream_t);
template int fmm_apply_adjoint_x<double>(Problem&, PrecisionData<double>&, ExecBuf<double>&,
                                         const c64*, c64*, c64*, hipStream_t);
template int fmm_apply_batch<float>(const std::vector<BatchItem<float>>&, bool,
                                    const BatchStreams&);
template int fmm_apply_batch<double>(const std::vector<BatchItem<double>>&, bool,
                                     const BatchStreams&);
template int fmm_apply<float>(Problem&, PrecisionData<float>&, const c64*, const c64*, c64*,
                              hipStream_t);
template int fmm_apply<double>(Problem&, PrecisionData<double>&, const c64*, const c64*, c64*,
                               hipStream_t);
template int fmm_apply_adjoint<float>(Problem&, PrecisionData<float>&, const c64*, c64*, c64*,
                                      hipStream_t);
template int fmm_apply_adjoint<double>(Problem&, PrecisionData<double>&, const c64*, c64*, c64*,
                                       hipStream_t);

}  // namespace bemfmm
