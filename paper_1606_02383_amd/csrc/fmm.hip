// The FMM-accelerated Burton-Miller product and its exact adjoint.
//
//   y = (I/2 - K - alpha H) p + (S + alpha K' + (alpha/2) I) q
//
// (the paper's boundary integral equation, Sec. 2.3, combined with its
// normal derivative).  Per product, in float32 or float64:
//   gather   caller order -> Morton order, split by precision
//   P2P      3-point-rule direct sum over neighbouring leaves (U lists), j != i
//   P2M      leaf multipoles from per-element matrices (monopole q, dipole p)
//   M2M      child -> parent, grouped by octant
//   M2L      interaction lists, grouped by translation vector
//   L2L      parent -> child
//   finish   L2P + near-field corrections (accurate - 3-point rule) + the
//            float64 diagonal (I/2, alpha/2 I and self integrals), scatter
// The grouped translations are gather-GEMM-scatter kernels: every pair of
// one group shares one dense matrix, the output columns are accumulated with
// atomics.  The adjoint applies the conjugate transpose of every stage in
// reverse order with the same lists and matrices.
//
// Pair kernel (rv = x - y, u = 1/r, G = exp(ikr)/(4 pi r)):
//   coefficient of p_j: -(G_y + alpha G_xy)
//       = G [a1 (rv.n_y + alpha n_x.n_y) + alpha a2 (rv.n_x)(rv.n_y) u^2]
//   coefficient of q_j:  G + alpha G_x = G [1 + alpha a1 rv.n_x]
// with a1 = iku - u^2 and a2 = 3u^2 - k^2 - 3iku.
#include <cmath>

#include "plan.h"

namespace bemfmm {

constexpr float INV_4PI_F = 0.07957747154594767f;
constexpr double INV_4PI_D = 0.07957747154594767;

template <typename R>
__device__ __forceinline__ void sincos_r(R x, R* s, R* c);
template <>
__device__ __forceinline__ void sincos_r<float>(float x, float* s, float* c) {
  sincosf(x, s, c);
}
template <>
__device__ __forceinline__ void sincos_r<double>(double x, double* s, double* c) {
  sincos(x, s, c);
}
template <typename R>
__device__ __forceinline__ R rsqrt_r(R x);
template <>
__device__ __forceinline__ float rsqrt_r<float>(float x) {
  return rsqrtf(x);
}
template <>
__device__ __forceinline__ double rsqrt_r<double>(double x) {
  return 1.0 / sqrt(x);
}

// kernel coefficients (cp, cq) of one (target, source point) pair; w
// includes the rule weight and 1/(4 pi).
template <typename R>
__device__ __forceinline__ void bm_pair(R xx, R xy, R xz, R nxx, R nxy, R nxz, R yx, R yy, R yz,
                                        R nyx, R nyy, R nyz, R w, R k, R alr, R ali,
                                        cplx<R>& cp, cplx<R>& cq) {
  R rx = xx - yx, ry = xy - yy, rz = xz - yz;
  R r2 = rx * rx + ry * ry + rz * rz;
  R u = rsqrt_r<R>(r2);
  R r = r2 * u;
  R sn, cs;
  sincos_r<R>(k * r, &sn, &cs);
  R gs = w * u;
  cplx<R> G = mk<R>(cs * gs, sn * gs);
  R u2 = u * u;
  cplx<R> a1 = mk<R>(-u2, k * u);
  cplx<R> a2 = mk<R>(R(3) * u2 - k * k, R(-3) * k * u);
  R rnx = rx * nxx + ry * nxy + rz * nxz;
  R rny = rx * nyx + ry * nyy + rz * nyz;
  R nn = nxx * nyx + nxy * nyy + nxz * nyz;
  cplx<R> al = mk<R>(alr, ali);
  // a1 * (rny + alpha nn) + alpha a2 rnx rny u^2
  cplx<R> t1 = cmul(a1, mk<R>(rny + alr * nn, ali * nn));
  cplx<R> t2 = cmul(al, cscale(a2, rnx * rny * u2));
  cp = cmul(G, cadd(t1, t2));
  cplx<R> t3 = cmul(al, cscale(a1, rnx));
  cq = cmul(G, mk<R>(R(1) + t3.re, t3.im));
}

// ---------------------------------------------------------------------------
// gather / scatter
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_gather_in(const c64* __restrict__ p, const c64* __restrict__ q,
                            const int* __restrict__ perm, int64_t n, cplx<R>* __restrict__ ps,
                            cplx<R>* __restrict__ qs, c64* __restrict__ p64,
                            c64* __restrict__ q64) {
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

template <typename R>
__global__ void k_zero(cplx<R>* __restrict__ a, int64_t cnt) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < cnt) a[i] = mk<R>(R(0), R(0));
}

// ---------------------------------------------------------------------------
// P2P: one block per leaf; sources of the U list staged in LDS in chunks
// ---------------------------------------------------------------------------
constexpr int P2P_THREADS = 256;
constexpr int P2P_CHUNK = 128;

template <typename R>
__global__ void __launch_bounds__(P2P_THREADS)
    k_p2p(const R* __restrict__ geo, int64_t n, const int* __restrict__ bstart,
          const int* __restrict__ u_ptr, const int* __restrict__ u_idx,
          const cplx<R>* __restrict__ ps, const cplx<R>* __restrict__ qs, R k, R alr, R ali,
          int all_src, cplx<R>* __restrict__ ys) {
  __shared__ R s_q[9][P2P_CHUNK];
  __shared__ R s_n[3][P2P_CHUNK];
  __shared__ R s_w[P2P_CHUNK];
  __shared__ R s_pq[4][P2P_CHUNK];
  __shared__ int s_id[P2P_CHUNK];
  __shared__ int s_nb[28], s_pre[28];
  __shared__ cplx<R> s_red[P2P_THREADS];
  const int b = blockIdx.x, tid = threadIdx.x;
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
        s_n[0][v] = geo[GEO_NX * n + j];
        s_n[1][v] = geo[GEO_NY * n + j];
        s_n[2][v] = geo[GEO_NZ * n + j];
        s_w[v] = geo[GEO_AREA * n + j] * R(1.0 / 3.0) * R(INV_4PI_D);
        cplx<R> pv = ps[j], qv = qs[j];
        s_pq[0][v] = pv.re;
        s_pq[1][v] = pv.im;
        s_pq[2][v] = qv.re;
        s_pq[3][v] = qv.im;
        s_id[v] = j;
      }
      __syncthreads();
      if (active) {
        for (int v = sl; v < cnt; v += nsl) {
          if (s_id[v] == i) continue;
          cplx<R> sp = mk<R>(0, 0), sq = mk<R>(0, 0);
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            cplx<R> cp, cq;
            bm_pair<R>(xx, xy, xz, nxx, nxy, nxz, s_q[3 * q][v], s_q[3 * q + 1][v],
                       s_q[3 * q + 2][v], s_n[0][v], s_n[1][v], s_n[2][v], s_w[v], k, alr, ali,
                       cp, cq);
            sp = cadd(sp, cp);
            sq = cadd(sq, cq);
          }
          cfma(acc, sp, mk<R>(s_pq[0][v], s_pq[1][v]));
          cfma(acc, sq, mk<R>(s_pq[2][v], s_pq[3][v]));
        }
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

// Adjoint P2P: one block per leaf of output elements j; iterates over the
// target elements i of the U list:  u_j += conj(cp_ij) y_i,  w_j += conj(cq_ij) y_i.
template <typename R>
__global__ void __launch_bounds__(P2P_THREADS)
    k_p2p_adj(const R* __restrict__ geo, int64_t n, const int* __restrict__ bstart,
              const int* __restrict__ u_ptr, const int* __restrict__ u_idx,
              const cplx<R>* __restrict__ ysrt, R k, R alr, R ali, int all_src,
              cplx<R>* __restrict__ us, cplx<R>* __restrict__ ws) {
  __shared__ R s_x[6][P2P_CHUNK];
  __shared__ R s_y[2][P2P_CHUNK];
  __shared__ int s_id[P2P_CHUNK];
  __shared__ int s_nb[28], s_pre[28];
  __shared__ cplx<R> s_red[2][P2P_THREADS];
  const int b = blockIdx.x, tid = threadIdx.x;
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
    R q[9], nyx = 0, nyy = 0, nyz = 0, w = 0;
    for (int c = 0; c < 9; ++c) q[c] = active ? geo[(GEO_QX0 + c) * n + j] : R(0);
    if (active) {
      nyx = geo[GEO_NX * n + j];
      nyy = geo[GEO_NY * n + j];
      nyz = geo[GEO_NZ * n + j];
      w = geo[GEO_AREA * n + j] * R(1.0 / 3.0) * R(INV_4PI_D);
    }
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
          cplx<R> sp = mk<R>(0, 0), sq = mk<R>(0, 0);
#pragma unroll
          for (int qq = 0; qq < 3; ++qq) {
            cplx<R> cp, cq;
            bm_pair<R>(s_x[0][v], s_x[1][v], s_x[2][v], s_x[3][v], s_x[4][v], s_x[5][v],
                       q[3 * qq], q[3 * qq + 1], q[3 * qq + 2], nyx, nyy, nyz, w, k, alr, ali,
                       cp, cq);
            sp = cadd(sp, cp);
            sq = cadd(sq, cq);
          }
          cplx<R> yv = mk<R>(s_y[0][v], s_y[1][v]);
          cfmac(au, sp, yv);
          cfmac(aw, sq, yv);
        }
      }
    }
    __syncthreads();
    s_red[0][tid] = active ? au : mk<R>(0, 0);
    s_red[1][tid] = active ? aw : mk<R>(0, 0);
    __syncthreads();
    if (tid < nTg) {
      cplx<R> su = mk<R>(0, 0), sw = mk<R>(0, 0);
      for (int q2 = 0; q2 < nsl; ++q2) {
        su = cadd(su, s_red[0][q2 * nTg + tid]);
        sw = cadd(sw, s_red[1][q2 * nTg + tid]);
      }
      us[t0 + tg + tid] = su;
      ws[t0 + tg + tid] = sw;
    }
  }
}

// ---------------------------------------------------------------------------
// P2M (forward) and L2P^H (adjoint): per leaf, per coefficient sums over the
// leaf's elements.  mode 0: M[b][c] = sum_e A[e][c][0] p_e + A[e][c][1] q_e;
// mode 1: M[b][c] = sum_e conj(B[e][c]) y_e.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_leaf_accumulate(const int* __restrict__ bstart, int ncoef,
                                  const cplx<R>* __restrict__ mat, const cplx<R>* __restrict__ a,
                                  const cplx<R>* __restrict__ bvec, int mode,
                                  cplx<R>* __restrict__ out) {
  const int b = blockIdx.x;
  const int e0 = bstart[b], e1 = bstart[b + 1];
  for (int c = threadIdx.x; c < ncoef; c += blockDim.x) {
    cplx<R> acc = mk<R>(0, 0);
    for (int e = e0; e < e1; ++e) {
      if (mode == 0) {
        cfma(acc, mat[((int64_t)e * ncoef + c) * 2], a[e]);
        cfma(acc, mat[((int64_t)e * ncoef + c) * 2 + 1], bvec[e]);
      } else {
        cfmac(acc, mat[(int64_t)e * ncoef + c], a[e]);
      }
    }
    out[(int64_t)b * ncoef + c] = acc;
  }
}

// ---------------------------------------------------------------------------
// grouped gather-GEMM-scatter on the matrix cores:
//   dst[pair_dst] += op_g src[pair_src]      (ADJ: op_g conjugate-transposed)
// Workgroup tile: 64 output rows x 64 pairs; four waves, each 32 x 32.  The
// complex product runs as four real 16x16x4 MFMA products per 16x16 block:
//   C_re += A_re B_re - A_im B_im,   C_im += A_re B_im + A_im B_re.
// Operands are staged through LDS, 16 complex k per stage; output columns are
// accumulated with atomics (pairs of one group never share a destination, but
// different groups do).
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

constexpr int G_RT = 64, G_CT = 64, G_KC = 16, G_LD = G_KC + 1;

template <typename R, bool ADJ, int KIND>
__global__ void __launch_bounds__(256)
    k_grouped_gemm(int mat_rows, int mat_cols, const int* __restrict__ tile_group,
                   const int* __restrict__ tile_pair0, const int* __restrict__ tile_npairs,
                   const int* __restrict__ tile_row0, const int* __restrict__ group_slot,
                   const cplx<R>* __restrict__ mats, const int* __restrict__ pair_dst,
                   const int* __restrict__ pair_src, const cplx<R>* __restrict__ src,
                   cplx<R>* __restrict__ dst, cplx<R>* __restrict__ cbuf) {
  typedef typename MfmaOp<R>::v4 v4;
  __shared__ R a_re[G_RT * G_LD], a_im[G_RT * G_LD];
  __shared__ R b_re[G_CT * G_LD], b_im[G_CT * G_LD];
  __shared__ int s_src[G_CT], s_dst[G_CT];
  // XCD-aware order: workgroups go to the 8 XCDs round-robin (block b on XCD
  // b % 8), so give each XCD a contiguous range of tiles; consecutive tiles
  // share their group's matrix, which then stays in that XCD's L2.
  const int nt = gridDim.x, xcd = blockIdx.x & 7, slot_in_xcd = blockIdx.x >> 3;
  const int tile = xcd * (nt >> 3) + min(xcd, nt & 7) + slot_in_xcd;
  const int tid = threadIdx.x;
  const int grp = tile_group[tile], p0 = tile_pair0[tile], np = tile_npairs[tile];
  const int r0 = tile_row0[tile];
  const int slot = group_slot[grp];
  const int out_rows = ADJ ? mat_cols : mat_rows;  // rows of the effective op
  const int in_cols = ADJ ? mat_rows : mat_cols;
  const cplx<R>* M = mats + (int64_t)slot * mat_rows * mat_cols;
  if (tid < G_CT) {
    s_src[tid] = (tid < np) ? pair_src[p0 + tid] : -1;
    s_dst[tid] = (tid < np) ? pair_dst[p0 + tid] : -1;
  }
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  v4 cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = v4{0, 0, 0, 0};
      ci[a][b] = v4{0, 0, 0, 0};
    }
  __syncthreads();
  for (int k0 = 0; k0 < in_cols; k0 += G_KC) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int e = tid + 256 * q;
      int kk, rr;
      if (ADJ) {
        rr = e % G_RT;
        kk = e / G_RT;
      } else {
        kk = e % G_KC;
        rr = e / G_KC;
      }
      int r = r0 + rr, c = k0 + kk;
      cplx<R> v = mk<R>(0, 0);
      if (r < out_rows && c < in_cols) {
        if (ADJ) {
          cplx<R> m = M[(int64_t)c * mat_cols + r];
          v = mk<R>(m.re, -m.im);
        } else {
          v = M[(int64_t)r * mat_cols + c];
        }
      }
      a_re[rr * G_LD + kk] = v.re;
      a_im[rr * G_LD + kk] = v.im;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int e = tid + 256 * q;
      int kk = e % G_KC, cc = e / G_KC;
      int c = k0 + kk;
      cplx<R> v = mk<R>(0, 0);
      if (cc < np && c < in_cols) v = src[(int64_t)s_src[cc] * in_cols + c];
      b_re[cc * G_LD + kk] = v.re;
      b_im[cc * G_LD + kk] = v.im;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < G_KC; ks += 4) {
      R ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        int row = wr * 32 + rb * 16 + li;
        ar[rb] = a_re[row * G_LD + ks + lk];
        ai[rb] = a_im[row * G_LD + ks + lk];
        nai[rb] = -ai[rb];
      }
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        int col = wc * 32 + cb * 16 + li;
        br[cb] = b_re[col * G_LD + ks + lk];
        bi[cb] = b_im[col * G_LD + ks + lk];
      }
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          cr[rb][cb] = MfmaOp<R>::mma(ar[rb], br[cb], cr[rb][cb]);
          cr[rb][cb] = MfmaOp<R>::mma(nai[rb], bi[cb], cr[rb][cb]);
          ci[rb][cb] = MfmaOp<R>::mma(ar[rb], bi[cb], ci[rb][cb]);
          ci[rb][cb] = MfmaOp<R>::mma(ai[rb], br[cb], ci[rb][cb]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int row = r0 + wr * 32 + rb * 16 + MfmaOp<R>::row(lk, e);
        int cc = wc * 32 + cb * 16 + li;
        if (row < out_rows && cc < np) {
          cplx<R> v = mk<R>(cr[rb][cb][e], ci[rb][cb][e]);
          if (cbuf) {  // per-pair output, reduced per destination afterwards
            cbuf[(int64_t)(p0 + cc) * out_rows + row] = v;
          } else if ((KIND == 2 && !ADJ) || (KIND == 1 && ADJ)) {
            // parent -> child: every child is the destination of exactly one pair
            cplx<R>* d = &dst[(int64_t)s_dst[cc] * out_rows + row];
            *d = cadd(*d, v);
          } else {
            atomic_cadd(&dst[(int64_t)s_dst[cc] * out_rows + row], v);
          }
        }
      }
}

// dst[b][c] (+)= sum over the pairs t of box b of cbuf[t][c]  (pairs listed
// per box in a fixed order: deterministic, no atomics)
// 256 threads per box: 4 slices of 64 coefficients, each slice sums every
// fourth pair, then the slices are added in a fixed order.
template <typename R>
__global__ void __launch_bounds__(256)
    k_pair_reduce(int ncoef, const int* __restrict__ ptr, const int* __restrict__ pairs,
                  const cplx<R>* __restrict__ cbuf, int accumulate, cplx<R>* __restrict__ dst) {
  __shared__ cplx<R> part[4][64];
  const int b = blockIdx.x;
  const int t0 = ptr[b], t1 = ptr[b + 1];
  const int lane = threadIdx.x & 63, slice = threadIdx.x >> 6;
  for (int c0 = 0; c0 < ncoef; c0 += 64) {
    const int c = c0 + lane;
    cplx<R> acc = mk<R>(0, 0);
    if (c < ncoef)
      for (int t = t0 + slice; t < t1; t += 4) acc = cadd(acc, cbuf[(int64_t)pairs[t] * ncoef + c]);
    part[slice][lane] = acc;
    __syncthreads();
    if (slice == 0 && c < ncoef) {
      cplx<R> s = accumulate ? dst[(int64_t)b * ncoef + c] : mk<R>(0, 0);
      s = cadd(s, cadd(cadd(part[0][lane], part[1][lane]), cadd(part[2][lane], part[3][lane])));
      dst[(int64_t)b * ncoef + c] = s;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// finish: one wavefront per element
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R wave_reduce(R v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
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
  int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (i >= n) return;
  cplx<R> acc = mk<R>(0, 0);
  if (ncoef > 0) {
    const cplx<R>* Bi = l2p + i * ncoef;
    const cplx<R>* Lb = Lc + (int64_t)elem_leaf[i] * ncoef;
    for (int c = lane; c < ncoef; c += 64) cfma(acc, Bi[c], Lb[c]);
  }
  for (int t = near_ptr[i] + lane; t < near_ptr[i + 1]; t += 64) {
    int j = near_col[t];
    cfma(acc, ncp[t], ps[j]);
    cfma(acc, ncq[t], qs[j]);
  }
  acc.re = wave_reduce(acc.re);
  acc.im = wave_reduce(acc.im);
  if (lane == 0) {
    cplx<R> s = cadd(acc, ys[i]);
    c64 out = mk((double)s.re, (double)s.im);
    cfma(out, dp[i], p64[i]);
    cfma(out, dq[i], q64[i]);
    y[perm[i]] = out;
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
  int64_t j = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (j >= n) return;
  cplx<R> au = mk<R>(0, 0), aw = mk<R>(0, 0);
  if (ncoef > 0) {
    const cplx<R>* Aj = p2m + j * ncoef * 2;
    const cplx<R>* Mb = Mc + (int64_t)elem_leaf[j] * ncoef;
    for (int c = lane; c < ncoef; c += 64) {
      cfmac(au, Aj[2 * c], Mb[c]);
      cfmac(aw, Aj[2 * c + 1], Mb[c]);
    }
  }
  for (int t = tptr[j] + lane; t < tptr[j + 1]; t += 64) {
    cplx<R> yv = ysrt[trow[t]];
    cfmac(au, tcp[t], yv);
    cfmac(aw, tcq[t], yv);
  }
  au.re = wave_reduce(au.re);
  au.im = wave_reduce(au.im);
  aw.re = wave_reduce(aw.re);
  aw.im = wave_reduce(aw.im);
  if (lane == 0) {
    cplx<R> su = cadd(au, us[j]), sw = cadd(aw, ws[j]);
    c64 ou = mk((double)su.re, (double)su.im), ow = mk((double)sw.re, (double)sw.im);
    cfmac(ou, dp[j], y64[j]);
    cfmac(ow, dq[j], y64[j]);
    int o = perm[j];
    if (u) u[o] = ou;
    if (w) w[o] = ow;
  }
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

#define PROF_BEGIN(var) int var = prof_begin(P, s)
#define PROF_END(var, stage)                                                  \
  do {                                                                        \
    int _pr = prof_end(P, var, (stage) + 8 * (sizeof(R) == 4) + 16 * ADJ_FLAG, s); \
    if (_pr) return _pr;                                                      \
  } while (0)

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------
// KIND only separates the kernel names (0 M2L, 1 M2M, 2 L2L) for profilers
// With cbuf (and the op's per-destination pair lists) the product is
// written per pair and then reduced per destination box, replacing dst
// (accumulate = 0) or adding to it; without, it is accumulated atomically.
template <typename R, int KIND>
static int launch_grouped(const GroupedOp<R>& op, bool adj, const cplx<R>* src, cplx<R>* dst,
                          hipStream_t s, cplx<R>* cbuf = nullptr, int accumulate = 0,
                          Problem* prof = nullptr) {
  int nt = adj ? op.n_tiles_adj : op.n_tiles;
  if (nt > 0) {
    int evg = prof ? prof_begin(*prof, s) : -1;
    if (adj)
      hipLaunchKernelGGL((k_grouped_gemm<R, true, KIND>), dim3(nt), dim3(256), 0, s, op.rows,
                         op.cols, op.tile_group_adj, op.tile_pair0_adj, op.tile_npairs_adj,
                         op.tile_row0_adj, op.group_slot, op.mats, op.pair_dst_adj,
                         op.pair_src_adj, src, dst, cbuf);
    else
      hipLaunchKernelGGL((k_grouped_gemm<R, false, KIND>), dim3(nt), dim3(256), 0, s, op.rows,
                         op.cols, op.tile_group, op.tile_pair0, op.tile_npairs, op.tile_row0,
                         op.group_slot, op.mats, op.pair_dst, op.pair_src, src, dst, cbuf);
    BEM_LAUNCH_CHECK();
    if (prof) {
      int pr = prof_end(*prof, evg, ST_M2L + 8 * (sizeof(R) == 4) + 16 * (adj ? 1 : 0), s);
      if (pr) return pr;
    }
  }
  if (cbuf && (adj ? op.n_red_adj : op.n_red) > 0) {
    int nb = adj ? op.n_red_adj : op.n_red;
    int nco = adj ? op.cols : op.rows;
    int ev = prof ? prof_begin(*prof, s) : -1;
    hipLaunchKernelGGL(k_pair_reduce<R>, dim3(nb), dim3(256), 0, s, nco,
                       adj ? op.red_ptr_adj : op.red_ptr, adj ? op.red_pairs_adj : op.red_pairs,
                       (const cplx<R>*)cbuf, accumulate, dst);
    BEM_LAUNCH_CHECK();
    if (prof) {
      int pr = prof_end(*prof, ev, ST_M2L_RED + 8 * (sizeof(R) == 4) + 16 * (adj ? 1 : 0), s);
      if (pr) return pr;
    }
  }
  return 0;
}

template <typename R>
static int zero(cplx<R>* a, int64_t cnt, hipStream_t s) {
  if (cnt <= 0) return 0;
  hipLaunchKernelGGL(k_zero<R>, dim3(ceil_div(cnt, 256)), dim3(256), 0, s, a, cnt);
  BEM_LAUNCH_CHECK();
  return 0;
}

template <typename R>
int fmm_apply(Problem& P, PrecisionData<R>& D, const c64* p, const c64* q, c64* y,
              hipStream_t s) {
  const int64_t n = P.n;
  const int L = P.L;
  const R k = (R)P.k, alr = (R)P.alpha.re, ali = (R)P.alpha.im;
  constexpr int ADJ_FLAG = 0;
  int nb = ceil_div(n, 256);
  PROF_BEGIN(e0);
  hipLaunchKernelGGL(k_gather_in<R>, dim3(nb), dim3(256), 0, s, p, q, P.perm, n, D.ps, D.qs,
                     P.p64s, P.q64s);
  BEM_LAUNCH_CHECK();
  PROF_END(e0, ST_GATHER);
  const int nleaf = P.nbox[L];
  // the near field runs on the side stream, concurrently with the far field
  hipStream_t sn = P.direct ? s : P.side;
  if (!P.direct) {
    BEM_HIP_TRY(hipEventRecord(P.ev_fork, s));
    BEM_HIP_TRY(hipStreamWaitEvent(sn, P.ev_fork, 0));
  }
  {
    int e1 = prof_begin(P, sn);
    hipLaunchKernelGGL(k_p2p<R>, dim3(nleaf), dim3(P2P_THREADS), 0, sn, (const R*)D.geo, n,
                       P.box_start[L], P.u_ptr, P.u_idx, D.ps, D.qs, k, alr, ali, (int)P.direct,
                       D.ys);
    BEM_LAUNCH_CHECK();
    int pr = prof_end(P, e1, ST_P2P + 8 * (sizeof(R) == 4), sn);
    if (pr) return pr;
  }
  if (!P.direct) BEM_HIP_TRY(hipEventRecord(P.ev_join, sn));
  int r = 0;
  if (P.direct) {
    hipLaunchKernelGGL(k_finish<R>, dim3(ceil_div(n * 64, 256)), dim3(256), 0, s, n, P.perm,
                       P.elem_leaf, 0, D.l2p, D.Lc[L], P.near_ptr, P.near_col, D.near_cp,
                       D.near_cq, D.ps, D.qs, D.ys, P.diag_p, P.diag_q, P.p64s, P.q64s, y);
    BEM_LAUNCH_CHECK();
    return 0;
  }
  PROF_BEGIN(e2);
  hipLaunchKernelGGL(k_leaf_accumulate<R>, dim3(nleaf), dim3(128), 0, s, P.box_start[L],
                     D.ncoef[L], D.p2m, D.ps, D.qs, 0, D.M[L]);
  BEM_LAUNCH_CHECK();
  PROF_END(e2, ST_P2M);
  // leaf-level M2L on its own stream: needs only the leaf multipoles
  BEM_HIP_TRY(hipEventRecord(P.ev_fork2, s));
  BEM_HIP_TRY(hipStreamWaitEvent(P.side2, P.ev_fork2, 0));
  if ((r = launch_grouped<R, 0>(D.m2l[L], false, D.M[L], D.Lc[L], P.side2, D.cbufL, 0,
                                P.prof_on ? &P : nullptr)))
    return r;
  BEM_HIP_TRY(hipEventRecord(P.ev_join2, P.side2));
  PROF_BEGIN(e3);
  for (int l = L; l >= 3; --l) {
    if ((r = zero<R>(D.M[l - 1], (int64_t)P.nbox[l - 1] * D.ncoef[l - 1], s))) return r;
    if ((r = launch_grouped<R, 1>(D.m2m[l], false, D.M[l], D.M[l - 1], s))) return r;
  }
  PROF_END(e3, ST_M2M);
  for (int l = 2; l < L; ++l)
    if ((r = launch_grouped<R, 0>(D.m2l[l], false, D.M[l], D.Lc[l], s, D.cbuf, 0,
                                  P.prof_on ? &P : nullptr))) return r;
  PROF_BEGIN(e5);
  for (int l = 3; l <= L; ++l) {
    if (l == L) BEM_HIP_TRY(hipStreamWaitEvent(s, P.ev_join2, 0));
    if ((r = launch_grouped<R, 2>(D.l2l[l], false, D.Lc[l - 1], D.Lc[l], s))) return r;
  }
  if (L < 3) BEM_HIP_TRY(hipStreamWaitEvent(s, P.ev_join2, 0));
  PROF_END(e5, ST_L2L);
  BEM_HIP_TRY(hipStreamWaitEvent(s, P.ev_join, 0));
  PROF_BEGIN(e6);
  hipLaunchKernelGGL(k_finish<R>, dim3(ceil_div(n * 64, 256)), dim3(256), 0, s, n, P.perm,
                     P.elem_leaf, D.ncoef[L], D.l2p, D.Lc[L], P.near_ptr, P.near_col, D.near_cp,
                     D.near_cq, D.ps, D.qs, D.ys, P.diag_p, P.diag_q, P.p64s, P.q64s, y);
  BEM_LAUNCH_CHECK();
  PROF_END(e6, ST_FINISH);
  return 0;
}

template <typename R>
__global__ void k_gather_adj(const c64* __restrict__ y, const int* __restrict__ perm, int64_t n,
                             cplx<R>* __restrict__ ys, c64* __restrict__ y64) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  c64 a = y[perm[i]];
  ys[i] = mk<R>((R)a.re, (R)a.im);
  y64[i] = a;
}

template <typename R>
int fmm_apply_adjoint(Problem& P, PrecisionData<R>& D, const c64* y, c64* u, c64* w,
                      hipStream_t s) {
  const int64_t n = P.n;
  const int L = P.L;
  const R k = (R)P.k, alr = (R)P.alpha.re, ali = (R)P.alpha.im;
  constexpr int ADJ_FLAG = 1;
  int nb = ceil_div(n, 256);
  // sorted input in D.ps, P.p64s; P2P results in D.ys (u) and D.ys2 (w)
  PROF_BEGIN(e0);
  hipLaunchKernelGGL(k_gather_adj<R>, dim3(nb), dim3(256), 0, s, y, P.perm, n, D.ps, P.p64s);
  BEM_LAUNCH_CHECK();
  PROF_END(e0, ST_GATHER);
  const int nleaf = P.nbox[L];
  hipStream_t sn = P.direct ? s : P.side;
  if (!P.direct) {
    BEM_HIP_TRY(hipEventRecord(P.ev_fork, s));
    BEM_HIP_TRY(hipStreamWaitEvent(sn, P.ev_fork, 0));
  }
  {
    int e1 = prof_begin(P, sn);
    hipLaunchKernelGGL(k_p2p_adj<R>, dim3(nleaf), dim3(P2P_THREADS), 0, sn, (const R*)D.geo, n,
                       P.box_start[L], P.u_ptr, P.u_idx, D.ps, k, alr, ali, (int)P.direct, D.ys,
                       D.ys2);
    BEM_LAUNCH_CHECK();
    int pr = prof_end(P, e1, ST_P2P + 8 * (sizeof(R) == 4) + 16, sn);
    if (pr) return pr;
  }
  if (!P.direct) BEM_HIP_TRY(hipEventRecord(P.ev_join, sn));
  int r = 0;
  if (P.direct) {
    hipLaunchKernelGGL(k_finish_adj<R>, dim3(ceil_div(n * 64, 256)), dim3(256), 0, s, n, P.perm,
                       P.elem_leaf, 0, D.p2m, D.M[L], P.neart_ptr, P.neart_row, D.neart_cp,
                       D.neart_cq, D.ps, D.ys, D.ys2, P.diag_p, P.diag_q, P.p64s, u, w);
    BEM_LAUNCH_CHECK();
    return 0;
  }
  // adjoint locals (L2P^H) in Lc, adjoint multipoles in M
  PROF_BEGIN(e2);
  hipLaunchKernelGGL(k_leaf_accumulate<R>, dim3(nleaf), dim3(128), 0, s, P.box_start[L],
                     D.ncoef[L], D.l2p, D.ps, (const cplx<R>*)nullptr, 1, D.Lc[L]);
  BEM_LAUNCH_CHECK();
  PROF_END(e2, ST_P2M);
  // leaf-level M2L^H on its own stream: needs only the leaf adjoint locals
  BEM_HIP_TRY(hipEventRecord(P.ev_fork2, s));
  BEM_HIP_TRY(hipStreamWaitEvent(P.side2, P.ev_fork2, 0));
  if ((r = launch_grouped<R, 0>(D.m2l[L], true, D.Lc[L], D.M[L], P.side2, D.cbufL, 0,
                                P.prof_on ? &P : nullptr)))
    return r;
  BEM_HIP_TRY(hipEventRecord(P.ev_join2, P.side2));
  PROF_BEGIN(e5);
  for (int l = L; l >= 3; --l) {
    if ((r = zero<R>(D.Lc[l - 1], (int64_t)P.nbox[l - 1] * D.ncoef[l - 1], s))) return r;
    if ((r = launch_grouped<R, 2>(D.l2l[l], true, D.Lc[l], D.Lc[l - 1], s))) return r;
  }
  PROF_END(e5, ST_L2L);
  for (int l = 2; l < L; ++l)
    if ((r = launch_grouped<R, 0>(D.m2l[l], true, D.Lc[l], D.M[l], s, D.cbuf, 0,
                                  P.prof_on ? &P : nullptr))) return r;
  PROF_BEGIN(e3);
  for (int l = 3; l <= L; ++l) {
    if (l == L) BEM_HIP_TRY(hipStreamWaitEvent(s, P.ev_join2, 0));
    if ((r = launch_grouped<R, 1>(D.m2m[l], true, D.M[l - 1], D.M[l], s))) return r;
  }
  if (L < 3) BEM_HIP_TRY(hipStreamWaitEvent(s, P.ev_join2, 0));
  PROF_END(e3, ST_M2M);
  BEM_HIP_TRY(hipStreamWaitEvent(s, P.ev_join, 0));
  PROF_BEGIN(e6);
  hipLaunchKernelGGL(k_finish_adj<R>, dim3(ceil_div(n * 64, 256)), dim3(256), 0, s, n, P.perm,
                     P.elem_leaf, D.ncoef[L], D.p2m, D.M[L], P.neart_ptr, P.neart_row,
                     D.neart_cp, D.neart_cq, D.ps, D.ys, D.ys2, P.diag_p, P.diag_q, P.p64s, u, w);
  BEM_LAUNCH_CHECK();
  PROF_END(e6, ST_FINISH);
  return 0;
}

template int fmm_apply<float>(Problem&, PrecisionData<float>&, const c64*, const c64*, c64*,
                              hipStream_t);
template int fmm_apply<double>(Problem&, PrecisionData<double>&, const c64*, const c64*, c64*,
                               hipStream_t);
template int fmm_apply_adjoint<float>(Problem&, PrecisionData<float>&, const c64*, c64*, c64*,
                                      hipStream_t);
template int fmm_apply_adjoint<double>(Problem&, PrecisionData<double>&, const c64*, c64*, c64*,
                                       hipStream_t);

}  // namespace bemfmm
