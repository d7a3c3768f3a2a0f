// Field and gradient of the integral representation at many points off the
// boundary (solver step 5 evaluated on the design-domain lattice of the
// topology loop, Sec. 3), with the boundary sums split by the problem's own
// FMM instead of summed directly.
//
// The points get an octree on the grid of the problem's tree (same origin,
// same box side per level), reaching PT_EXT level-2 boxes beyond its root
// cube.  A point box of level l is split further only while some source box
// of level l touches it (Chebyshev distance <= 1); otherwise every source is
// already well separated at this level or above and the box is a leaf.
// Interactions, for a point box t of level l:
//   * M2L from the source boxes of level l in its interaction list: every
//     non-touching source box at level 2; at l > 2 the children of the
//     source boxes touching t's parent that do not touch t,
//   * L2L from t's parent (l > 2),
//   * at a leaf: evaluation of the local expansion, value and gradient,
//     at its points (L2P),
//   * at a leaf of the deepest level: the 3-point rule summed directly over
//     the elements of the touching source leaves (P2P).
// Every element reaches every point exactly once: through the first level
// at which the element's box and the point's box stop touching, or, if they
// touch down to the deepest level, directly.  The sums use the 3-point rule
// for every element, as the direct evaluation does, so the two differ only
// by the expansions' truncation.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "../../include/bemfmm.h"
#include "kernel_math.h"
#include "plan.h"
#include "wavefun.h"

namespace bemfmm {

#define ARENA_ALLOC(arena, ptr, count)                                              \
  do {                                                                              \
    int _r = (arena).alloc((void**)&(ptr), sizeof(*(ptr)) * (size_t)(count));      \
    if (_r) return _r;                                                              \
  } while (0)

namespace {

constexpr double INV4PI_PT = 0.07957747154594767;
constexpr int PT_CHUNK = 64;  // points per workgroup (one wave)

// ---------------------------------------------------------------------------
// host: the point octree
// ---------------------------------------------------------------------------
uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffff;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}
uint32_t compact3h(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x | (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x | (x >> 4)) & 0x100f00f00f00f00full;
  x = (x | (x >> 8)) & 0x1f0000ff0000ffull;
  x = (x | (x >> 16)) & 0x1f00000000ffffull;
  x = (x | (x >> 32)) & 0x1fffff;
  return (uint32_t)x;
}
// Morton key with x on bit 3b+2, y on 3b+1, z on 3b (the problem's layout)
uint64_t morton(uint32_t x, uint32_t y, uint32_t z) {
  return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}
int floor_half(int a) { return a >= 0 ? a / 2 : -((1 - a) / 2); }

struct PBox {
  uint64_t key;   // point key of this level (shifted coordinates)
  int pt0, pt1;   // sorted points
  int parent;
  bool refined;
  int c[3];       // coordinates on the problem's grid of this level (may be < 0)
};

// source boxes of one level, by their coordinates
struct SourceLevel {
  int side = 0;
  std::unordered_map<uint64_t, int> at;
  std::vector<std::array<int, 3>> coord;
  int find(int x, int y, int z) const {
    if (x < 0 || y < 0 || z < 0 || x >= side || y >= side || z >= side) return -1;
    auto it = at.find(morton((uint32_t)x, (uint32_t)y, (uint32_t)z));
    return it == at.end() ? -1 : it->second;
  }
};

int cheb(const int* a, const int* b) {
  return std::max(std::abs(a[0] - b[0]), std::max(std::abs(a[1] - b[1]), std::abs(a[2] - b[2])));
}
int pt_code(int dx, int dy, int dz) {
  return ((dx + PT_OFF) * PT_W + (dy + PT_OFF)) * PT_W + (dz + PT_OFF);
}

// ---------------------------------------------------------------------------
// device: local expansions at the points (L2P), value and gradient
// ---------------------------------------------------------------------------
// phi(x) = sum_nm Lt_n^m R_n^m(x - c) with Lt = L~ / f_n (the stored locals
// of the point box, level scaling removed), and
//   d.grad R_n^m = sum_{sg, mu} gc[(cidx(n,m)*2 + sg)*3 + mu+1] c_mu(d) R_{n'}^{m-mu},
// n' = n + 1 (sg = 1) or n - 1 (sg = 0).  Collected per wave function
// R_{n'}^{m'} (n' <= p + 1) as A_mu = sum_sg Lt_n^{m'+mu} gc(...), the
// gradient is sum R_{n'}^{m'} B_a(n', m') with
//   B_x = c (A_-1 - A_+1),  B_y = -i c (A_+1 + A_-1),  B_z = c0 A_0,
//   c = sqrt(3/(8 pi)), c0 = sqrt(3/(4 pi)).
// Each workgroup (one chunk of a leaf's points; one launch per level, so
// that LDS is sized by that level's order) first forms the four coefficient
// arrays (value: Lt; B_x, B_y, B_z) and the Legendre recurrence
// coefficients in LDS, then every lane generates the wave functions of its
// point in m-major order by the normalised Legendre recurrences
// (Condon-Shortley phase), j_n in LDS per lane, and reads the coefficients
// with wave-uniform (broadcast) LDS loads.  Arithmetic type T: float64 for
// the float64 evaluation, float32 for the float32 one.
__host__ __device__ inline int cidx_pt(int n, int m) { return n * n + n + m; }

// LDS of the L2P kernel for expansion order p and jn_top tabulated Bessel
// recurrence reciprocals: j_n per lane, the reciprocals, the Legendre
// recurrence coefficients a, b per (n, m >= 0), the four coefficient arrays
template <typename T>
__host__ __device__ inline size_t l2p_lds_bytes(int p, int jn_top) {
  return sizeof(T) * ((size_t)(p + 2) * PT_CHUNK + jn_top + 2 * (p + 2) * (p + 2)) +
         sizeof(cplx<T>) * 4 * (p + 2) * (p + 2);
}

// j_n(x), n = 0..nmax, into out[n * stride] by the downward (Miller)
// recurrence of sph_jn, with 1/((2n+1)(2n+3)) from the table inv for
// n < ninv
template <typename T>
__device__ inline void jn_tab(int nmax, T x, T* out, int stride, const T* __restrict__ inv,
                              int ninv) {
  if (x == T(0)) {
    out[0] = T(1);
    for (int nn = 1; nn <= nmax; ++nn) out[nn * stride] = T(0);
    return;
  }
  const int top = nmax + 24 + (int)(T(1.5) * x);
  const T x2 = x * x;
  T jp1 = T(1) - x2 / (T(2) * (2 * top + 5)), jn = T(1) - x2 / (T(2) * (2 * top + 3));
  for (int nn = top; nn >= 1; --nn) {
    const T rc = nn < ninv ? inv[nn] : T(1) / ((T(2) * nn + T(1)) * (T(2) * nn + T(3)));
    const T jm1 = jn - jp1 * x2 * rc;
    jp1 = jn;
    jn = jm1;
    if (nn - 1 <= nmax) out[(nn - 1) * stride] = jm1;
  }
  const T sn = sin(x), cs = cos(x);
  const T j0 = (fabs(x) < T(1e-4)) ? T(1) - x2 / T(6) + x2 * x2 / T(120) : sn / x;
  T scale;
  if (nmax >= 1 && fabs(x) > T(1)) {
    const T j1 = (sn / x - cs) / x;
    scale = (fabs(j0) >= fabs(j1)) ? j0 / out[0] : j1 / (out[stride] * x / T(3));
  } else {
    scale = j0 / out[0];
  }
  T fct = T(1);  // x^n / (2n+1)!!
  for (int nn = 0; nn <= nmax; ++nn) {
    if (nn > 0) fct *= x / (T(2) * nn + T(1));
    out[nn * stride] *= scale * fct;
  }
}

template <typename R, typename T>
__global__ void __launch_bounds__(PT_CHUNK)
    k_points_l2p(const cplx<R>* __restrict__ Lc, int p, int jn_top, int chunk0,
                 const int* __restrict__ chunk_leaf, const int* __restrict__ chunk_pt,
                 const int* __restrict__ chunk_cnt, const int* __restrict__ leaf_box,
                 const double* __restrict__ leaf_c, const double* __restrict__ xyz, int64_t n,
                 double k, const double* __restrict__ fi, const double* __restrict__ gc,
                 c64* __restrict__ acc) {
  extern __shared__ double pt_lds[];
  const int chunk = chunk0 + blockIdx.x, t = threadIdx.x;
  const int leaf = chunk_leaf[chunk];
  const int ncoef = (p + 1) * (p + 1), P2 = (p + 2) * (p + 2);
  const cplx<R>* __restrict__ Lb = Lc + (int64_t)leaf_box[leaf] * ncoef;
  T* s_j = (T*)pt_lds;
  T* s_inv = s_j + (p + 2) * PT_CHUNK;
  T* s_a = s_inv + jn_top;
  T* s_b = s_a + P2;
  cplx<T>* sB = (cplx<T>*)(s_b + P2);
  for (int c = t; c < jn_top; c += PT_CHUNK)
    s_inv[c] = (T)(1.0 / ((2.0 * c + 1.0) * (2.0 * c + 3.0)));
  constexpr double C1 = 0.3454941494713355, C0 = 0.4886025119029199;
  auto Lt = [&](int nn, int m) -> c64 {
    const cplx<R> v = Lb[cidx_pt(nn, m)];
    return mk((double)v.re * fi[nn], (double)v.im * fi[nn]);
  };
  for (int c = t; c < P2; c += PT_CHUNK) {
    int n2 = (int)sqrt((double)c);
    while (n2 * n2 > c) --n2;
    while ((n2 + 1) * (n2 + 1) <= c) ++n2;
    const int m2 = c - n2 * n2 - n2;
    c64 A[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
    for (int mu = -1; mu <= 1; ++mu) {
      const int ms = m2 + mu;
      for (int sg = 0; sg < 2; ++sg) {
        const int nn = sg ? n2 - 1 : n2 + 1;
        if (nn < 0 || nn > p || abs(ms) > nn) continue;
        const double* g = gc + ((int64_t)(cidx_pt(nn, ms) * 2 + sg) * 3 + (mu + 1)) * 2;
        cfma(A[mu + 1], Lt(nn, ms), mk(g[0], g[1]));
      }
    }
    const c64 s2 = cadd(A[2], A[0]);
    const c64 v0 = n2 <= p ? Lt(n2, m2) : mk(0.0, 0.0);
    const c64 v1 = cscale(csub(A[0], A[2]), C1);      // c (A_-1 - A_+1)
    const c64 v2 = mk(C1 * s2.im, -C1 * s2.re);       // -i c (A_+1 + A_-1)
    const c64 v3 = cscale(A[1], C0);
    sB[c] = mk<T>((T)v0.re, (T)v0.im);
    sB[P2 + c] = mk<T>((T)v1.re, (T)v1.im);
    sB[2 * P2 + c] = mk<T>((T)v2.re, (T)v2.im);
    sB[3 * P2 + c] = mk<T>((T)v3.re, (T)v3.im);
    // Legendre recurrence coefficients of (n2, m2 >= 0), n2 >= m2 + 2
    if (m2 >= 0 && n2 >= m2 + 2) {
      s_a[c] = (T)sqrt((4.0 * n2 * n2 - 1.0) / ((double)n2 * n2 - (double)m2 * m2));
      s_b[c] = (T)sqrt(((n2 - 1.0) * (n2 - 1.0) - (double)m2 * m2) /
                       (4.0 * (n2 - 1.0) * (n2 - 1.0) - 1.0));
    }
  }
  __syncthreads();
  const bool active = t < chunk_cnt[chunk];
  const int64_t i = chunk_pt[chunk] + t;
  T vx = T(1), vy = T(0), vz = T(0);
  if (active) {
    vx = (T)(xyz[i] - leaf_c[3 * leaf]);
    vy = (T)(xyz[n + i] - leaf_c[3 * leaf + 1]);
    vz = (T)(xyz[2 * n + i] - leaf_c[3 * leaf + 2]);
  }
  const T r = sqrt(vx * vx + vy * vy + vz * vz);
  const T ct = r > T(0) ? vz / r : T(1);
  const T st = sqrt(fmax(T(0), T(1) - ct * ct));
  const T rxy = sqrt(vx * vx + vy * vy);
  const T cp = rxy > T(0) ? vx / rxy : T(1), sp = rxy > T(0) ? vy / rxy : T(0);
  jn_tab<T>(p + 1, (T)k * r, s_j + t, PT_CHUNK, s_inv, jn_top);
  cplx<T> f = mk<T>(0, 0), gx = mk<T>(0, 0), gy = mk<T>(0, 0), gz = mk<T>(0, 0);
  auto add = [&](int c, cplx<T> Rv) {
    cfma(f, sB[c], Rv);
    cfma(gx, sB[P2 + c], Rv);
    cfma(gy, sB[2 * P2 + c], Rv);
    cfma(gz, sB[3 * P2 + c], Rv);
  };
  T tmm = T(0.28209479177387814);  // 1/sqrt(4 pi)
  T er = T(1), ei = T(0);          // exp(i m phi)
  for (int m = 0; m <= p + 1; ++m) {
    if (m > 0) {
      const T tr = er * cp - ei * sp;
      ei = er * sp + ei * cp;
      er = tr;
      tmm = -sqrt((T(2) * m + T(1)) / (T(2) * m)) * st * tmm;
    }
    const T sgn = (m & 1) ? T(-1) : T(1);
    T t0 = T(0), t1 = tmm;
    for (int nn = m; nn <= p + 1; ++nn) {
      T th;
      if (nn == m) {
        th = tmm;
      } else if (nn == m + 1) {
        th = sqrt(T(2) * m + T(3)) * ct * tmm;
        t0 = tmm;
        t1 = th;
      } else {
        const int c = cidx_pt(nn, m);
        th = s_a[c] * (ct * t1 - s_b[c] * t0);
        t0 = t1;
        t1 = th;
      }
      const T jt = s_j[nn * PT_CHUNK + t] * th;
      add(cidx_pt(nn, m), mk<T>(jt * er, jt * ei));
      // R_n^-m = (-1)^m conj(R_n^m) (j_n real)
      if (m > 0) add(cidx_pt(nn, -m), mk<T>(sgn * jt * er, -sgn * jt * ei));
    }
  }
  if (active) {
    acc[4 * i] = mk((double)f.re, (double)f.im);
    acc[4 * i + 1] = mk((double)gx.re, (double)gx.im);
    acc[4 * i + 2] = mk((double)gy.re, (double)gy.im);
    acc[4 * i + 3] = mk((double)gz.re, (double)gz.im);
  }
}

// ---------------------------------------------------------------------------
// device: direct sums over the touching source leaves (P2P)
// ---------------------------------------------------------------------------
// phi_near(x) = sum_j w_j sum_q [G(x - y_jq) q_j - dG/dn_y(x - y_jq) p_j] and its
// gradient, w_j = A_j / (3 * 4 pi); with rv = x - y, u = 1/|rv|,
// G' = G (ik - u), G'' = G ((ik - u)^2 + u^2):
//   grad G = G' u rv,  grad dG/dn_y = -(G'' - G' u)(rv.n_y) u^2 rv - G' u n_y.
// One wave per chunk of a leaf's points: lane = point * S + slice, the S
// slices of a point split the elements and are summed by lane shuffles.
// The elements of the touching leaves are staged through LDS in batches of
// 64 (one per lane, coalesced loads; rule points, normal, the densities
// with their weight folded in), then read back as broadcasts.
template <typename R>
__device__ __forceinline__ R wave_sum(R v, int S) {
  for (int o = S >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

constexpr int PT_MAX_NEAR = 27;  // touching leaves of a point leaf

template <typename R>
__global__ void __launch_bounds__(PT_CHUNK)
    k_points_p2p(const int* __restrict__ near_pt, const int* __restrict__ near_cnt,
                 const int* __restrict__ near_s0, const int* __restrict__ near_s1,
                 const int* __restrict__ near_src, const int* __restrict__ bstart,
                 const R* __restrict__ geo, int64_t ne, const cplx<R>* __restrict__ ps,
                 const cplx<R>* __restrict__ qs, const double* __restrict__ xyz, int64_t n,
                 R k, R k_turns, c64* __restrict__ acc) {
  __shared__ int s_pref[PT_MAX_NEAR + 1], s_first[PT_MAX_NEAR];
  __shared__ R s_y[9][PT_CHUNK], s_n[3][PT_CHUNK], s_d[4][PT_CHUNK];
  const int c = blockIdx.x, lane = threadIdx.x;
  const int cnt = near_cnt[c];
  const int j0 = near_s0[c], nl = near_s1[c] - j0;
  // prefix counts of the touching leaves' element ranges
  if (lane < nl) {
    const int sleaf = near_src[j0 + lane];
    s_first[lane] = bstart[sleaf];
    s_pref[lane + 1] = bstart[sleaf + 1] - bstart[sleaf];
  }
  if (lane == 0) s_pref[0] = 0;
  __syncthreads();
  if (lane == 0)
    for (int j = 1; j <= nl; ++j) s_pref[j] += s_pref[j - 1];
  __syncthreads();
  const int total = s_pref[nl];
  int S = 1;
  while (S * 2 * cnt <= PT_CHUNK) S *= 2;
  const int ip = lane / S, sl = lane % S;
  const bool active = ip < cnt;
  const int64_t i = near_pt[c] + (active ? ip : 0);
  const R x0 = (R)xyz[i], x1 = (R)xyz[n + i], x2 = (R)xyz[2 * n + i];
  R fr = 0, fi = 0, g0r = 0, g0i = 0, g1r = 0, g1i = 0, g2r = 0, g2i = 0;
  for (int b0 = 0; b0 < total; b0 += PT_CHUNK) {
    const int v = b0 + lane;
    if (v < total) {
      int j = 0;
      while (j + 1 < nl && s_pref[j + 1] <= v) ++j;
      const int64_t e = s_first[j] + (v - s_pref[j]);
      for (int q = 0; q < 9; ++q) s_y[q][lane] = geo[(GEO_QX0 + q) * ne + e];
      s_n[0][lane] = geo[GEO_NX * ne + e];
      s_n[1][lane] = geo[GEO_NY * ne + e];
      s_n[2][lane] = geo[GEO_NZ * ne + e];
      const R w = geo[GEO_AREA * ne + e] * R(INV4PI_PT / 3.0);
      const cplx<R> pv = ps[e], qv = qs[e];
      s_d[0][lane] = pv.re * w;
      s_d[1][lane] = pv.im * w;
      s_d[2][lane] = qv.re * w;
      s_d[3][lane] = qv.im * w;
    }
    __syncthreads();
    const int nb = min(PT_CHUNK, total - b0);
    if (active) {
      for (int u = sl; u < nb; u += S) {
        const R pr = s_d[0][u], pi = s_d[1][u], qr = s_d[2][u], qi = s_d[3][u];
        const R ny0 = s_n[0][u], ny1 = s_n[1][u], ny2 = s_n[2][u];
#pragma unroll
        for (int qq = 0; qq < 3; ++qq) {
          const R r0 = x0 - s_y[3 * qq][u];
          const R r1 = x1 - s_y[3 * qq + 1][u];
          const R r2 = x2 - s_y[3 * qq + 2][u];
          const R rr = r0 * r0 + r1 * r1 + r2 * r2;
          const R uu = rsqrt_r<R>(rr);
          R sn, cs;
          phase<R>(rr * uu, k, k_turns, &sn, &cs);
          const R Gr = cs * uu, Gi = sn * uu;
          // G' = G (ik - u), G'' = G ((ik - u)^2 + u^2) = G (2 u^2 - k^2 - 2 i k u)
          const R G1r = -Gr * uu - Gi * k, G1i = Gr * k - Gi * uu;
          const R ar = R(2) * uu * uu - k * k, ai = R(-2) * k * uu;
          const R G2r = Gr * ar - Gi * ai, G2i = Gr * ai + Gi * ar;
          const R rny = r0 * ny0 + r1 * ny1 + r2 * ny2;
          // dG/dn_y = -G' u rny
          const R Gyr = -G1r * uu * rny, Gyi = -G1i * uu * rny;
          // phi: G q - G_y p
          fr += Gr * qr - Gi * qi - (Gyr * pr - Gyi * pi);
          fi += Gr * qi + Gi * qr - (Gyr * pi + Gyi * pr);
          // grad: coefficient of rv: G' u q + (G'' - G' u) rny u^2 p; of n_y: G' u p
          const R h = rny * uu * uu;
          const R dr = (G2r - G1r * uu) * h, di = (G2i - G1i * uu) * h;
          const R a1r = G1r * uu, a1i = G1i * uu;  // G' u
          const R crv_r = a1r * qr - a1i * qi + dr * pr - di * pi;
          const R crv_i = a1r * qi + a1i * qr + dr * pi + di * pr;
          const R cn_r = a1r * pr - a1i * pi, cn_i = a1r * pi + a1i * pr;
          g0r += crv_r * r0 + cn_r * ny0;
          g0i += crv_i * r0 + cn_i * ny0;
          g1r += crv_r * r1 + cn_r * ny1;
          g1i += crv_i * r1 + cn_i * ny1;
          g2r += crv_r * r2 + cn_r * ny2;
          g2i += crv_i * r2 + cn_i * ny2;
        }
      }
    }
    __syncthreads();
  }
  fr = wave_sum(fr, S);
  fi = wave_sum(fi, S);
  g0r = wave_sum(g0r, S);
  g0i = wave_sum(g0i, S);
  g1r = wave_sum(g1r, S);
  g1i = wave_sum(g1i, S);
  g2r = wave_sum(g2r, S);
  g2i = wave_sum(g2i, S);
  if (active && sl == 0) {
    acc[4 * i] = mk((double)fr, (double)fi);
    acc[4 * i + 1] = mk((double)g0r, (double)g0i);
    acc[4 * i + 2] = mk((double)g1r, (double)g1i);
    acc[4 * i + 3] = mk((double)g2r, (double)g2i);
  }
}

// total field = incident part - phi (the representation's boundary sums are
// -phi: phi = S q - K p, far part in acc, direct part in acc_near where
// near_flag is set), written in the caller's point order
__global__ void k_points_finish(const double* __restrict__ xyz, const int* __restrict__ perm,
                                int64_t n, const c64* __restrict__ acc,
                                const c64* __restrict__ acc_near,
                                const uint8_t* __restrict__ near_flag, double k, int has_pw,
                                double dx, double dy, double dz, const double* __restrict__ src,
                                const c64* __restrict__ amp, int nsrc, c64* __restrict__ out,
                                c64* __restrict__ grad) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x0 = xyz[i], x1 = xyz[n + i], x2 = xyz[2 * n + i];
  c64 a0 = acc[4 * i], a1 = acc[4 * i + 1], a2 = acc[4 * i + 2], a3 = acc[4 * i + 3];
  if (near_flag[i]) {
    a0 = cadd(a0, acc_near[4 * i]);
    a1 = cadd(a1, acc_near[4 * i + 1]);
    a2 = cadd(a2, acc_near[4 * i + 2]);
    a3 = cadd(a3, acc_near[4 * i + 3]);
  }
  c64 f = cscale(a0, -1.0), f0 = cscale(a1, -1.0), f1 = cscale(a2, -1.0), f2 = cscale(a3, -1.0);
  if (has_pw) {
    double sn, cs;
    sincos(k * (dx * x0 + dy * x1 + dz * x2), &sn, &cs);
    const c64 ike = mk(-k * sn, k * cs);
    f = cadd(f, mk(cs, sn));
    f0 = cadd(f0, cscale(ike, dx));
    f1 = cadd(f1, cscale(ike, dy));
    f2 = cadd(f2, cscale(ike, dz));
  }
  for (int m = 0; m < nsrc; ++m) {
    const double r0 = x0 - src[3 * m], r1 = x1 - src[3 * m + 1], r2 = x2 - src[3 * m + 2];
    const double r = sqrt(r0 * r0 + r1 * r1 + r2 * r2), u = 1.0 / r;
    double sn, cs;
    sincos(k * r, &sn, &cs);
    const c64 G = cmul(mk(cs * u * INV4PI_PT, sn * u * INV4PI_PT), amp[m]);
    const c64 g1u = cscale(cmul(G, mk(-u, k)), u);  // A G' / r
    f = cadd(f, G);
    f0 = cadd(f0, cscale(g1u, r0));
    f1 = cadd(f1, cscale(g1u, r1));
    f2 = cadd(f2, cscale(g1u, r2));
  }
  const int o = perm[i];
  out[o] = f;
  if (grad) {
    grad[3 * o] = f0;
    grad[3 * o + 1] = f1;
    grad[3 * o + 2] = f2;
  }
}

template <typename R>
PrecisionData<R>& pdata(Problem& P);
template <>
PrecisionData<float>& pdata<float>(Problem& P) {
  return P.f32;
}
template <>
PrecisionData<double>& pdata<double>(Problem& P) {
  return P.f64;
}
template <typename R>
PointOps<R>& pops(FieldPoints& F);
template <>
PointOps<float>& pops<float>(FieldPoints& F) {
  return F.f32;
}
template <>
PointOps<double>& pops<double>(FieldPoints& F) {
  return F.f64;
}

}  // namespace

// ---------------------------------------------------------------------------
// host: create
// ---------------------------------------------------------------------------
template <typename R>
static int build_points_precision(Problem& P, const PointLists& lists, FieldPoints& F,
                                  hipStream_t s) {
  PrecisionData<R>& D = pdata<R>(P);
  int r = build_point_ops<R>(P, D, lists, F, pops<R>(F), s);
  if (!r) r = build_point_rotations<R>(P, D, F, pops<R>(F), s);
  if (r) return r;
  int pmax = 0;
  for (int l = 2; l <= F.L; ++l) pmax = std::max(pmax, D.order[l]);
  F.max_order = pmax;
  // 1 / f_n per level, f_n = (k h_l)^n / (2n+1)!!
  std::vector<double> finv((size_t)(MAX_LEVEL + 1) * (MAXP_PT + 1), 0.0);
  for (int l = 2; l <= F.L; ++l) {
    double v = 1.0;
    for (int nn = 0; nn <= D.order[l]; ++nn) {
      if (nn > 0) v *= P.k * P.h[l] / (2.0 * nn + 1.0);
      finv[(size_t)l * (MAXP_PT + 1) + nn] = 1.0 / v;
    }
  }
  ARENA_ALLOC(F.arena, F.finv, finv.size());
  BEM_HIP_TRY(hipMemcpyAsync(F.finv, finv.data(), sizeof(double) * finv.size(),
                             hipMemcpyHostToDevice, s));
  DevArena scratch;
  std::vector<double> gc;
  r = derivative_table(P, pmax, gc, scratch, s);
  scratch.release();
  if (r) return r;
  ARENA_ALLOC(F.arena, F.gcoef, gc.size());
  BEM_HIP_TRY(hipMemcpyAsync(F.gcoef, gc.data(), sizeof(double) * gc.size(),
                             hipMemcpyHostToDevice, s));
  BEM_HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

static int build_point_tree(Problem& P, const double* pts, FieldPoints& F, PointLists& lists,
                            hipStream_t s) {
  const int L = P.L;
  const int64_t n = F.n;
  if (L + 3 > NBITS) {
    set_error("tree too deep for the point octree");
    return BEM_E_INVALID;
  }
  // ---- source boxes of every level (host copies of the problem's tree) ----
  std::vector<SourceLevel> src(L + 1);
  for (int l = 2; l <= L; ++l) {
    std::vector<uint64_t> keys(P.nbox[l]);
    if (P.nbox[l] > 0)
      BEM_HIP_TRY(hipMemcpyAsync(keys.data(), P.box_keys[l], sizeof(uint64_t) * keys.size(),
                                 hipMemcpyDeviceToHost, s));
    BEM_HIP_TRY(hipStreamSynchronize(s));
    src[l].side = 1 << l;
    src[l].coord.resize(keys.size());
    for (size_t b = 0; b < keys.size(); ++b) {
      src[l].at[keys[b]] = (int)b;
      src[l].coord[b] = {(int)compact3h(keys[b] >> 2), (int)compact3h(keys[b] >> 1),
                         (int)compact3h(keys[b])};
    }
  }
  std::vector<int> bstart(P.nbox[L] + 1);
  BEM_HIP_TRY(hipMemcpyAsync(bstart.data(), P.box_start[L], sizeof(int) * bstart.size(),
                             hipMemcpyDeviceToHost, s));
  BEM_HIP_TRY(hipStreamSynchronize(s));
  // ---- point keys: level-L coordinates shifted by PT_EXT level-2 boxes ----
  const int64_t shift = (int64_t)PT_EXT << (L - 2);
  const int64_t side = (int64_t)(4 + 2 * PT_EXT) << (L - 2);
  std::vector<uint64_t> key(n);
  for (int64_t i = 0; i < n; ++i) {
    uint32_t u[3];
    for (int a = 0; a < 3; ++a) {
      const double f = (pts[3 * i + a] - P.lo[a]) / P.h[L];
      if (!std::isfinite(f)) {
        set_error("evaluation point " + std::to_string(i) + " is not finite");
        return BEM_E_INVALID;
      }
      const double fl = std::floor(f);
      if (fl < -(double)shift || fl >= (double)(side - shift)) {
        set_error("evaluation point " + std::to_string(i) +
                  " lies farther than two root-cube widths from the tree's root cube");
        return BEM_E_INVALID;
      }
      u[a] = (uint32_t)((int64_t)fl + shift);
    }
    key[i] = morton(u[0], u[1], u[2]);
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
  std::vector<uint64_t> skey(n);
  std::vector<double> xyz(3 * n);
  for (int64_t i = 0; i < n; ++i) {
    skey[i] = key[order[i]];
    for (int a = 0; a < 3; ++a) xyz[a * n + i] = pts[3 * (int64_t)order[i] + a];
  }
  // ---- point boxes, top down ----
  std::vector<std::vector<PBox>> T(L + 1);
  auto group = [&](int l, int a, int b, int parent) {
    const int sh = 3 * (L - l);
    const int off = PT_EXT << (l - 2);
    for (int i = a; i < b;) {
      const uint64_t k = skey[i] >> sh;
      int j = i + 1;
      while (j < b && (skey[j] >> sh) == k) ++j;
      PBox B;
      B.key = k;
      B.pt0 = i;
      B.pt1 = j;
      B.parent = parent;
      B.refined = false;
      B.c[0] = (int)compact3h(k >> 2) - off;
      B.c[1] = (int)compact3h(k >> 1) - off;
      B.c[2] = (int)compact3h(k) - off;
      T[l].push_back(B);
      i = j;
    }
  };
  group(2, 0, (int)n, -1);
  for (int l = 2; l <= L; ++l) {
    for (size_t b = 0; b < T[l].size(); ++b) {
      PBox& B = T[l][b];
      if (l < L) {
        for (int d = 0; d < 27 && !B.refined; ++d)
          B.refined = src[l].find(B.c[0] + d / 9 - 1, B.c[1] + (d / 3) % 3 - 1, B.c[2] + d % 3 - 1) >= 0;
      }
      if (B.refined) group(l + 1, B.pt0, B.pt1, (int)b);
    }
    F.nbox[l] = (int)T[l].size();
  }
  // ---- translation lists ----
  for (int l = 2; l <= L; ++l) {
    auto& md = lists.m2l_dst[l];
    auto& ms = lists.m2l_src[l];
    auto& mc = lists.m2l_code[l];
    for (size_t t = 0; t < T[l].size(); ++t) {
      const PBox& B = T[l][t];
      if (l == 2) {
        for (size_t sb = 0; sb < src[2].coord.size(); ++sb) {
          const int* c = src[2].coord[sb].data();
          if (cheb(B.c, c) < 2) continue;
          md.push_back((int)t);
          ms.push_back((int)sb);
          mc.push_back(pt_code(B.c[0] - c[0], B.c[1] - c[1], B.c[2] - c[2]));
        }
        continue;
      }
      const int pc[3] = {floor_half(B.c[0]), floor_half(B.c[1]), floor_half(B.c[2])};
      for (int d = 0; d < 27; ++d) {
        const int q[3] = {pc[0] + d / 9 - 1, pc[1] + (d / 3) % 3 - 1, pc[2] + d % 3 - 1};
        if (src[l - 1].find(q[0], q[1], q[2]) < 0) continue;
        for (int ch = 0; ch < 8; ++ch) {
          const int c[3] = {2 * q[0] + ((ch >> 2) & 1), 2 * q[1] + ((ch >> 1) & 1),
                            2 * q[2] + (ch & 1)};
          const int si = src[l].find(c[0], c[1], c[2]);
          if (si < 0 || cheb(B.c, c) < 2) continue;
          md.push_back((int)t);
          ms.push_back(si);
          mc.push_back(pt_code(B.c[0] - c[0], B.c[1] - c[1], B.c[2] - c[2]));
        }
      }
      lists.l2l_dst[l].push_back((int)t);
      lists.l2l_src[l].push_back(B.parent);
      lists.l2l_code[l].push_back((int)(B.key & 7));
    }
  }
  // ---- leaves in point order, chunks, near lists ----
  struct Leaf {
    int pt0, pt1, level, box;
  };
  std::vector<Leaf> leaves;
  for (int l = 2; l <= L; ++l)
    for (size_t b = 0; b < T[l].size(); ++b)
      if (!T[l][b].refined) leaves.push_back({T[l][b].pt0, T[l][b].pt1, l, (int)b});
  std::sort(leaves.begin(), leaves.end(), [](const Leaf& a, const Leaf& b) { return a.pt0 < b.pt0; });
  int64_t covered = 0;
  for (const Leaf& lf : leaves) {
    if (lf.pt0 != covered) {
      set_error("internal: point leaves do not partition the points");
      return BEM_E_INVALID;
    }
    covered = lf.pt1;
  }
  if (covered != n) {
    set_error("internal: point leaves do not cover the points");
    return BEM_E_INVALID;
  }
  std::vector<int> lb, cl, cpt, ccnt, npt, ncnt, ns0, ns1, nsrc;
  std::vector<std::vector<std::array<int, 3>>> lchunks(L + 1);  // (leaf, first point, count)
  std::vector<double> lc;
  int64_t near_pairs = 0;
  for (size_t q = 0; q < leaves.size(); ++q) {
    const Leaf& lf = leaves[q];
    const PBox& B = T[lf.level][lf.box];
    lb.push_back(lf.box);
    for (int a = 0; a < 3; ++a) lc.push_back(P.lo[a] + (B.c[a] + 0.5) * P.h[lf.level]);
    for (int a = lf.pt0; a < lf.pt1; a += PT_CHUNK)
      lchunks[lf.level].push_back({(int)q, a, std::min(PT_CHUNK, lf.pt1 - a)});
    if (lf.level != L) continue;
    const int s0 = (int)nsrc.size();
    int64_t nel = 0;
    for (int d = 0; d < 27; ++d) {
      const int si = src[L].find(B.c[0] + d / 9 - 1, B.c[1] + (d / 3) % 3 - 1, B.c[2] + d % 3 - 1);
      if (si < 0) continue;
      nsrc.push_back(si);
      nel += bstart[si + 1] - bstart[si];
    }
    if ((int)nsrc.size() == s0) continue;
    near_pairs += nel * (lf.pt1 - lf.pt0);
    for (int a = lf.pt0; a < lf.pt1; a += PT_CHUNK) {
      npt.push_back(a);
      ncnt.push_back(std::min(PT_CHUNK, lf.pt1 - a));
      ns0.push_back(s0);
      ns1.push_back((int)nsrc.size());
    }
  }
  // far-field chunks grouped by level (one launch per level)
  F.chunk_off.fill(0);
  for (int l = 2; l <= L; ++l) {
    F.chunk_off[l] = (int)cl.size();
    for (const auto& c : lchunks[l]) {
      cl.push_back(c[0]);
      cpt.push_back(c[1]);
      ccnt.push_back(c[2]);
    }
  }
  F.chunk_off[L + 1] = (int)cl.size();
  F.n_leaf = (int)leaves.size();
  F.n_chunk = (int)cl.size();
  F.n_near_chunk = (int)npt.size();
  F.n_near_pairs = near_pairs;
  auto up_i = [&](const std::vector<int>& h, int** d) -> int {
    ARENA_ALLOC(F.arena, *d, std::max<size_t>(1, h.size()));
    if (!h.empty())
      BEM_HIP_TRY(hipMemcpyAsync(*d, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice, s));
    return 0;
  };
  int r = 0;
  if ((r = up_i(lb, &F.leaf_box)) || (r = up_i(cl, &F.chunk_leaf)) ||
      (r = up_i(cpt, &F.chunk_pt)) || (r = up_i(ccnt, &F.chunk_cnt)) || (r = up_i(npt, &F.near_pt)) ||
      (r = up_i(ncnt, &F.near_cnt)) || (r = up_i(ns0, &F.near_s0)) || (r = up_i(ns1, &F.near_s1)) ||
      (r = up_i(nsrc, &F.near_src)) || (r = up_i(order, &F.perm)))
    return r;
  ARENA_ALLOC(F.arena, F.leaf_c, std::max<size_t>(1, lc.size()));
  if (!lc.empty())
    BEM_HIP_TRY(hipMemcpyAsync(F.leaf_c, lc.data(), sizeof(double) * lc.size(),
                               hipMemcpyHostToDevice, s));
  ARENA_ALLOC(F.arena, F.xyz, std::max<int64_t>(1, 3 * n));
  if (n > 0)
    BEM_HIP_TRY(hipMemcpyAsync(F.xyz, xyz.data(), sizeof(double) * xyz.size(),
                               hipMemcpyHostToDevice, s));
  ARENA_ALLOC(F.arena, F.acc, std::max<int64_t>(1, 4 * n));
  ARENA_ALLOC(F.arena, F.acc_near, std::max<int64_t>(1, 4 * n));
  std::vector<uint8_t> flag(std::max<int64_t>(1, n), 0);
  for (size_t c = 0; c < npt.size(); ++c)
    for (int a = 0; a < ncnt[c]; ++a) flag[npt[c] + a] = 1;
  ARENA_ALLOC(F.arena, F.near_flag, flag.size());
  BEM_HIP_TRY(hipMemcpyAsync(F.near_flag, flag.data(), flag.size(), hipMemcpyHostToDevice, s));
  BEM_HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

int field_points_create(Problem& P, int prec, const double* pts, int64_t n, FieldPoints** out,
                        hipStream_t s) {
  if (prec != 0 && prec != 1) {
    set_error("evaluation points: precision must be float64 or float32 (no refinement)");
    return BEM_E_INVALID;
  }
  if (n < 0 || (n > 0 && !pts) || n > (int64_t)1 << 30) {
    set_error("evaluation points: bad point count or pointer");
    return BEM_E_INVALID;
  }
  FieldPoints* F = new FieldPoints();
  F->P = &P;
  F->prec = prec;
  F->n = n;
  F->L = P.L;
  int r = 0;
  if (P.direct || P.L < 2) {
    // no far field in this problem: the points are kept in caller order
    // for the direct sum
    ARENA_ALLOC(F->arena, F->xyz, std::max<int64_t>(1, 3 * n));
    if (n > 0) {
      r = hipMemcpyAsync(F->xyz, pts, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s) != hipSuccess
              ? BEM_E_HIP
              : 0;
      if (!r && hipStreamSynchronize(s) != hipSuccess) r = BEM_E_HIP;
    }
  } else {
    PointLists lists;
    r = build_point_tree(P, pts, *F, lists, s);
    if (!r)
      r = prec == 0 ? build_points_precision<double>(P, lists, *F, s)
                    : build_points_precision<float>(P, lists, *F, s);
  }
  if (r) {
    if (r == BEM_E_HIP) set_error("HIP error while building the evaluation points");
    field_points_destroy(F);
    return r;
  }
  *out = F;
  return 0;
}

void field_points_destroy(FieldPoints* F) {
  if (!F) return;
  F->arena.release();
  delete F;
}

template <typename R>
static int eval_points(FieldPoints& F, const c64* p, const c64* q, c64* acc, hipStream_t s) {
  Problem& P = *F.P;
  PrecisionData<R>& D = pdata<R>(P);
  PointOps<R>& O = pops<R>(F);
  // the direct sums need only the gathered densities: on the problem's side
  // stream, concurrently with the far field (joined before the finish)
  const bool near = F.n_near_chunk > 0;
  int r = point_far_field<R>(P, D, F, O, p, q, s, near ? P.ev_fork : nullptr);
  if (r) return r;
  if (near) {
    BEM_HIP_TRY(hipStreamWaitEvent(P.side, P.ev_fork, 0));
    const R k = (R)P.k, k_turns = (R)(P.k / (2.0 * M_PI));
    const int ev = prof_begin(P, P.side);
    hipLaunchKernelGGL(k_points_p2p<R>, dim3(F.n_near_chunk), dim3(PT_CHUNK), 0, P.side,
                       F.near_pt, F.near_cnt, F.near_s0, F.near_s1, F.near_src,
                       P.box_start[P.L], D.geo, P.n, O.X.ps, O.X.qs, F.xyz, F.n, k, k_turns,
                       F.acc_near);
    BEM_LAUNCH_CHECK();
    if ((r = prof_end(P, ev, prof_slot(ST_PT_P2P, sizeof(R) == 4, false), P.side))) return r;
    BEM_HIP_TRY(hipEventRecord(P.ev_join, P.side));
  }
  // local expansions at the points, one launch per level (chunks grouped by
  // level, LDS sized by the level's order)
  typedef typename std::conditional<sizeof(R) == 4, float, double>::type T;
  const int ev = prof_begin(P, s);
  for (int l = 2; l <= F.L; ++l) {
    const int nc = F.chunk_off[l + 1] - F.chunk_off[l];
    if (nc <= 0) continue;
    const int p = D.order[l];
    // the recurrence starts at p + 25 + 1.5 k r, r <= sqrt(3)/2 h_l
    const int jn_top = std::min(p + 28 + (int)(1.5 * P.k * 0.87 * P.h[l]), 512);
    const size_t lds = l2p_lds_bytes<T>(p, jn_top);
    if (lds > 65536)
      BEM_HIP_TRY(hipFuncSetAttribute((const void*)k_points_l2p<R, T>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL((k_points_l2p<R, T>), dim3(nc), dim3(PT_CHUNK), lds, s, O.Lc[l], p,
                       jn_top, F.chunk_off[l], F.chunk_leaf, F.chunk_pt, F.chunk_cnt,
                       F.leaf_box, F.leaf_c, F.xyz, F.n, P.k, F.finv + l * (MAXP_PT + 1),
                       F.gcoef, acc);
    BEM_LAUNCH_CHECK();
  }
  if ((r = prof_end(P, ev, prof_slot(ST_PT_L2P, sizeof(R) == 4, false), s))) return r;
  if (near) BEM_HIP_TRY(hipStreamWaitEvent(s, P.ev_join, 0));
  return 0;
}

int eval_field_grad_fmm(FieldPoints& F, const c64* p, const c64* q, const double* d,
                        const double* src, const c64* amp, int n_src, c64* out, c64* grad,
                        hipStream_t s) {
  if (F.n == 0) return 0;
  Problem& P = *F.P;
  if (P.direct || P.L < 2)
    return eval_field_grad(P, p, q, F.xyz, (int)F.n, d, src, amp, n_src, out, grad, s);
  double dx = 0, dy = 0, dz = 0;
  if (d) {
    const double nrm = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (!(nrm > 0)) {
      set_error("zero incidence direction");
      return BEM_E_INVALID;
    }
    dx = d[0] / nrm;
    dy = d[1] / nrm;
    dz = d[2] / nrm;
  }
  int r = F.prec == 0 ? eval_points<double>(F, p, q, F.acc, s)
                      : eval_points<float>(F, p, q, F.acc, s);
  if (r) return r;
  hipLaunchKernelGGL(k_points_finish, dim3(ceil_div(F.n, 256)), dim3(256), 0, s, F.xyz, F.perm,
                     F.n, F.acc, F.acc_near, F.near_flag, P.k, d ? 1 : 0, dx, dy, dz, src, amp,
                     src ? n_src : 0, out, grad);
  BEM_LAUNCH_CHECK();
  return 0;
}

}  // namespace bemfmm
