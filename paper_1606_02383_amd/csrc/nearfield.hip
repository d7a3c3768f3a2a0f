// Near-field precompute: near-pair lists, accurate near-singular integrals,
// self (diagonal) terms, and the correction coefficients
//     C_ij = A^accurate_ij - A^3-point_ij
// that turn the 3-point-rule direct sum into the exact discrete operator.
//
// Kernel (paper Sec. 2.3): G = exp(ikr)/(4 pi r); with rv = x - y,
// G' = G(ik - 1/r), G'' = G((ik - 1/r)^2 + 1/r^2):
//   G_y = -G' rv.n_y / r,  G_x = G' rv.n_x / r,
//   G_xy = -(G'' - G'/r)(rv.n_x)(rv.n_y)/r^2 - (G'/r) n_x.n_y.
// Near pairs (j != i, |x_i - c_j|^2 < (eta l_j)^2, l_j the longest edge of
// element j): each integral over the flat source triangle is computed by
// geometric subdivision - a sub-triangle is split into its four midpoint
// children until its distance to x is at least 1.5 times its longest edge -
// and an 8 x 8 collapsed Gauss rule on each accepted sub-triangle.  The
// traversal is stackless (a node is its child path from the root), so one
// wavefront handles one pair with every lane on one rule point.
// Self terms (x = centroid of the element, in its plane): K_ii = K'_ii = 0,
//   S_ii = (1/4pi) sum_edges int (exp(ikR) - 1)/(ik) dphi,
//   H_ii = ik/2 - (1/4pi) sum_edges int exp(ikR)/R dphi,  R = d_e / cos(phi),
// i.e. polar coordinates about x with the Hadamard finite part of the
// hypersingular integral (the 1/(2 eps) term of the circular exclusion
// dropped); each edge's angle range is done by 64-point Gauss-Legendre.
#include <cmath>
#include <vector>

#include "plan.h"

namespace bemfmm {

#define ARENA_ALLOC(arena, ptr, count)                                              \
  do {                                                                              \
    int _r = (arena).alloc((void**)&(ptr), sizeof(*(ptr)) * (size_t)(count));      \
    if (_r) return _r;                                                              \
  } while (0)

constexpr double INV_4PI = 0.07957747154594767;  // 1/(4 pi)

struct V3 {
  double x, y, z;
};
__device__ __forceinline__ V3 v3(double x, double y, double z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 vsub(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 vadd(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 vscale(V3 a, double s) { return v3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ double vdot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 vcross(V3 a, V3 b) {
  return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ V3 vmid(V3 a, V3 b) { return vscale(vadd(a, b), 0.5); }
__device__ __forceinline__ V3 ld3(const double* g, int64_t n, int c, int64_t i) {
  return v3(g[c * n + i], g[(c + 1) * n + i], g[(c + 2) * n + i]);
}

__device__ double seg_dist(V3 x, V3 p, V3 q) {
  V3 d = vsub(q, p);
  double t = vdot(vsub(x, p), d) / vdot(d, d);
  t = fmin(fmax(t, 0.0), 1.0);
  V3 f = vsub(x, vadd(p, vscale(d, t)));
  return sqrt(vdot(f, f));
}

__device__ double point_tri_dist(V3 x, V3 a, V3 b, V3 c) {
  V3 nrm = vcross(vsub(b, a), vsub(c, a));
  double nn = sqrt(vdot(nrm, nrm));
  nrm = vscale(nrm, 1.0 / nn);
  double h = vdot(vsub(x, a), nrm);
  V3 x0 = vsub(x, vscale(nrm, h));
  bool inside = vdot(vcross(vsub(b, a), vsub(x0, a)), nrm) >= 0.0 &&
                vdot(vcross(vsub(c, b), vsub(x0, b)), nrm) >= 0.0 &&
                vdot(vcross(vsub(a, c), vsub(x0, c)), nrm) >= 0.0;
  if (inside) return fabs(h);
  return fmin(fmin(seg_dist(x, a, b), seg_dist(x, b, c)), seg_dist(x, c, a));
}

// G, G_y, G_x, G_xy at (x, nx) from (y, ny), float64
__device__ __forceinline__ void kernels64(V3 x, V3 nx, V3 y, V3 ny, double k, c64& G, c64& Gy,
                                          c64& Gx, c64& Gxy) {
  V3 rv = vsub(x, y);
  double r2 = vdot(rv, rv);
  double r = sqrt(r2);
  double u = 1.0 / r;
  double sn, cs;
  sincos(k * r, &sn, &cs);
  G = mk(cs * u * INV_4PI, sn * u * INV_4PI);
  c64 a = mk(-u, k);                                      // ik - 1/r
  c64 g1 = cmul(G, a);                                    // G'
  c64 a2 = cmul(a, a);
  c64 g2 = cmul(G, mk(a2.re + u * u, a2.im));             // G''
  double rnx = vdot(rv, nx), rny = vdot(rv, ny), nxny = vdot(nx, ny);
  Gy = cscale(g1, -rny * u);
  Gx = cscale(g1, rnx * u);
  c64 t = csub(g2, cscale(g1, u));
  Gxy = csub(cscale(t, -rnx * rny * u * u), cscale(g1, u * nxny));
}

__device__ __forceinline__ void node_vertices(V3 A, V3 B, V3 C, uint32_t path, int depth, V3& a,
                                              V3& b, V3& c) {
  a = A;
  b = B;
  c = C;
  for (int d = 0; d < depth; ++d) {
    int ch = (path >> (2 * (depth - 1 - d))) & 3;
    V3 ab = vmid(a, b), bc = vmid(b, c), ca = vmid(c, a);
    if (ch == 0) {
      b = ab;
      c = ca;
    } else if (ch == 1) {
      a = b;
      b = bc;
      c = ab;
    } else if (ch == 2) {
      a = c;
      b = ca;
      c = bc;
    } else {
      a = ab;
      b = bc;
      c = ca;
    }
  }
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int NEAR_MAX_DEPTH = 12;
constexpr double NEAR_GAMMA = 1.5;

// One wavefront per near pair.  rule: 64 x (l1, l2, w) barycentric rule with
// weights summing to 1 (collapsed 8 x 8 Gauss).
__global__ void __launch_bounds__(256) k_near_integrals(
    const double* __restrict__ g, int64_t n, const int* __restrict__ near_row,
    const int* __restrict__ near_col, int64_t nnear, double k, double alr, double ali,
    const double* __restrict__ rule, c64* __restrict__ cp, c64* __restrict__ cq,
    c32* __restrict__ cp32, c32* __restrict__ cq32) {
  int64_t pair = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (pair >= nnear) return;
  int i = near_row[pair], j = near_col[pair];
  V3 x = ld3(g, n, GEO_CX, i), nx = ld3(g, n, GEO_NX, i);
  V3 A = ld3(g, n, GEO_AX, j), B = ld3(g, n, GEO_BX, j), C = ld3(g, n, GEO_CXV, j);
  V3 ny = ld3(g, n, GEO_NX, j);
  double l1 = rule[3 * lane], l2 = rule[3 * lane + 1], w = rule[3 * lane + 2];
  c64 sG = mk(0.0, 0.0), sGy = sG, sGx = sG, sGxy = sG;
  uint32_t path = 0;
  int depth = 0;
  for (int guard = 0; guard < (1 << 20); ++guard) {
    V3 a, b, c;
    node_vertices(A, B, C, path, depth, a, b, c);
    V3 e1 = vsub(b, a), e2 = vsub(c, b), e3 = vsub(a, c);
    double diam = sqrt(fmax(fmax(vdot(e1, e1), vdot(e2, e2)), vdot(e3, e3)));
    double dist = point_tri_dist(x, a, b, c);
    if (dist >= NEAR_GAMMA * diam || depth >= NEAR_MAX_DEPTH) {
      V3 cr = vcross(vsub(b, a), vsub(c, a));
      double area = 0.5 * sqrt(vdot(cr, cr));
      V3 y = vadd(vadd(vscale(a, l1), vscale(b, l2)), vscale(c, 1.0 - l1 - l2));
      c64 G, Gy, Gx, Gxy;
      kernels64(x, nx, y, ny, k, G, Gy, Gx, Gxy);
      double ww = w * area;
      sG = cadd(sG, cscale(G, ww));
      sGy = cadd(sGy, cscale(Gy, ww));
      sGx = cadd(sGx, cscale(Gx, ww));
      sGxy = cadd(sGxy, cscale(Gxy, ww));
      // next node in depth-first order
      while (depth > 0 && (path & 3) == 3) {
        path >>= 2;
        --depth;
      }
      if (depth == 0) break;
      path += 1;
    } else {
      path <<= 2;
      ++depth;
    }
  }
  double v[8] = {sG.re, sG.im, sGy.re, sGy.im, sGx.re, sGx.im, sGxy.re, sGxy.im};
  for (int t = 0; t < 8; ++t) v[t] = wave_sum(v[t]);
  // the 3-point-rule values of the same pair (lanes 0..2, then reduced)
  c64 qG = mk(0.0, 0.0), qGy = qG, qGx = qG, qGxy = qG;
  if (lane < 3) {
    V3 y = ld3(g, n, GEO_QX0 + 3 * lane, j);
    double ww = g[GEO_AREA * n + j] / 3.0;
    kernels64(x, nx, y, ny, k, qG, qGy, qGx, qGxy);
    qG = cscale(qG, ww);
    qGy = cscale(qGy, ww);
    qGx = cscale(qGx, ww);
    qGxy = cscale(qGxy, ww);
  }
  double q[8] = {qG.re, qG.im, qGy.re, qGy.im, qGx.re, qGx.im, qGxy.re, qGxy.im};
  for (int t = 0; t < 8; ++t) q[t] = wave_sum(q[t]);
  if (lane == 0) {
    c64 dS = mk(v[0] - q[0], v[1] - q[1]);
    c64 dK = mk(v[2] - q[2], v[3] - q[3]);
    c64 dKp = mk(v[4] - q[4], v[5] - q[5]);
    c64 dH = mk(v[6] - q[6], v[7] - q[7]);
    c64 al = mk(alr, ali);
    c64 vp = mk(-dK.re, -dK.im);
    vp = csub(vp, cmul(al, dH));          // -(dK + alpha dH)
    c64 vq = cadd(dS, cmul(al, dKp));     // dS + alpha dK'
    cp[pair] = vp;
    cq[pair] = vq;
    cp32[pair] = mk((float)vp.re, (float)vp.im);
    cq32[pair] = mk((float)vq.re, (float)vq.im);
  }
}

// One wavefront per element: self terms; gl: 64 Gauss-Legendre (t, w) on [-1,1].
__global__ void __launch_bounds__(256) k_self_terms(const double* __restrict__ g, int64_t n,
                                                    double k, double alr, double ali,
                                                    const double* __restrict__ gl,
                                                    c64* __restrict__ dp, c64* __restrict__ dq) {
  int64_t e = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (e >= n) return;
  V3 x = ld3(g, n, GEO_CX, e);
  V3 P[3] = {ld3(g, n, GEO_AX, e), ld3(g, n, GEO_BX, e), ld3(g, n, GEO_CXV, e)};
  double t = gl[2 * lane], w = gl[2 * lane + 1];
  double sr = 0, si = 0, hr = 0, hi = 0;
  for (int ed = 0; ed < 3; ++ed) {
    V3 P0 = P[ed], P1 = P[(ed + 1) % 3];
    V3 d = vsub(P1, P0);
    double len = sqrt(vdot(d, d));
    V3 tu = vscale(d, 1.0 / len);
    double s0 = vdot(vsub(x, P0), tu);
    V3 foot = vadd(P0, vscale(tu, s0));
    V3 fx = vsub(x, foot);
    double de = sqrt(vdot(fx, fx));
    double pm = atan2(-s0, de), pp = atan2(len - s0, de);
    double half = 0.5 * (pp - pm);
    double phi = 0.5 * (pp + pm) + half * t;
    double ww = half * w;
    double R = de / cos(phi);
    double kr = k * R;
    double sn, cs;
    sincos(kr, &sn, &cs);
    double sh = sin(0.5 * kr);
    // (exp(ikR) - 1)/(ik) = (sin kR + 2i sin^2(kR/2)) / k
    sr += ww * sn / k;
    si += ww * 2.0 * sh * sh / k;
    hr -= ww * cs / R;
    hi -= ww * sn / R;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  hr = wave_sum(hr);
  hi = wave_sum(hi);
  if (lane == 0) {
    c64 S = mk(sr * INV_4PI, si * INV_4PI);
    c64 H = mk(hr * INV_4PI, hi * INV_4PI + 0.5 * k);
    c64 al = mk(alr, ali);
    dp[e] = csub(mk(0.5, 0.0), cmul(al, H));   // 1/2 - alpha H_ii  (K_ii = 0)
    dq[e] = cadd(S, cscale(al, 0.5));          // S_ii + alpha/2    (K'_ii = 0)
  }
}

__device__ __forceinline__ bool is_near(const double* __restrict__ g, int64_t n, int i, int j,
                                        double eta) {
#pragma clang fp contract(off)
  double dx = g[GEO_CX * n + i] - g[GEO_CX * n + j];
  double dy = g[GEO_CY * n + i] - g[GEO_CY * n + j];
  double dz = g[GEO_CZ * n + i] - g[GEO_CZ * n + j];
  double d2 = dx * dx + dy * dy + dz * dz;
  double t = eta * g[GEO_ELL * n + j];
  return d2 < t * t;
}

// near pairs by target (transpose = 0) or by source (transpose = 1);
// pass 0 counts, pass 1 writes the partner indices (ascending).  Candidates
// are the elements of the adjacent leaves, or every element (brute) when the
// leaves are not wider than the near radius.
__global__ void k_near_lists(const double* __restrict__ g, int64_t n,
                             const int* __restrict__ elem_leaf, const int* __restrict__ u_ptr,
                             const int* __restrict__ u_idx, const int* __restrict__ bstart,
                             double eta, int transpose, int brute, const int* __restrict__ ptr,
                             int* __restrict__ cnt, int* __restrict__ partner, int fill) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  int b = elem_leaf[e];
  int c = 0, o = fill ? ptr[e] : 0;
  if (brute) {
    // leaves narrower than the near radius: search every element
    for (int f = 0; f < (int)n; ++f) {
      if (f == e) continue;
      bool nr = transpose ? is_near(g, n, f, (int)e, eta) : is_near(g, n, (int)e, f, eta);
      if (!nr) continue;
      if (fill) partner[o + c] = f;
      ++c;
    }
    if (!fill) cnt[e] = c;
    return;
  }
  for (int t = u_ptr[b]; t < u_ptr[b + 1]; ++t) {
    int nb = u_idx[t];
    for (int f = bstart[nb]; f < bstart[nb + 1]; ++f) {
      if (f == e) continue;
      bool nr = transpose ? is_near(g, n, f, (int)e, eta) : is_near(g, n, (int)e, f, eta);
      if (!nr) continue;
      if (fill) partner[o + c] = f;
      ++c;
    }
  }
  if (!fill) cnt[e] = c;
}

__global__ void k_rows_of(const int* __restrict__ ptr, int64_t n, int* __restrict__ row) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int t = ptr[i]; t < ptr[i + 1]; ++t) row[t] = (int)i;
}

// values of the transposed list: entry (j, i) copies row i's entry for column j
template <typename T>
__global__ void k_transpose_values(const int* __restrict__ tptr, const int* __restrict__ trow,
                                   int64_t n, const int* __restrict__ ptr,
                                   const int* __restrict__ col, const T* __restrict__ a,
                                   const T* __restrict__ b, T* __restrict__ ta,
                                   T* __restrict__ tb) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int t = tptr[j]; t < tptr[j + 1]; ++t) {
    int i = trow[t];
    int lo = ptr[i], hi = ptr[i + 1];
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (col[mid] < (int)j)
        lo = mid + 1;
      else
        hi = mid;
    }
    ta[t] = a[lo];
    tb[t] = b[lo];
  }
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_m.
void gauss_legendre(int m, std::vector<double>& t, std::vector<double>& w) {
  t.assign(m, 0.0);
  w.assign(m, 0.0);
  for (int i = 0; i < m; ++i) {
    double z = cos(M_PI * (i + 0.75) / (m + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int kk = 2; kk <= m; ++kk) {
        double p2 = ((2.0 * kk - 1.0) * z * p1 - (kk - 1.0) * p0) / kk;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_m(z), p0 = P_{m-1}(z)
      double dp = m * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int kk = 2; kk <= m; ++kk) {
      double p2 = ((2.0 * kk - 1.0) * z * p1 - (kk - 1.0) * p0) / kk;
      p0 = p1;
      p1 = p2;
    }
    double dp = m * (z * p1 - p0) / (z * z - 1.0);
    t[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

int build_near_field(Problem& P, hipStream_t s) {
  const int64_t n = P.n;
  DevArena scratch;
  struct Guard {
    DevArena& a;
    ~Guard() { a.release(); }
  } guard{scratch};
  int* cnt;
  ARENA_ALLOC(scratch, cnt, n);
  ARENA_ALLOC(P.arena, P.near_ptr, n + 1);
  ARENA_ALLOC(P.arena, P.neart_ptr, n + 1);
  const int* bstart = P.box_start[P.L];
  int nb = ceil_div(n, 128);
  int total = 0, total_t = 0;
  const int brute = P.direct ? 1 : 0;
  if (brute && n > 200000) {
    set_error("mesh too coarse for its size: elements wider than the finest usable leaf");
    return -1;
  }
  // by target
  hipLaunchKernelGGL(k_near_lists, dim3(nb), dim3(128), 0, s, P.geo, n, P.elem_leaf, P.u_ptr,
                     P.u_idx, bstart, P.eta, 0, brute, (const int*)nullptr, cnt, (int*)nullptr, 0);
  BEM_LAUNCH_CHECK();
  int r = exclusive_scan(cnt, P.near_ptr, (int)n, &total, scratch, s);
  if (r) return r;
  BEM_HIP_TRY(hipMemcpyAsync(P.near_ptr + n, &total, sizeof(int), hipMemcpyHostToDevice, s));
  ARENA_ALLOC(P.arena, P.near_col, total);
  hipLaunchKernelGGL(k_near_lists, dim3(nb), dim3(128), 0, s, P.geo, n, P.elem_leaf, P.u_ptr,
                     P.u_idx, bstart, P.eta, 0, brute, P.near_ptr, cnt, P.near_col, 1);
  BEM_LAUNCH_CHECK();
  // by source
  hipLaunchKernelGGL(k_near_lists, dim3(nb), dim3(128), 0, s, P.geo, n, P.elem_leaf, P.u_ptr,
                     P.u_idx, bstart, P.eta, 1, brute, (const int*)nullptr, cnt, (int*)nullptr, 0);
  BEM_LAUNCH_CHECK();
  r = exclusive_scan(cnt, P.neart_ptr, (int)n, &total_t, scratch, s);
  if (r) return r;
  if (total_t != total) {
    set_error("internal: near list and its transpose differ in size");
    return -3;
  }
  BEM_HIP_TRY(hipMemcpyAsync(P.neart_ptr + n, &total_t, sizeof(int), hipMemcpyHostToDevice, s));
  ARENA_ALLOC(P.arena, P.neart_row, total);
  hipLaunchKernelGGL(k_near_lists, dim3(nb), dim3(128), 0, s, P.geo, n, P.elem_leaf, P.u_ptr,
                     P.u_idx, bstart, P.eta, 1, brute, P.neart_ptr, cnt, P.neart_row, 1);
  BEM_LAUNCH_CHECK();
  P.n_near = total;
  // accurate integrals
  int* row;
  ARENA_ALLOC(scratch, row, total);
  hipLaunchKernelGGL(k_rows_of, dim3(nb), dim3(128), 0, s, P.near_ptr, n, row);
  BEM_LAUNCH_CHECK();
  ARENA_ALLOC(P.arena, P.f64.near_cp, total);
  ARENA_ALLOC(P.arena, P.f64.near_cq, total);
  ARENA_ALLOC(P.arena, P.f32.near_cp, total);
  ARENA_ALLOC(P.arena, P.f32.near_cq, total);
  ARENA_ALLOC(P.arena, P.f64.neart_cp, total);
  ARENA_ALLOC(P.arena, P.f64.neart_cq, total);
  ARENA_ALLOC(P.arena, P.f32.neart_cp, total);
  ARENA_ALLOC(P.arena, P.f32.neart_cq, total);
  // 8 x 8 collapsed Gauss rule on the triangle
  std::vector<double> t8, w8, rule(3 * 64), t64, w64, gl(2 * 64);
  gauss_legendre(NEAR_RULE, t8, w8);
  for (int a = 0; a < NEAR_RULE; ++a)
    for (int b = 0; b < NEAR_RULE; ++b) {
      double u = 0.5 * (t8[a] + 1.0), wu = 0.5 * w8[a];
      double v = 0.5 * (t8[b] + 1.0), wv = 0.5 * w8[b];
      int q = a * NEAR_RULE + b;
      rule[3 * q] = u;
      rule[3 * q + 1] = (1.0 - u) * v;
      rule[3 * q + 2] = 2.0 * wu * wv * (1.0 - u);
    }
  gauss_legendre(SELF_RULE, t64, w64);
  for (int q = 0; q < 64; ++q) {
    gl[2 * q] = t64[q];
    gl[2 * q + 1] = w64[q];
  }
  double *drule, *dgl;
  ARENA_ALLOC(scratch, drule, rule.size());
  ARENA_ALLOC(scratch, dgl, gl.size());
  BEM_HIP_TRY(hipMemcpyAsync(drule, rule.data(), sizeof(double) * rule.size(),
                             hipMemcpyHostToDevice, s));
  BEM_HIP_TRY(hipMemcpyAsync(dgl, gl.data(), sizeof(double) * gl.size(), hipMemcpyHostToDevice, s));
  if (total > 0) {
    int64_t threads = (int64_t)total * 64;
    hipLaunchKernelGGL(k_near_integrals, dim3(ceil_div(threads, 256)), dim3(256), 0, s, P.geo, n,
                       row, P.near_col, (int64_t)total, P.k, P.alpha.re, P.alpha.im, drule,
                       P.f64.near_cp, P.f64.near_cq, P.f32.near_cp, P.f32.near_cq);
    BEM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_transpose_values<c64>, dim3(nb), dim3(128), 0, s, P.neart_ptr,
                       P.neart_row, n, P.near_ptr, P.near_col, P.f64.near_cp, P.f64.near_cq,
                       P.f64.neart_cp, P.f64.neart_cq);
    BEM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_transpose_values<c32>, dim3(nb), dim3(128), 0, s, P.neart_ptr,
                       P.neart_row, n, P.near_ptr, P.near_col, P.f32.near_cp, P.f32.near_cq,
                       P.f32.neart_cp, P.f32.neart_cq);
    BEM_LAUNCH_CHECK();
  }
  ARENA_ALLOC(P.arena, P.diag_p, n);
  ARENA_ALLOC(P.arena, P.diag_q, n);
  hipLaunchKernelGGL(k_self_terms, dim3(ceil_div(n * 64, 256)), dim3(256), 0, s, P.geo, n, P.k,
                     P.alpha.re, P.alpha.im, dgl, P.diag_p, P.diag_q);
  BEM_LAUNCH_CHECK();
  BEM_HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

}  // namespace bemfmm
