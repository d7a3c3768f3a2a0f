// Far-field operators, built once per plan in float64 on the device.
//
// The paper applies its BEM blocks with a low-frequency FMM (Sec. 2.3) whose
// formulas it does not give; this is our own design from the published
// spherical-wave expansion of the Helmholtz kernel.  With orthonormal
// spherical harmonics Y_n^m (Condon-Shortley phase), regular and singular
// wave functions R_n^m(v) = j_n(k|v|) Y_n^m(v^), S_n^m(v) = h_n(k|v|) Y_n^m(v^)
// (h_n = j_n + i y_n, outgoing for the exp(-i omega t) convention of
// Sec. 2.1), the kernel G = exp(ikr)/(4 pi r) separates as
//     G(x - y) = ik sum_nm S_n^m(x - c) conj(R_n^m(y - c)),  |y-c| < |x-c|.
// Translations follow from the plane-wave integral of R_n^m and the Gaunt
// coefficients g(n,m; n',m'; l) = int Y_n^m conj(Y_n'^m') conj(Y_l^(m-m')):
//     F_n^m(r + t) = sum_n'm' (F|R)_{n'm',nm}(t) R_n'^m'(r),
//     (F|R)_{n'm',nm}(t) = sum_l 4 pi i^(n'+l-n) F_l^(m-m')(t) g(n,m;n',m';l)
// with F = S for multipole-to-local (|r| < |t|) and F = R for local-to-local;
// the multipole-to-multipole matrix equals the regular one.  Gradients use
// the l = 1 terms of the same formula.  Gaunt coefficients are integrated
// exactly by Gauss-Legendre quadrature in cos(theta).
//
// Coefficients are scaled per level so that every stored number is O(1) in
// float32: with f_n = (k h_l)^n / (2n+1)!! (h_l the box side), multipoles are
// kept as M_n / f_n and locals as L_n f_n.
#include <cmath>
#include <complex>
#include <vector>

#include "plan.h"
#include "wavefun.h"

namespace bemfmm {

#define ARENA_ALLOC(arena, ptr, count)                                              \
  do {                                                                              \
    int _r = (arena).alloc((void**)&(ptr), sizeof(*(ptr)) * (size_t)(count));      \
    if (_r) return _r;                                                              \
  } while (0)

void gauss_legendre(int m, std::vector<double>& t, std::vector<double>& w);
int build_vlist(Problem& P, int l, int** dst, int** src, int** code, int* npairs,
                DevArena& scratch, hipStream_t s);

constexpr double FOUR_PI = 12.566370614359172;
constexpr int MAXP = 40;         // largest supported expansion order
constexpr int MAXL = 2 * MAXP + 2;

__host__ __device__ __forceinline__ int cidx(int n, int m) { return n * n + n + m; }

// Theta_n^m(x), 0 <= m <= n <= nmax, normalised associated Legendre functions
// with Condon-Shortley phase (Y_n^m = Theta_n^m(cos t) exp(i m phi)), written
// to out[n*(nmax+1) + m].  Standard three-term recurrences.
__device__ void theta_table(int nmax, double x, double* out, int stride) {
  double s = sqrt(fmax(0.0, 1.0 - x * x));
  double tmm = 0.28209479177387814;  // 1/sqrt(4 pi)
  for (int m = 0; m <= nmax; ++m) {
    if (m > 0) tmm = -sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * tmm;
    out[m * stride + m] = tmm;
    if (m < nmax) {
      double t1 = sqrt(2.0 * m + 3.0) * x * tmm;
      out[(m + 1) * stride + m] = t1;
      double t0 = tmm;
      for (int n = m + 2; n <= nmax; ++n) {
        double a = sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
        double b = sqrt(((n - 1.0) * (n - 1.0) - (double)m * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
        double t2 = a * (x * t1 - b * t0);
        out[n * stride + m] = t2;
        t0 = t1;
        t1 = t2;
      }
    }
  }
}

// spherical Bessel y_n(x), upward recurrence (stable for y)
__device__ void sph_yn(int nmax, double x, double* out) {
  double sn = sin(x), cs = cos(x);
  out[0] = -cs / x;
  if (nmax >= 1) out[1] = -cs / (x * x) - sn / x;
  for (int n = 1; n < nmax; ++n) out[n + 1] = (2.0 * n + 1.0) / x * out[n] - out[n - 1];
}

// All R_n^m (sing = 0) or S_n^m (sing = 1) at v for n <= nmax, into out
// (complex, cidx order).  tmp: >= (nmax+1)^2 + 2(nmax+1) doubles.
__device__ void wave_functions(int nmax, double k, double vx, double vy, double vz, int sing,
                               c64* out, double* tmp) {
  double r = sqrt(vx * vx + vy * vy + vz * vz);
  double ct = (r > 0.0) ? vz / r : 1.0;
  double rxy = sqrt(vx * vx + vy * vy);
  double cp = (rxy > 0.0) ? vx / rxy : 1.0, sp = (rxy > 0.0) ? vy / rxy : 0.0;
  double* th = tmp;                          // (nmax+1)^2
  double* jr = tmp + (nmax + 1) * (nmax + 1);  // nmax+1
  double* yr = jr + (nmax + 1);
  theta_table(nmax, ct, th, nmax + 1);
  sph_jn(nmax, k * r, jr);
  if (sing) sph_yn(nmax, k * r, yr);
  double er = 1.0, ei = 0.0;  // exp(i m phi)
  for (int m = 0; m <= nmax; ++m) {
    if (m > 0) {
      double t = er * cp - ei * sp;
      ei = er * sp + ei * cp;
      er = t;
    }
    double sgn = (m & 1) ? -1.0 : 1.0;
    for (int n = m; n <= nmax; ++n) {
      double t = th[n * (nmax + 1) + m];
      c64 rad = sing ? mk(jr[n], yr[n]) : mk(jr[n], 0.0);
      c64 y = mk(t * er, t * ei);
      out[cidx(n, m)] = cmul(rad, y);
      if (m > 0) {
        // Y_n^-m = (-1)^m conj(Y_n^m)
        c64 yneg = mk(sgn * t * er, -sgn * t * ei);
        out[cidx(n, -m)] = cmul(rad, yneg);
      }
    }
  }
}

// Gaunt table: for input (n,m) (n <= pin) and output (n',m') (n' <= pout),
// gt[(in * Pout + out) * J + j] = g(n,m; n',m'; l) with l = |n-n'| + 2j,
// j < J = min(pin,pout)+1 (zero where |m-m'| > l or l > lmax).
// th: Theta tables at the K Gauss nodes, th[(q*(tmax+1) + l)*(tmax+1) + mu],
// tmax = max(pin, pout, lmax).
__global__ void k_gaunt(int pin, int pout, int lmax, int tmax, int K,
                        const double* __restrict__ gw, const double* __restrict__ th,
                        double* __restrict__ gt) {
  int Pin = (pin + 1) * (pin + 1), Pout = (pout + 1) * (pout + 1);
  int J = min(pin, pout) + 1;
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)Pin * Pout) return;
  int in = (int)(t / Pout), out = (int)(t % Pout);
  int n = (int)sqrt((double)in);
  while (n * n > in) --n;
  while ((n + 1) * (n + 1) <= in) ++n;
  int m = in - n * n - n;
  int n2 = (int)sqrt((double)out);
  while (n2 * n2 > out) --n2;
  while ((n2 + 1) * (n2 + 1) <= out) ++n2;
  int m2 = out - n2 * n2 - n2;
  int mu = m - m2;
  int L1 = tmax + 1;
  for (int j = 0; j < J; ++j) {
    int l = abs(n - n2) + 2 * j;
    double val = 0.0;
    if (l <= n + n2 && l <= lmax && abs(mu) <= l) {
      for (int q = 0; q < K; ++q) {
        const double* T = th + (int64_t)q * L1 * L1;
        double a = T[n * L1 + abs(m)] * ((m < 0 && (m & 1)) ? -1.0 : 1.0);
        double b = T[n2 * L1 + abs(m2)] * ((m2 < 0 && (m2 & 1)) ? -1.0 : 1.0);
        double c = T[l * L1 + abs(mu)] * ((mu < 0 && (mu & 1)) ? -1.0 : 1.0);
        val += gw[q] * a * b * c;
      }
      val *= 6.283185307179586;  // 2 pi from the phi integral
    }
    gt[t * J + j] = val;
  }
}

__global__ void k_theta_nodes(int lmax, int K, const double* __restrict__ gx,
                              double* __restrict__ th) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= K) return;
  theta_table(lmax, gx[q], th + (int64_t)q * (lmax + 1) * (lmax + 1), lmax + 1);
}

// F_l^mu(t_g) for each group vector, l <= lmax: out[g * (lmax+1)^2 + cidx(l,mu)]
__global__ void k_group_waves(int ngroups, const double* __restrict__ tv, double k, int lmax,
                              int sing, c64* __restrict__ out, double* __restrict__ tmp) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroups) return;
  int L1 = lmax + 1;
  wave_functions(lmax, k, tv[3 * g], tv[3 * g + 1], tv[3 * g + 2], sing, out + (int64_t)g * L1 * L1,
                 tmp + (int64_t)g * (L1 * L1 + 2 * L1));
}

// Translation matrices, one per group: mats[g][out][in] (row-major),
//   T = sum_l 4 pi i^(n'+l-n) F_l^(m-m')(t_g) g(n,m;n',m';l),
// times the level scaling rs[out] * cs[in].
template <typename R>
__global__ void k_translation(int ngroups, int pin, int pout, int lmax,
                              const c64* __restrict__ F, const double* __restrict__ gt,
                              const double* __restrict__ rs, const double* __restrict__ cs,
                              cplx<R>* __restrict__ mats) {
  int Pin = (pin + 1) * (pin + 1), Pout = (pout + 1) * (pout + 1);
  int J = min(pin, pout) + 1;
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t per = (int64_t)Pin * Pout;
  if (t >= per * ngroups) return;
  int g = (int)(t / per);
  int64_t e = t % per;
  int out = (int)(e / Pin), in = (int)(e % Pin);
  int n = (int)sqrt((double)in);
  while (n * n > in) --n;
  while ((n + 1) * (n + 1) <= in) ++n;
  int m = in - n * n - n;
  int n2 = (int)sqrt((double)out);
  while (n2 * n2 > out) --n2;
  while ((n2 + 1) * (n2 + 1) <= out) ++n2;
  int m2 = out - n2 * n2 - n2;
  int mu = m - m2;
  const c64* Fg = F + (int64_t)g * (lmax + 1) * (lmax + 1);
  const double* G = gt + ((int64_t)in * Pout + out) * J;
  c64 acc = mk(0.0, 0.0);
  for (int j = 0; j < J; ++j) {
    int l = abs(n - n2) + 2 * j;
    if (l > n + n2 || l > lmax || abs(mu) > l) continue;
    double gv = G[j];
    if (gv == 0.0) continue;
    c64 f = Fg[cidx(l, mu)];
    int e4 = (n2 + l - n) & 3;  // i^e
    c64 ie = (e4 == 0) ? mk(1.0, 0.0) : (e4 == 1) ? mk(0.0, 1.0) : (e4 == 2) ? mk(-1.0, 0.0) : mk(0.0, -1.0);
    acc = cadd(acc, cscale(cmul(ie, f), FOUR_PI * gv));
  }
  acc = cscale(acc, rs[out] * cs[in]);
  mats[t] = mk((R)acc.re, (R)acc.im);
}

// Directional derivative coefficients: for unit vector d,
//   d . grad R_n^m = sum_{s=+-1, mu} gc[(cidx(n,m)*2 + (s>0))*3 + mu+1] c_mu(d) R_{n+s}^{m-mu}
// with c_0 = sqrt(3/4pi) d_z, c_{+1} = -sqrt(3/8pi)(d_x + i d_y),
// c_{-1} = sqrt(3/8pi)(d_x - i d_y); gc holds 4 pi i^(n'+1-n) (k/3) g(n,m;n',m';1).
__device__ __forceinline__ c64 cmu(int mu, double dx, double dy, double dz) {
  if (mu == 0) return mk(0.4886025119029199 * dz, 0.0);
  if (mu == 1) return mk(-0.3454941494713355 * dx, -0.3454941494713355 * dy);
  return mk(0.3454941494713355 * dx, -0.3454941494713355 * dy);
}

// Per element (sorted order) P2M columns and L2P row at leaf centre c:
//  p2m[e][c][1] (q column) = ik/f_n * (A/3) sum_q conj(R_n^m(y_q - c))
//  p2m[e][c][0] (p column) = -ik/f_n * (A/3) sum_q conj(n_e . grad R_n^m(y_q - c))
//  l2p[e][c]               = (R_n^m + alpha n_e . grad R_n^m)(x_e - c) / f_n
// Rbuf: per thread scratch for (p+2)^2 wave functions of 4 points.
template <typename R>
__global__ void k_p2m_l2p(const double* __restrict__ g, int64_t n, int64_t e0, int64_t ne,
                          const int* __restrict__ elem_leaf, const uint64_t* __restrict__ lkeys,
                          int L, const double* __restrict__ lo, double hL, double k, double alr,
                          double ali, int p, const double* __restrict__ gc,
                          const double* __restrict__ finv, c64* __restrict__ Rbuf,
                          double* __restrict__ tmpbuf, cplx<R>* __restrict__ p2m,
                          cplx<R>* __restrict__ l2p) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= ne) return;
  int64_t e = e0 + t;
  int P1 = (p + 2) * (p + 2), P = (p + 1) * (p + 1);
  c64* Rb = Rbuf + t * 4 * P1;
  double* tmp = tmpbuf + t * ((p + 2) * (p + 2) + 2 * (p + 2));
  uint64_t key = lkeys[elem_leaf[e]];
  double c[3];
  uint32_t ix = 0, iy = 0, iz = 0;
  for (int b = 0; b < L; ++b) {
    ix |= (uint32_t)((key >> (3 * b + 2)) & 1) << b;
    iy |= (uint32_t)((key >> (3 * b + 1)) & 1) << b;
    iz |= (uint32_t)((key >> (3 * b)) & 1) << b;
  }
  c[0] = lo[0] + (ix + 0.5) * hL;
  c[1] = lo[1] + (iy + 0.5) * hL;
  c[2] = lo[2] + (iz + 0.5) * hL;
  for (int q = 0; q < 3; ++q) {
    double vx = g[(GEO_QX0 + 3 * q) * n + e] - c[0];
    double vy = g[(GEO_QX0 + 3 * q + 1) * n + e] - c[1];
    double vz = g[(GEO_QX0 + 3 * q + 2) * n + e] - c[2];
    wave_functions(p + 1, k, vx, vy, vz, 0, Rb + q * P1, tmp);
  }
  wave_functions(p + 1, k, g[GEO_CX * n + e] - c[0], g[GEO_CY * n + e] - c[1],
                 g[GEO_CZ * n + e] - c[2], 0, Rb + 3 * P1, tmp);
  double nx = g[GEO_NX * n + e], ny = g[GEO_NY * n + e], nz = g[GEO_NZ * n + e];
  double w3 = g[GEO_AREA * n + e] / 3.0;
  c64 cm[3] = {cmu(-1, nx, ny, nz), cmu(0, nx, ny, nz), cmu(1, nx, ny, nz)};
  c64 al = mk(alr, ali);
  for (int nn = 0; nn <= p; ++nn) {
    for (int m = -nn; m <= nn; ++m) {
      int ci = cidx(nn, m);
      c64 sq = mk(0.0, 0.0), sp = mk(0.0, 0.0), rt = mk(0.0, 0.0), gt = mk(0.0, 0.0);
      for (int pt = 0; pt < 4; ++pt) {
        const c64* Rv = Rb + pt * P1;
        c64 grad = mk(0.0, 0.0);
        for (int sgn = 0; sgn < 2; ++sgn) {
          int n2 = sgn ? nn + 1 : nn - 1;
          if (n2 < 0) continue;
          for (int mu = -1; mu <= 1; ++mu) {
            int m2 = m - mu;
            if (abs(m2) > n2) continue;
            const double* gg = gc + ((int64_t)(ci * 2 + sgn) * 3 + (mu + 1)) * 2;
            c64 coef = mk(gg[0], gg[1]);
            grad = cadd(grad, cmul(cmul(coef, cm[mu + 1]), Rv[cidx(n2, m2)]));
          }
        }
        if (pt < 3) {
          sq = cadd(sq, cconj(Rv[ci]));
          sp = cadd(sp, cconj(grad));
        } else {
          rt = Rv[ci];
          gt = grad;
        }
      }
      double fi = finv[nn];  // 1 / f_n
      c64 ik = mk(0.0, k);
      c64 aq = cscale(cmul(ik, sq), w3 * fi);
      c64 ap = cscale(cmul(ik, sp), -w3 * fi);
      c64 b = cscale(cadd(rt, cmul(al, gt)), fi);
      p2m[(e * P + ci) * 2 + 0] = mk((R)ap.re, (R)ap.im);
      p2m[(e * P + ci) * 2 + 1] = mk((R)aq.re, (R)aq.im);
      l2p[e * P + ci] = mk((R)b.re, (R)b.im);
    }
  }
}

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------
struct GauntSet {
  double* d = nullptr;
  int pin = 0, pout = 0, lmax = 0;
};

static int make_gaunt(int pin, int pout, int lmax, GauntSet& G, DevArena& scratch, hipStream_t s) {
  int K = (pin + pout + lmax) / 2 + 2;
  int tmax = std::max(std::max(pin, pout), lmax);
  std::vector<double> gx, gw;
  gauss_legendre(K, gx, gw);
  double *dgx, *dgw, *th;
  ARENA_ALLOC(scratch, dgx, K);
  ARENA_ALLOC(scratch, dgw, K);
  ARENA_ALLOC(scratch, th, (int64_t)K * (tmax + 1) * (tmax + 1));
  BEM_HIP_TRY(hipMemcpyAsync(dgx, gx.data(), sizeof(double) * K, hipMemcpyHostToDevice, s));
  BEM_HIP_TRY(hipMemcpyAsync(dgw, gw.data(), sizeof(double) * K, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_theta_nodes, dim3(ceil_div(K, 64)), dim3(64), 0, s, tmax, K, dgx, th);
  BEM_LAUNCH_CHECK();
  int64_t Pin = (pin + 1) * (pin + 1), Pout = (pout + 1) * (pout + 1);
  int J = std::min(pin, pout) + 1;
  ARENA_ALLOC(scratch, G.d, Pin * Pout * J);
  hipLaunchKernelGGL(k_gaunt, dim3(ceil_div(Pin * Pout, 128)), dim3(128), 0, s, pin, pout, lmax,
                     tmax, K, dgw, th, G.d);
  BEM_LAUNCH_CHECK();
  G.pin = pin;
  G.pout = pout;
  G.lmax = lmax;
  return 0;
}

// scaling vector per coefficient: f_n^power, f_n = (k h)^n / (2n+1)!!
static std::vector<double> coef_scale(int p, double kh, int power) {
  std::vector<double> f(p + 1), out((p + 1) * (p + 1));
  double v = 1.0;
  for (int nn = 0; nn <= p; ++nn) {
    if (nn > 0) v *= kh / (2.0 * nn + 1.0);
    f[nn] = v;
  }
  for (int nn = 0; nn <= p; ++nn)
    for (int m = -nn; m <= nn; ++m) out[cidx(nn, m)] = (power > 0) ? f[nn] : 1.0 / f[nn];
  return out;
}

// out[g][c][r] = conj(in[g][r][c]) for n matrices of rows x cols
template <typename R>
__global__ void k_conj_transpose(const cplx<R>* __restrict__ in, int n, int rows, int cols,
                                 cplx<R>* __restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * rows * cols) return;
  const int64_t per = (int64_t)rows * cols, g = t / per;
  const int r = (int)((t - g * per) / cols), c = (int)(t - g * per - (int64_t)r * cols);
  const cplx<R> v = in[t];
  out[g * per + (int64_t)c * rows + r] = mk<R>(v.re, -v.im);
}

// out[t] = in[2 t] (the p columns of the interleaved P2M matrices)
template <typename R>
__global__ void k_p_columns(const cplx<R>* __restrict__ in, int64_t cnt,
                            cplx<R>* __restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < cnt) out[t] = in[2 * t];
}

// mats[g][r][c] = 0 for c >= kc[g] (n matrices of rows x cols)
template <typename R>
__global__ void k_zero_columns(cplx<R>* __restrict__ mats, int n, int rows, int cols,
                               const int* __restrict__ kc) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * rows * cols) return;
  const int64_t per = (int64_t)rows * cols, g = t / per;
  const int c = (int)((t - g * per) % cols);
  if (c >= kc[g]) mats[t] = mk<R>(0, 0);
}

// Input cut of the M2L translations across three boxes (Chebyshev distance
// 3 of the offset code c in the 7^3 table, or of the PT_W^3 table): with
// far_cut > 0 their operators read only the coefficients of degree
// <= p - far_cut of the source multipole.  Zeroes the operator columns
// beyond the cut (slot order) and returns the per-group counts (code
// order) on the device, or null when nothing is cut.
template <typename R>
static int cut_far_translations(GroupedOp<R>& op, int p, int far_cut, int ngroups, int width,
                                const std::vector<int>& slot, DevArena& keep,
                                DevArena& scratch, hipStream_t s) {
  op.group_kc = nullptr;
  if (far_cut <= 0 || op.n_slots == 0) return 0;
  const int pf = std::max(0, p - far_cut), kcut = (pf + 1) * (pf + 1);
  const int off = width / 2;
  std::vector<int> kc_group(ngroups, op.cols), kc_slot(op.n_slots, op.cols);
  for (int c = 0; c < ngroups; ++c) {
    const int dx = c / (width * width) - off, dy = (c / width) % width - off, dz = c % width - off;
    const int cheb = std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz)));
    if (cheb >= 3) {
      kc_group[c] = kcut;
      if (slot[c] >= 0) kc_slot[slot[c]] = kcut;
    }
  }
  int* dks;
  ARENA_ALLOC(scratch, dks, op.n_slots);
  ARENA_ALLOC(keep, op.group_kc, ngroups);
  BEM_HIP_TRY(hipMemcpyAsync(dks, kc_slot.data(), sizeof(int) * op.n_slots, hipMemcpyHostToDevice, s));
  BEM_HIP_TRY(hipMemcpyAsync(op.group_kc, kc_group.data(), sizeof(int) * ngroups,
                             hipMemcpyHostToDevice, s));
  const int64_t tot = (int64_t)op.n_slots * op.rows * op.cols;
  hipLaunchKernelGGL(k_zero_columns<R>, dim3(ceil_div(tot, 256)), dim3(256), 0, s, op.mats,
                     op.n_slots, op.rows, op.cols, dks);
  BEM_LAUNCH_CHECK();
  BEM_HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

template <typename R>
static int make_translations(Problem& P, DevArena& keep, int ngroups,
                             const std::vector<double>& tvec, int sing, int pin, int pout,
                             const std::vector<double>& rs, const std::vector<double>& cs,
                             cplx<R>** mats, DevArena& scratch, hipStream_t s) {
  int lmax = pin + pout;
  GauntSet G;
  int r = make_gaunt(pin, pout, lmax, G, scratch, s);
  if (r) return r;
  int L1 = lmax + 1;
  double *dtv, *tmp, *drs, *dcs;
  c64* F;
  ARENA_ALLOC(scratch, dtv, 3 * ngroups);
  ARENA_ALLOC(scratch, F, (int64_t)ngroups * L1 * L1);
  ARENA_ALLOC(scratch, tmp, (int64_t)ngroups * (L1 * L1 + 2 * L1));
  ARENA_ALLOC(scratch, drs, rs.size());
  ARENA_ALLOC(scratch, dcs, cs.size());
  BEM_HIP_TRY(hipMemcpyAsync(dtv, tvec.data(), sizeof(double) * 3 * ngroups, hipMemcpyHostToDevice, s));
  BEM_HIP_TRY(hipMemcpyAsync(drs, rs.data(), sizeof(double) * rs.size(), hipMemcpyHostToDevice, s));
  BEM_HIP_TRY(hipMemcpyAsync(dcs, cs.data(), sizeof(double) * cs.size(), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_group_waves, dim3(ceil_div(ngroups, 64)), dim3(64), 0, s, ngroups, dtv,
                     P.k, lmax, sing, F, tmp);
  BEM_LAUNCH_CHECK();
  int64_t Pin = (pin + 1) * (pin + 1), Pout = (pout + 1) * (pout + 1);
  ARENA_ALLOC(keep, *mats, Pin * Pout * ngroups);
  int64_t tot = Pin * Pout * ngroups;
  hipLaunchKernelGGL(k_translation<R>, dim3(ceil_div(tot, 256)), dim3(256), 0, s, ngroups, pin,
                     pout, lmax, F, G.d, drs, dcs, *mats);
  BEM_LAUNCH_CHECK();
  return 0;
}

// make_translations into D.ops through the precision's cache: the matrices
// are a function of the arguments (k is the problem's), so a build whose
// arguments equal the cached entry's copies that entry instead
template <typename R>
static int cached_translations(Problem& P, PrecisionData<R>& D, int key, int ngroups,
                               const std::vector<double>& tv, int sing, int pin, int pout,
                               const std::vector<double>& rs, const std::vector<double>& cs,
                               cplx<R>** mats, DevArena& scratch, hipStream_t s) {
  auto& e = D.tcache[key];
  if (!(e.mats && e.ngroups == ngroups && e.sing == sing && e.pin == pin && e.pout == pout &&
        e.tv == tv && e.rs == rs && e.cs == cs)) {
    e.arena.release();
    e.mats = nullptr;
    e.ngroups = -1;
    int r = make_translations<R>(P, e.arena, ngroups, tv, sing, pin, pout, rs, cs, &e.mats,
                                 scratch, s);
    if (r) {
      e.arena.release();
      e.mats = nullptr;
      return r;
    }
    e.ngroups = ngroups;
    e.sing = sing;
    e.pin = pin;
    e.pout = pout;
    e.tv = tv;
    e.rs = rs;
    e.cs = cs;
  }
  const int64_t cnt = (int64_t)ngroups * (pin + 1) * (pin + 1) * (pout + 1) * (pout + 1);
  ARENA_ALLOC(D.ops, *mats, cnt);
  BEM_HIP_TRY(hipMemcpyAsync(*mats, e.mats, sizeof(cplx<R>) * cnt, hipMemcpyDeviceToDevice, s));
  return 0;
}

// Expansion order of a level: ceil(k sqrt(3) h) + extra, at least `base`;
// req > 0 fixes it, req < 0 replaces the minimum by -req.
// shift (calibration) moves both terms; the result lies in [1, pmax].
static int auto_order(double k, double h, int req, int base, int extra, int shift, int pmax) {
  pmax = std::max(1, std::min(pmax, MAXP));
  if (req > 0) return std::min(req, pmax);
  if (req < 0) base = -req;
  double d = sqrt(3.0) * h;
  int p = (int)ceil(k * d) + extra + shift;
  return std::min(std::max(std::max(p, base + shift), 1), pmax);
}

// Tiles of a grouped op: (group, first pair, pair count, first row)
static void make_tiles(const std::vector<int>& gstart, int rows, int CT, int RT,
                       std::vector<int>& tg, std::vector<int>& tp0, std::vector<int>& tnp,
                       std::vector<int>& tr0) {
  int ng = (int)gstart.size() - 1;
  for (int gi = 0; gi < ng; ++gi) {
    int a = gstart[gi], b = gstart[gi + 1];
    for (int p0 = a; p0 < b; p0 += CT)
      for (int r0 = 0; r0 < rows; r0 += RT) {
        tg.push_back(gi);
        tp0.push_back(p0);
        tnp.push_back(std::min(CT, b - p0));
        tr0.push_back(r0);
      }
  }
}

constexpr int GEMM_RT = 64;  // output rows per tile

// Pair-tile width of a grouped product: the widest of the supported widths
// (128 is float32 only) that still gives at least ~4 tiles per compute unit
// and fills its tiles at least half on average, else the narrowest.  Narrow
// tiles keep sparse groups (few pairs per translation vector, coarse levels)
// from multiplying mostly-zero columns and spread small launches over more
// compute units.
static int pick_pair_tile(const std::vector<int>& gstart, int rows, bool f32) {
  const int widths[4] = {128, 64, 32, 16};
  const int row_tiles = (rows + GEMM_RT - 1) / GEMM_RT;
  for (int w : widths) {
    if (w == 128 && !f32) continue;
    int64_t col_tiles = 0, pairs = 0;
    for (size_t g = 0; g + 1 < gstart.size(); ++g) {
      col_tiles += (gstart[g + 1] - gstart[g] + w - 1) / w;
      pairs += gstart[g + 1] - gstart[g];
    }
    if (col_tiles * row_tiles >= 1024 && 2 * pairs >= col_tiles * w) return w;
  }
  return 16;
}

__global__ void k_group_starts(const int* __restrict__ code, int np, int ngroups,
                               int* __restrict__ cnt) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < np) atomicAdd(&cnt[code[t]], 1);
}

__global__ void k_sort_keys(const int* __restrict__ code, const int* __restrict__ dst, int np,
                            int dbits, uint64_t* __restrict__ keys, int* __restrict__ idx) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np) return;
  keys[t] = ((uint64_t)code[t] << dbits) | (uint64_t)dst[t];
  idx[t] = t;
}

__global__ void k_permute3(const int* __restrict__ idx, int np, const int* __restrict__ a,
                           const int* __restrict__ b, const int* __restrict__ c,
                           int* __restrict__ ao, int* __restrict__ bo, int* __restrict__ co) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np) return;
  int i = idx[t];
  ao[t] = a[i];
  bo[t] = b[i];
  co[t] = c[i];
}

__global__ void k_octant_pairs(const uint64_t* __restrict__ ckeys, const int* __restrict__ parent,
                               int nbox, int* __restrict__ dst, int* __restrict__ src,
                               int* __restrict__ code) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nbox) return;
  dst[c] = parent[c];
  src[c] = c;
  code[c] = (int)(ckeys[c] & 7);
}

// (ancestor at `depth` levels up, leaf, position code of the leaf inside the
// ancestor: the low 3 depth bits of its Morton key)
struct ParentChain {
  const int* par[MAX_DIRECT];  // par[i]: parent index of the boxes of level L - i
};
__global__ void k_ancestor_pairs(const uint64_t* __restrict__ leaf_keys, const ParentChain pc,
                                 int depth, int nleaf, int* __restrict__ dst,
                                 int* __restrict__ src, int* __restrict__ code) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  int a = b;
  for (int i = 0; i < depth; ++i) a = pc.par[i][a];
  dst[b] = a;
  src[b] = b;
  code[b] = (int)(leaf_keys[b] & ((1ull << (3 * depth)) - 1));
}

// Group (dst, src, code) pairs by code (stable by dst), upload tiles for the
// forward and adjoint directions.  code < ngroups.
template <typename R>
static int finish_grouped(GroupedOp<R>& op, int* d0, int* s0, int* c0, int np, int ngroups,
                          const std::vector<int>& slot_of_group, DevArena& arena,
                          DevArena& scratch, hipStream_t s, int force_ct = 0) {
  op.n_pairs = np;
  int dbits = 1;
  while ((1 << dbits) < 1 << 30 && (1 << dbits) <= np + 1) ++dbits;
  dbits = 30;
  uint64_t* keys;
  int* idx;
  ARENA_ALLOC(scratch, keys, np);
  ARENA_ALLOC(scratch, idx, np);
  if (np > 0) {
    hipLaunchKernelGGL(k_sort_keys, dim3(ceil_div(np, 256)), dim3(256), 0, s, c0, d0, np, dbits,
                       keys, idx);
    BEM_LAUNCH_CHECK();
    int cbits = 1;
    while ((1 << cbits) < ngroups) ++cbits;
    int r = sort_pairs_u64(keys, idx, np, dbits + cbits, scratch, s);
    if (r) return r;
  }
  int* code_sorted;
  ARENA_ALLOC(arena, op.pair_dst, np);
  ARENA_ALLOC(arena, op.pair_src, np);
  ARENA_ALLOC(scratch, code_sorted, np);
  if (np > 0) {
    hipLaunchKernelGGL(k_permute3, dim3(ceil_div(np, 256)), dim3(256), 0, s, idx, np, d0, s0, c0,
                       op.pair_dst, op.pair_src, code_sorted);
    BEM_LAUNCH_CHECK();
  }
  int* gcnt;
  ARENA_ALLOC(scratch, gcnt, ngroups);
  BEM_HIP_TRY(hipMemsetAsync(gcnt, 0, sizeof(int) * ngroups, s));
  if (np > 0) {
    hipLaunchKernelGGL(k_group_starts, dim3(ceil_div(np, 256)), dim3(256), 0, s, code_sorted, np,
                       ngroups, gcnt);
    BEM_LAUNCH_CHECK();
  }
  std::vector<int> hcnt(ngroups);
  BEM_HIP_TRY(hipMemcpyAsync(hcnt.data(), gcnt, sizeof(int) * ngroups, hipMemcpyDeviceToHost, s));
  BEM_HIP_TRY(hipStreamSynchronize(s));
  std::vector<int> gstart(ngroups + 1, 0);
  for (int g = 0; g < ngroups; ++g) gstart[g + 1] = gstart[g] + hcnt[g];
  op.gstart_h = gstart;
  std::vector<int> tg, tp0, tnp, tr0, ta, tap0, tanp, tar0;
  op.ct = force_ct ? force_ct : pick_pair_tile(gstart, op.rows, sizeof(R) == 4);
  op.ct_adj = force_ct ? force_ct : pick_pair_tile(gstart, op.cols, sizeof(R) == 4);
  make_tiles(gstart, op.rows, op.ct, GEMM_RT, tg, tp0, tnp, tr0);
  make_tiles(gstart, op.cols, op.ct_adj, GEMM_RT, ta, tap0, tanp, tar0);
  op.n_tiles = (int)tg.size();
  op.n_tiles_adj = (int)ta.size();
  ARENA_ALLOC(arena, op.tile_group, op.n_tiles);
  ARENA_ALLOC(arena, op.tile_pair0, op.n_tiles);
  ARENA_ALLOC(arena, op.tile_npairs, op.n_tiles);
  ARENA_ALLOC(arena, op.tile_row0, op.n_tiles);
  ARENA_ALLOC(arena, op.tile_group_adj, op.n_tiles_adj);
  ARENA_ALLOC(arena, op.tile_pair0_adj, op.n_tiles_adj);
  ARENA_ALLOC(arena, op.tile_npairs_adj, op.n_tiles_adj);
  ARENA_ALLOC(arena, op.tile_row0_adj, op.n_tiles_adj);
  ARENA_ALLOC(arena, op.group_slot, ngroups);
  auto up = [&](int* d, const std::vector<int>& h) -> int {
    if (!h.empty())
      BEM_HIP_TRY(hipMemcpyAsync(d, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice, s));
    return 0;
  };
  int r = 0;
  if ((r = up(op.tile_group, tg)) || (r = up(op.tile_pair0, tp0)) || (r = up(op.tile_npairs, tnp)) ||
      (r = up(op.tile_row0, tr0)) || (r = up(op.tile_group_adj, ta)) ||
      (r = up(op.tile_pair0_adj, tap0)) || (r = up(op.tile_npairs_adj, tanp)) ||
      (r = up(op.tile_row0_adj, tar0)) || (r = up(op.group_slot, slot_of_group)))
    return r;
  op.pair_dst_adj = op.pair_src;
  op.pair_src_adj = op.pair_dst;
  BEM_HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

// Forward tiles of a grouped op rebuilt for pair-tile width ct (16, 32, 64,
// or 128 in float32) from its group ranges; the pairs, operators and
// reduction lists are unchanged.
template <typename R>
int retile_forward(GroupedOp<R>& op, int ct, DevArena& arena, hipStream_t s) {
  if (op.gstart_h.empty() || op.ct == ct) return 0;
  std::vector<int> tg, tp0, tnp, tr0;
  make_tiles(op.gstart_h, op.rows, ct, GEMM_RT, tg, tp0, tnp, tr0);
  const int nt = (int)tg.size();
  int *g, *p0, *np, *r0;
  ARENA_ALLOC(arena, g, nt);
  ARENA_ALLOC(arena, p0, nt);
  ARENA_ALLOC(arena, np, nt);
  ARENA_ALLOC(arena, r0, nt);
  if (nt > 0) {
    BEM_HIP_TRY(hipMemcpyAsync(g, tg.data(), sizeof(int) * nt, hipMemcpyHostToDevice, s));
    BEM_HIP_TRY(hipMemcpyAsync(p0, tp0.data(), sizeof(int) * nt, hipMemcpyHostToDevice, s));
    BEM_HIP_TRY(hipMemcpyAsync(np, tnp.data(), sizeof(int) * nt, hipMemcpyHostToDevice, s));
    BEM_HIP_TRY(hipMemcpyAsync(r0, tr0.data(), sizeof(int) * nt, hipMemcpyHostToDevice, s));
  }
  BEM_HIP_TRY(hipStreamSynchronize(s));
  op.tile_group = g;
  op.tile_pair0 = p0;
  op.tile_npairs = np;
  op.tile_row0 = r0;
  op.n_tiles = nt;
  op.ct = ct;
  return 0;
}
template int retile_forward<float>(GroupedOp<float>&, int, DevArena&, hipStream_t);
template int retile_forward<double>(GroupedOp<double>&, int, DevArena&, hipStream_t);

__global__ void k_count_boxes(const int* __restrict__ box, int np, int* __restrict__ cnt) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < np) atomicAdd(&cnt[box[t]], 1);
}

__global__ void k_keys_from_box(const int* __restrict__ box, int np, uint64_t* __restrict__ keys,
                                int* __restrict__ idx) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np) return;
  keys[t] = (uint64_t)box[t];
  idx[t] = t;
}

// CSR lists of pair indices per box (ascending pair index within a box), by
// destination (forward) and by source (adjoint).
static int pairs_by_box(const int* box, int np, int nbox, int** ptr_out, int** pairs_out,
                        DevArena& arena, DevArena& scratch, hipStream_t s) {
  int *cnt, *ptr, *pairs;
  uint64_t* keys;
  ARENA_ALLOC(scratch, cnt, nbox);
  ARENA_ALLOC(arena, ptr, nbox + 1);
  ARENA_ALLOC(arena, pairs, np);
  ARENA_ALLOC(scratch, keys, np);
  BEM_HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(int) * nbox, s));
  if (np > 0) {
    hipLaunchKernelGGL(k_count_boxes, dim3(ceil_div(np, 256)), dim3(256), 0, s, box, np, cnt);
    BEM_LAUNCH_CHECK();
  }
  int total = 0;
  int r = exclusive_scan(cnt, ptr, nbox, &total, scratch, s);
  if (r) return r;
  BEM_HIP_TRY(hipMemcpyAsync(ptr + nbox, &total, sizeof(int), hipMemcpyHostToDevice, s));
  if (np > 0) {
    hipLaunchKernelGGL(k_keys_from_box, dim3(ceil_div(np, 256)), dim3(256), 0, s, box, np, keys,
                       pairs);
    BEM_LAUNCH_CHECK();
    int nbits = 1;
    while ((1 << nbits) <= nbox) ++nbits;
    r = sort_pairs_u64(keys, pairs, np, nbits, scratch, s);
    if (r) return r;
  }
  BEM_HIP_TRY(hipStreamSynchronize(s));
  *ptr_out = ptr;
  *pairs_out = pairs;
  return 0;
}

template <typename R>
static int build_reduce_lists(GroupedOp<R>& op, int nbox, DevArena& arena, DevArena& scratch,
                              hipStream_t s) {
  int r = pairs_by_box(op.pair_dst, op.n_pairs, nbox, &op.red_ptr, &op.red_pairs, arena, scratch, s);
  if (r) return r;
  r = pairs_by_box(op.pair_src, op.n_pairs, nbox, &op.red_ptr_adj, &op.red_pairs_adj, arena,
                   scratch, s);
  if (r) return r;
  op.n_red = op.n_red_adj = nbox;
  return 0;
}

// Directional derivative coefficients of the regular wave functions up to
// order p (the l = 1 terms of the translation formula, output order p + 1),
// as interleaved complex pairs: see cmu() for their use.
int derivative_table(Problem& P, int p, std::vector<double>& gc, DevArena& scratch,
                     hipStream_t s) {
  const int P1 = (p + 2) * (p + 2), Pc = (p + 1) * (p + 1);
  GauntSet G1;
  int r = make_gaunt(p, p + 1, 1, G1, scratch, s);
  if (r) return r;
  const int J = std::min(p, p + 1) + 1;
  std::vector<double> hg((size_t)Pc * P1 * J);
  BEM_HIP_TRY(hipMemcpyAsync(hg.data(), G1.d, sizeof(double) * hg.size(), hipMemcpyDeviceToHost, s));
  BEM_HIP_TRY(hipStreamSynchronize(s));
  gc.assign((size_t)Pc * 2 * 3 * 2, 0.0);
  for (int nn = 0; nn <= p; ++nn)
    for (int m = -nn; m <= nn; ++m)
      for (int sg = 0; sg < 2; ++sg) {
        int n2 = sg ? nn + 1 : nn - 1;
        if (n2 < 0) continue;
        for (int mu = -1; mu <= 1; ++mu) {
          int m2 = m - mu;
          if (abs(m2) > n2) continue;
          // l = 1 = |nn - n2| + 2j -> j = 0
          double gv = hg[((size_t)cidx(nn, m) * P1 + cidx(n2, m2)) * J + 0];
          std::complex<double> ie = std::pow(std::complex<double>(0, 1), (n2 + 1 - nn) & 3);
          std::complex<double> cf = ie * (FOUR_PI * gv * P.k / 3.0);
          size_t o = ((size_t)(cidx(nn, m) * 2 + sg) * 3 + (mu + 1)) * 2;
          gc[o] = cf.real();
          gc[o + 1] = cf.imag();
        }
      }
  return 0;
}

template <typename R>
static int build_precision(Problem& P, PrecisionData<R>& D, bool is64, DevArena& scratch,
                           hipStream_t s) {
  const int L = P.L;
  const double k = P.k;
  for (int l = 2; l <= L; ++l) {
    const int sh = l == L ? D.shift : D.shift_c;
    D.order[l] = is64 ? auto_order(k, P.h[l], P.order64_req, 12, 8, sh, P.p_max)
                      : auto_order(k, P.h[l], P.order32_req, 7, 3, sh, P.p_max);
    D.ncoef[l] = (D.order[l] + 1) * (D.order[l] + 1);
  }
  // ---- M2L: one matrix per offset present at each level ----
  int64_t cbuf_count = 0;
  for (int l = 2; l <= L; ++l) {
    if (P.vl_n[l] < 0) {  // the tree's V-list of this level, once per problem
      int *vd, *vs, *vc, nv = 0;
      int r = build_vlist(P, l, &vd, &vs, &vc, &nv, scratch, s);
      if (r) return r;
      ARENA_ALLOC(P.arena, P.vl_dst[l], std::max(nv, 1));
      ARENA_ALLOC(P.arena, P.vl_src[l], std::max(nv, 1));
      ARENA_ALLOC(P.arena, P.vl_code[l], std::max(nv, 1));
      if (nv > 0) {
        BEM_HIP_TRY(hipMemcpyAsync(P.vl_dst[l], vd, sizeof(int) * nv, hipMemcpyDeviceToDevice, s));
        BEM_HIP_TRY(hipMemcpyAsync(P.vl_src[l], vs, sizeof(int) * nv, hipMemcpyDeviceToDevice, s));
        BEM_HIP_TRY(hipMemcpyAsync(P.vl_code[l], vc, sizeof(int) * nv, hipMemcpyDeviceToDevice, s));
      }
      P.vl_n[l] = nv;
    }
    int* d0 = P.vl_dst[l];
    int* s0 = P.vl_src[l];
    int* c0 = P.vl_code[l];
    const int np = P.vl_n[l];
    int r = 0;
    P.n_m2l[l] = np;
    int p = D.order[l];
    // present offsets
    std::vector<int> hc(np);
    if (np) BEM_HIP_TRY(hipMemcpyAsync(hc.data(), c0, sizeof(int) * np, hipMemcpyDeviceToHost, s));
    BEM_HIP_TRY(hipStreamSynchronize(s));
    std::vector<int> slot(N_OFFSETS, -1);
    std::vector<double> tv;
    int ns = 0;
    int64_t nfar = 0;
    for (int c : hc) {
      if (slot[c] < 0) slot[c] = 0;
      const int dx = c / 49 - 3, dy = (c / 7) % 7 - 3, dz = c % 7 - 3;
      nfar += std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) == 3;
    }
    P.n_m2l_far[l] = nfar;
    for (int c = 0; c < N_OFFSETS; ++c)
      if (slot[c] == 0) {
        slot[c] = ns++;
        int dx = c / 49 - 3, dy = (c / 7) % 7 - 3, dz = c % 7 - 3;
        tv.push_back(dx * P.h[l]);
        tv.push_back(dy * P.h[l]);
        tv.push_back(dz * P.h[l]);
      }
    GroupedOp<R>& op = D.m2l[l];
    op.rows = op.cols = D.ncoef[l];
    op.n_slots = ns;
    op.group_kc = nullptr;
    if (ns > 0) {
      // L~ = f_n' (S|R) M~ f_n  (locals times f, multipoles over f)
      std::vector<double> rs = coef_scale(p, k * P.h[l], +1), cs = coef_scale(p, k * P.h[l], +1);
      r = cached_translations<R>(P, D, 0 * 64 + l, ns, tv, 1, p, p, rs, cs, &op.mats, scratch, s);
      if (r) return r;
      r = cut_far_translations<R>(op, p, D.far_cut, N_OFFSETS, 7, slot, D.ops, scratch, s);
      if (r) return r;
      const int64_t tot = (int64_t)ns * op.rows * op.cols;
      ARENA_ALLOC(D.ops, op.mats_h, tot);
      hipLaunchKernelGGL(k_conj_transpose<R>, dim3(ceil_div(tot, 256)), dim3(256), 0, s,
                         op.mats, ns, op.rows, op.cols, op.mats_h);
      BEM_LAUNCH_CHECK();
    }
    r = finish_grouped<R>(op, d0, s0, c0, np, N_OFFSETS, slot, D.ops, scratch, s);
    if (r) return r;
    r = build_reduce_lists<R>(op, P.nbox[l], D.ops, scratch, s);
    if (r) return r;
    if (l < L) {
      D.cbuf_off[l] = cbuf_count;
      cbuf_count += (int64_t)np * D.ncoef[l];
    } else {
      D.cbufL_count = (int64_t)np * D.ncoef[l];
    }
  }
  // ---- M2M (child level l -> parent l-1) and L2L (l-1 -> l), l >= 3 ----
  for (int l = 3; l <= L; ++l) {
    int nb = P.nbox[l];
    int *d0, *s0, *c0;
    ARENA_ALLOC(scratch, d0, nb);
    ARENA_ALLOC(scratch, s0, nb);
    ARENA_ALLOC(scratch, c0, nb);
    hipLaunchKernelGGL(k_octant_pairs, dim3(ceil_div(nb, 256)), dim3(256), 0, s, P.box_keys[l],
                       P.box_parent[l], nb, d0, s0, c0);
    BEM_LAUNCH_CHECK();
    int pc = D.order[l], pp = D.order[l - 1];
    std::vector<int> slot(8);
    std::vector<double> tv_m2m, tv_l2l;
    for (int o = 0; o < 8; ++o) {
      slot[o] = o;
      // child centre minus parent centre = (+-1/2 h_l per axis)
      double ox = (((o >> 2) & 1) ? 0.5 : -0.5) * P.h[l];
      double oy = (((o >> 1) & 1) ? 0.5 : -0.5) * P.h[l];
      double oz = ((o & 1) ? 0.5 : -0.5) * P.h[l];
      tv_m2m.push_back(-ox);  // parent - child
      tv_m2m.push_back(-oy);
      tv_m2m.push_back(-oz);
      tv_l2l.push_back(ox);  // child - parent
      tv_l2l.push_back(oy);
      tv_l2l.push_back(oz);
    }
    // M~_par = (1/f^(l-1)_n') (R|R) f^(l)_n M~_child
    GroupedOp<R>& mm = D.m2m[l];
    mm.rows = D.ncoef[l - 1];
    mm.cols = D.ncoef[l];
    mm.n_slots = 8;
    std::vector<double> rs = coef_scale(pp, k * P.h[l - 1], -1), cs = coef_scale(pc, k * P.h[l], +1);
    int r = cached_translations<R>(P, D, 1 * 64 + l, 8, tv_m2m, 0, pc, pp, rs, cs, &mm.mats,
                                   scratch, s);
    if (r) return r;
    r = finish_grouped<R>(mm, d0, s0, c0, nb, 8, slot, D.ops, scratch, s);
    if (r) return r;
    // L~_child = f^(l)_n' (R|R) (1/f^(l-1)_n) L~_par ; pairs (dst child, src parent)
    GroupedOp<R>& ll = D.l2l[l];
    ll.rows = D.ncoef[l];
    ll.cols = D.ncoef[l - 1];
    ll.n_slots = 8;
    rs = coef_scale(pc, k * P.h[l], +1);
    cs = coef_scale(pp, k * P.h[l - 1], -1);
    r = cached_translations<R>(P, D, 2 * 64 + l, 8, tv_l2l, 0, pp, pc, rs, cs, &ll.mats, scratch,
                               s);
    if (r) return r;
    r = finish_grouped<R>(ll, s0, d0, c0, nb, 8, slot, D.ops, scratch, s);
    if (r) return r;
  }
  // ---- direct translations between the leaves and the MAX_DIRECT levels
  // above them (leaf -> ancestor for the upward pass, ancestor -> leaf for
  // the downward one): one launch per pass instead of a chain of dependent
  // level-by-level launches.  A depth is used while its 8^depth operators
  // stay within DIRECT_BYTES; the levels above are chained. ----
  D.n_direct = 0;
  for (int d = 1; d <= MAX_DIRECT && L - d >= 2; ++d) {
    const int a = L - d, ng = 1 << (3 * d), pL = D.order[L], pa = D.order[a];
    const int64_t bytes = 2 * (int64_t)ng * D.ncoef[L] * D.ncoef[a] * (int64_t)sizeof(cplx<R>);
    if (bytes > DIRECT_BYTES) break;
    const int nb = P.nbox[L];
    int *d0, *s0, *c0;
    ARENA_ALLOC(scratch, d0, nb);
    ARENA_ALLOC(scratch, s0, nb);
    ARENA_ALLOC(scratch, c0, nb);
    ParentChain pcn{};
    for (int i = 0; i < d; ++i) pcn.par[i] = P.box_parent[L - i];
    hipLaunchKernelGGL(k_ancestor_pairs, dim3(ceil_div(nb, 256)), dim3(256), 0, s, P.box_keys[L],
                       pcn, d, nb, d0, s0, c0);
    BEM_LAUNCH_CHECK();
    std::vector<int> slot(ng);
    std::vector<double> tv_up, tv_down;
    for (int c = 0; c < ng; ++c) {
      slot[c] = c;
      // leaf centre minus ancestor centre: the steps from level a + 1 down
      double o[3] = {0, 0, 0};
      for (int i = 1; i <= d; ++i) {
        const int dig = (c >> (3 * (d - i))) & 7;
        for (int ax = 0; ax < 3; ++ax)
          o[ax] += (((dig >> (2 - ax)) & 1) ? 0.5 : -0.5) * P.h[a + i];
      }
      for (int ax = 0; ax < 3; ++ax) {
        tv_up.push_back(-o[ax]);   // ancestor - leaf
        tv_down.push_back(o[ax]);  // leaf - ancestor
      }
    }
    GroupedOp<R>& mu = D.m2m_dir[d];  // M~_anc += (1/f^(a)) (R|R) f^(L) M~_leaf
    mu.rows = D.ncoef[a];
    mu.cols = D.ncoef[L];
    mu.n_slots = ng;
    std::vector<double> rs = coef_scale(pa, k * P.h[a], -1), cs = coef_scale(pL, k * P.h[L], +1);
    int r = cached_translations<R>(P, D, 3 * 64 + a, ng, tv_up, 0, pL, pa, rs, cs, &mu.mats,
                                   scratch, s);
    if (r) return r;
    // few pairs per position code: 16-pair tiles (all depths share a launch)
    r = finish_grouped<R>(mu, d0, s0, c0, nb, ng, slot, D.ops, scratch, s, 16);
    if (r) return r;
    GroupedOp<R>& ld = D.l2l_dir[d];  // L~_leaf += f^(L) (R|R) (1/f^(a)) L~_anc
    ld.rows = D.ncoef[L];
    ld.cols = D.ncoef[a];
    ld.n_slots = ng;
    rs = coef_scale(pL, k * P.h[L], +1);
    cs = coef_scale(pa, k * P.h[a], -1);
    r = cached_translations<R>(P, D, 4 * 64 + a, ng, tv_down, 0, pa, pL, rs, cs, &ld.mats,
                               scratch, s);
    if (r) return r;
    r = finish_grouped<R>(ld, s0, d0, c0, nb, ng, slot, D.ops, scratch, s, 16);
    if (r) return r;
    D.n_direct = d;
  }
  D.cbuf_count = cbuf_count;
  // ---- P2M and L2P per element (kept while the leaf order stays) ----
  if (D.leaf_order != D.order[L] || !D.p2m) {
    int p = D.order[L];
    D.leafops.release();
    D.p2m = D.p2m_p = D.l2p = nullptr;
    D.leaf_order = -1;
    int P1 = (p + 2) * (p + 2);
    int Pc = (p + 1) * (p + 1);
    std::vector<double> gc;
    int r = derivative_table(P, p, gc, scratch, s);
    if (r) return r;
    double *dgc, *dfinv, *dlo;
    ARENA_ALLOC(scratch, dgc, gc.size());
    ARENA_ALLOC(scratch, dfinv, p + 1);
    ARENA_ALLOC(scratch, dlo, 3);
    std::vector<double> finv(p + 1);
    double v = 1.0;
    for (int nn = 0; nn <= p; ++nn) {
      if (nn > 0) v *= k * P.h[L] / (2.0 * nn + 1.0);
      finv[nn] = 1.0 / v;
    }
    BEM_HIP_TRY(hipMemcpyAsync(dgc, gc.data(), sizeof(double) * gc.size(), hipMemcpyHostToDevice, s));
    BEM_HIP_TRY(hipMemcpyAsync(dfinv, finv.data(), sizeof(double) * (p + 1), hipMemcpyHostToDevice, s));
    BEM_HIP_TRY(hipMemcpyAsync(dlo, P.lo, sizeof(double) * 3, hipMemcpyHostToDevice, s));
    ARENA_ALLOC(D.leafops, D.p2m, (int64_t)P.n * Pc * 2);
    ARENA_ALLOC(D.leafops, D.l2p, (int64_t)P.n * Pc);
    int64_t chunk = 16384;
    c64* Rbuf;
    double* tmpb;
    ARENA_ALLOC(scratch, Rbuf, chunk * 4 * P1);
    ARENA_ALLOC(scratch, tmpb, chunk * (P1 + 2 * (p + 2)));
    for (int64_t e0 = 0; e0 < P.n; e0 += chunk) {
      int64_t ne = std::min(chunk, P.n - e0);
      hipLaunchKernelGGL(k_p2m_l2p<R>, dim3(ceil_div(ne, 64)), dim3(64), 0, s, P.geo, P.n, e0, ne,
                         P.elem_leaf, P.box_keys[L], L, dlo, P.h[L], k, P.alpha.re, P.alpha.im, p,
                         dgc, dfinv, Rbuf, tmpb, D.p2m, D.l2p);
      BEM_LAUNCH_CHECK();
    }
    ARENA_ALLOC(D.leafops, D.p2m_p, (int64_t)P.n * Pc);
    hipLaunchKernelGGL(k_p_columns<R>, dim3(ceil_div((int64_t)P.n * Pc, 256)), dim3(256), 0, s,
                       D.p2m, (int64_t)P.n * Pc, D.p2m_p);
    BEM_LAUNCH_CHECK();
    BEM_HIP_TRY(hipStreamSynchronize(s));
    D.leaf_order = p;
  }
  return 0;
}

__global__ void k_geo_to_float(const double* __restrict__ g, int64_t cnt, float* __restrict__ f) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < cnt) f[i] = (float)g[i];
}

template <typename R>
int alloc_exec(const Problem& P, const PrecisionData<R>& D, ExecBuf<R>& X, DevArena& arena) {
  int r = 0;
  exec_buffers(P, D, X, [&](auto*& ptr, int64_t count) {
    if (!r) r = arena.alloc((void**)&ptr, sizeof(*ptr) * (size_t)count);
  });
  return r;
}
template int alloc_exec<float>(const Problem&, const PrecisionData<float>&, ExecBuf<float>&,
                               DevArena&);
template int alloc_exec<double>(const Problem&, const PrecisionData<double>&, ExecBuf<double>&,
                                DevArena&);

template <typename R>
int rebuild_precision(Problem& P, PrecisionData<R>& D, int shift_c, int shift_l, hipStream_t s) {
  BEM_HIP_TRY(hipStreamSynchronize(s));  // no product still uses the old data
  PrecisionData<R> keep;
  keep.near_cp = D.near_cp;
  keep.near_cq = D.near_cq;
  keep.neart_cp = D.neart_cp;
  keep.neart_cq = D.neart_cq;
  keep.geo = D.geo;
  D.ops.release();
  D.order = keep.order;
  D.ncoef = keep.ncoef;
  D.m2l = keep.m2l;
  D.m2m = keep.m2m;
  D.l2l = keep.l2l;
  D.n_direct = 0;
  D.m2m_dir = keep.m2m_dir;
  D.l2l_dir = keep.l2l_dir;
  D.cbuf_off = keep.cbuf_off;
  D.cbuf_count = D.cbufL_count = 0;
  D.X = ExecBuf<R>{};
  D.shift = shift_l;
  D.shift_c = shift_c;
  DevArena scratch;
  struct Guard {
    DevArena& a;
    ~Guard() { a.release(); }
  } guard{scratch};
  int r = build_precision<R>(P, D, sizeof(R) == 8, scratch, s);
  if (!r) r = alloc_exec<R>(P, D, D.X, D.ops);
  if (!r) BEM_HIP_TRY(hipStreamSynchronize(s));
  return r;
}
template int rebuild_precision<float>(Problem&, PrecisionData<float>&, int, int, hipStream_t);
template int rebuild_precision<double>(Problem&, PrecisionData<double>&, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// tables of the rotation-based M2L
// ---------------------------------------------------------------------------
// A translation t = |t| Q e_z with Q = R_z(phi) R_y(theta) factors as
//     T(t) = D(Q) T(|t| e_z) D(Q)^H,   D(Q) = Phi d,
// where D(Q)[m][m'] = int conj(Y_n^m(x)) Y_n^m'(Q^T x) dOmega (block-diagonal
// in the degree n: rotating a field rotates its expansions in either kind of
// wave functions alike), Phi = diag(e^{-i m phi}) and d = D(R_y(theta)),
// real with the Condon-Shortley phase; T(|t| e_z) couples equal orders m
// only (Y_l^mu(e_z) = 0 for mu != 0).  The level scaling depends on n alone
// and commutes with D.

// Theta_n^m(x) for one degree and order (the recurrence of theta_table
// along n at fixed m)
__device__ double theta_one(int n, int m, double x) {
  const double s = sqrt(fmax(0.0, 1.0 - x * x));
  double tmm = 0.28209479177387814;
  for (int i = 1; i <= m; ++i) tmm = -sqrt((2.0 * i + 1.0) / (2.0 * i)) * s * tmm;
  if (n == m) return tmm;
  double t0 = tmm, t1 = sqrt(2.0 * m + 3.0) * x * tmm;
  for (int nn = m + 2; nn <= n; ++nn) {
    const double a = sqrt((4.0 * nn * nn - 1.0) / ((double)nn * nn - (double)m * m));
    const double b =
        sqrt(((nn - 1.0) * (nn - 1.0) - (double)m * m) / (4.0 * (nn - 1.0) * (nn - 1.0) - 1.0));
    const double t2 = a * (x * t1 - b * t0);
    t0 = t1;
    t1 = t2;
  }
  return t1;
}

// d_n(theta)[m][m'] by a product rule exact for the integrand (degree <= 2n
// on the sphere): nu >= n + 1 Gauss-Legendre nodes in the cosine of the
// polar angle times nph > 2n equispaced azimuths.  One workgroup per
// (rotation class c, degree n); cs[2c], cs[2c+1] = cos, sin theta_c;
// dtab[c * rot_dsz(p) + rot_doff(n) + (m + n)(2n + 1) + (m' + n)].
constexpr int ROT_QCH = 64;  // quadrature points per LDS chunk
template <typename R>
__global__ void __launch_bounds__(256)
    k_rot_small_d(int p, const double* __restrict__ cs, int nu, int nph,
                  const double* __restrict__ gx, const double* __restrict__ gw,
                  R* __restrict__ dtab) {
  constexpr int EPT = ((2 * ROT_MAXP + 1) * (2 * ROT_MAXP + 1) + 255) / 256;
  __shared__ double ta[ROT_QCH][ROT_MAXP + 1], tb[ROT_QCH][ROT_MAXP + 1];
  __shared__ double fa[ROT_QCH], fb[ROT_QCH], wq[ROT_QCH];
  const int c = blockIdx.x, n = blockIdx.y, s = 2 * n + 1, ne = s * s;
  const double ct = cs[2 * c], st = cs[2 * c + 1];
  const double two_pi = 6.283185307179586;
  double acc[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) acc[i] = 0.0;
  const int nq = nu * nph;
  for (int q0 = 0; q0 < nq; q0 += ROT_QCH) {
    const int nqc = min(ROT_QCH, nq - q0);
    // Theta_n^|m| at the nodes x and at R_y(theta)^T x, with the azimuths
    for (int it = threadIdx.x; it < 2 * nqc * (n + 1); it += blockDim.x) {
      const int qq = it % nqc, rest = it / nqc, mm = rest % (n + 1), rot = rest / (n + 1);
      const int q = q0 + qq, iu = q / nph, ip = q % nph;
      const double u = gx[iu], az = two_pi * ip / nph;
      double x = u, a = az;
      if (rot) {
        const double sn = sqrt(fmax(0.0, 1.0 - u * u));
        const double vx = sn * cos(az), vy = sn * sin(az);
        x = fmin(1.0, fmax(-1.0, st * vx + ct * u));
        a = atan2(vy, ct * vx - st * u);
      }
      (rot ? tb : ta)[qq][mm] = theta_one(n, mm, x);
      if (mm == 0) {
        (rot ? fb : fa)[qq] = a;
        if (!rot) wq[qq] = gw[iu] * two_pi / nph;
      }
    }
    __syncthreads();
    // Re[conj(Y_n^m(x)) Y_n^m'(x')], Y_n^m = sigma_m Theta_n^|m| e^{i m phi}
    // with sigma_m = (-1)^m for m < 0
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + 256 * i;
      if (e < ne) {
        const int m = e / s - n, m2 = e % s - n;
        const int am = abs(m), am2 = abs(m2);
        double sum = 0.0;
        for (int qq = 0; qq < nqc; ++qq)
          sum += wq[qq] * ta[qq][am] * tb[qq][am2] * cos(m2 * fb[qq] - m * fa[qq]);
        const bool neg = ((m < 0) && (am & 1)) != ((m2 < 0) && (am2 & 1));
        acc[i] += neg ? -sum : sum;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + 256 * i;
    if (e < ne) dtab[(int64_t)c * rot_dsz(p) + rot_doff(n) + e] = (R)acc[i];
  }
}

// Coaxial blocks from the dense translations along e_z (one per distance
// class, rows = outputs): coax[c][coff(m) + i s + j] = T_c[(|m|+i, m)][(|m|+j, m)]
// with s = p + 1 - |m|, and coax_h the block-wise conjugate transposes.
template <typename R>
__global__ void k_rot_coax(int p, int ndist, const cplx<R>* __restrict__ dense,
                           cplx<R>* __restrict__ coax, cplx<R>* __restrict__ coax_h) {
  const int csz = rot_csz(p), nc = (p + 1) * (p + 1);
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)ndist * csz) return;
  const int c = (int)(t / csz), e = (int)(t % csz);
  int m = -p;
  while (m < p && rot_coff(p, m + 1) <= e) ++m;
  const int am = m < 0 ? -m : m, s = p + 1 - am, o = e - rot_coff(p, m);
  const int i = o / s, j = o % s;
  const cplx<R>* T = dense + (int64_t)c * nc * nc;
  const int ri = cidx(am + i, m), rj = cidx(am + j, m);
  coax[t] = T[(int64_t)ri * nc + rj];
  const cplx<R> v = T[(int64_t)rj * nc + ri];
  coax_h[t] = mk<R>(v.re, -v.im);
}

// Matrix-core layout of the degree blocks: out[c][o][rot_dpoff(n) + chunk]
// with o = 0 for d_n, 1 for d_n^T (from dtab, rot_dsz(p) per class).
template <typename R>
__global__ void k_rot_pad_d(int p, int nth, const R* __restrict__ dtab, R* __restrict__ out) {
  const int dp = rot_dpsz(p);
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)nth * 2 * dp) return;
  const int c = (int)(t / (2 * dp)), o = (int)(t / dp % 2), e = (int)(t % dp);
  int n = 0;
  while (n < p && rot_dpoff(n + 1) <= e) ++n;
  const int s = 2 * n + 1, nks = rot_nks(s), l = e - rot_dpoff(n);
  const int chunk = l >> 6, lane = l & 63, mt = chunk / nks, ks = chunk % nks;
  const int row = 16 * mt + (lane & 15), col = 4 * ks + (lane >> 4);
  R v = 0;
  if (row < s && col < s) {
    const R* A = dtab + (int64_t)c * rot_dsz(p) + rot_doff(n);
    v = o ? A[col * s + row] : A[row * s + col];
  }
  out[t] = v;
}

// Matrix-core layout of the coaxial blocks: out[c][rot_cpoff(p, m) + chunk]
// (from coax, rot_csz(p) per class)
template <typename R>
__global__ void k_rot_pad_c(int p, int ndist, const cplx<R>* __restrict__ coax,
                            cplx<R>* __restrict__ out) {
  const int cp = rot_cpsz(p);
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)ndist * cp) return;
  const int c = (int)(t / cp), e = (int)(t % cp);
  int m = -p;
  while (m < p && rot_cpoff(p, m + 1) <= e) ++m;
  const int s = p + 1 - (m < 0 ? -m : m), nks = rot_nks(s), l = e - rot_cpoff(p, m);
  const int chunk = l >> 6, lane = l & 63, mt = chunk / nks, ks = chunk % nks;
  const int row = 16 * mt + (lane & 15), col = 4 * ks + (lane >> 4);
  cplx<R> v = mk<R>(0, 0);
  if (row < s && col < s) v = coax[(int64_t)c * rot_csz(p) + rot_coff(p, m) + row * s + col];
  out[t] = v;
}

// Rotation tables and tiles of one M2L op at order p on a level of box side
// h, whose offset codes index a width^3 table (offset + width / 2 per axis).
template <typename R>
static int rot_tables(Problem& P, GroupedOp<R>& op, int p, double h, int width, DevArena& keep,
                      hipStream_t s) {
  const int ncodes = width * width * width, off = width / 2;
  if (op.rot_ready || op.n_pairs == 0 || p > ROT_MAXP || (int)op.gstart_h.size() != ncodes + 1)
    return 0;
  DevArena scratch;
  struct Guard {
    DevArena& a;
    ~Guard() { a.release(); }
  } guard{scratch};
  // classes: polar angle by (dz, dx^2 + dy^2), distance by |d|^2 (offsets
  // in box sides; the translation vector is the offset times h)
  std::vector<std::array<int, 3>> tkeys, dkeys;
  std::vector<int> g_theta(ncodes, 0), g_dist(ncodes, 0);
  std::vector<double> cs_theta, tv_dist;
  std::vector<R> phase((size_t)ncodes * (p + 1) * 2, R(0));
  std::vector<int> tg, tp0, tnp;
  for (int c = 0; c < ncodes; ++c) {
    const int a = op.gstart_h[c], b = op.gstart_h[c + 1];
    if (b <= a) continue;
    const int dx = c / (width * width) - off, dy = (c / width) % width - off, dz = c % width - off;
    const int rxy2 = dx * dx + dy * dy, r2 = rxy2 + dz * dz;
    const double r = std::sqrt((double)r2);
    const std::array<int, 3> tk{dz, rxy2, 0}, dk{r2, 0, 0};
    int ti = 0, di = 0;
    while (ti < (int)tkeys.size() && tkeys[ti] != tk) ++ti;
    if (ti == (int)tkeys.size()) {
      tkeys.push_back(tk);
      cs_theta.push_back(dz / r);
      cs_theta.push_back(std::sqrt((double)rxy2) / r);
    }
    while (di < (int)dkeys.size() && dkeys[di] != dk) ++di;
    if (di == (int)dkeys.size()) {
      dkeys.push_back(dk);
      tv_dist.push_back(0.0);
      tv_dist.push_back(0.0);
      tv_dist.push_back(r * h);
    }
    g_theta[c] = ti;
    g_dist[c] = di;
    const double phi = rxy2 > 0 ? std::atan2((double)dy, (double)dx) : 0.0;
    for (int m = 0; m <= p; ++m) {
      phase[((size_t)c * (p + 1) + m) * 2] = (R)std::cos(m * phi);
      phase[((size_t)c * (p + 1) + m) * 2 + 1] = (R)std::sin(m * phi);
    }
    for (int p0 = a; p0 < b; p0 += ROT_CT) {
      tg.push_back(c);
      tp0.push_back(p0);
      tnp.push_back(std::min(ROT_CT, b - p0));
    }
  }
  const int nth = (int)tkeys.size(), ndist = (int)dkeys.size(), nt = (int)tg.size();
  ARENA_ALLOC(keep, op.rot_tile_group, nt);
  ARENA_ALLOC(keep, op.rot_tile_pair0, nt);
  ARENA_ALLOC(keep, op.rot_tile_npairs, nt);
  ARENA_ALLOC(keep, op.rot_theta, ncodes);
  ARENA_ALLOC(keep, op.rot_dist, ncodes);
  ARENA_ALLOC(keep, op.rot_phase, phase.size());
  ARENA_ALLOC(keep, op.rot_dtab, (int64_t)nth * 2 * rot_dpsz(p));
  ARENA_ALLOC(keep, op.rot_coax, (int64_t)ndist * rot_cpsz(p));
  ARENA_ALLOC(keep, op.rot_coax_h, (int64_t)ndist * rot_cpsz(p));
  R* dtab;
  cplx<R>*coax, *coax_h;
  ARENA_ALLOC(scratch, dtab, (int64_t)nth * rot_dsz(p));
  ARENA_ALLOC(scratch, coax, (int64_t)ndist * rot_csz(p));
  ARENA_ALLOC(scratch, coax_h, (int64_t)ndist * rot_csz(p));
  auto up = [&](void* d, const void* hp, size_t bytes) -> int {
    if (bytes) BEM_HIP_TRY(hipMemcpyAsync(d, hp, bytes, hipMemcpyHostToDevice, s));
    return 0;
  };
  int r = 0;
  if ((r = up(op.rot_tile_group, tg.data(), sizeof(int) * nt)) ||
      (r = up(op.rot_tile_pair0, tp0.data(), sizeof(int) * nt)) ||
      (r = up(op.rot_tile_npairs, tnp.data(), sizeof(int) * nt)) ||
      (r = up(op.rot_theta, g_theta.data(), sizeof(int) * ncodes)) ||
      (r = up(op.rot_dist, g_dist.data(), sizeof(int) * ncodes)) ||
      (r = up(op.rot_phase, phase.data(), sizeof(R) * phase.size())))
    return r;
  // rotation blocks by quadrature
  std::vector<double> gx, gw;
  gauss_legendre(p + 1, gx, gw);
  double *dgx, *dgw, *dcs;
  ARENA_ALLOC(scratch, dgx, p + 1);
  ARENA_ALLOC(scratch, dgw, p + 1);
  ARENA_ALLOC(scratch, dcs, cs_theta.size());
  if ((r = up(dgx, gx.data(), sizeof(double) * (p + 1))) ||
      (r = up(dgw, gw.data(), sizeof(double) * (p + 1))) ||
      (r = up(dcs, cs_theta.data(), sizeof(double) * cs_theta.size())))
    return r;
  hipLaunchKernelGGL(k_rot_small_d<R>, dim3(nth, p + 1), dim3(256), 0, s, p, dcs, p + 1,
                     2 * p + 2, dgx, dgw, dtab);
  BEM_LAUNCH_CHECK();
  const int64_t totd = (int64_t)nth * 2 * rot_dpsz(p);
  hipLaunchKernelGGL(k_rot_pad_d<R>, dim3(ceil_div(totd, 256)), dim3(256), 0, s, p, nth, dtab,
                     op.rot_dtab);
  BEM_LAUNCH_CHECK();
  // coaxial blocks: the dense translations along e_z, same level scaling
  std::vector<double> rs = coef_scale(p, P.k * h, +1), cs = coef_scale(p, P.k * h, +1);
  cplx<R>* dense = nullptr;
  r = make_translations<R>(P, scratch, ndist, tv_dist, 1, p, p, rs, cs, &dense, scratch, s);
  if (r) return r;
  const int64_t tot = (int64_t)ndist * rot_csz(p);
  hipLaunchKernelGGL(k_rot_coax<R>, dim3(ceil_div(tot, 256)), dim3(256), 0, s, p, ndist, dense,
                     coax, coax_h);
  BEM_LAUNCH_CHECK();
  const int64_t totc = (int64_t)ndist * rot_cpsz(p);
  hipLaunchKernelGGL(k_rot_pad_c<R>, dim3(ceil_div(totc, 256)), dim3(256), 0, s, p, ndist, coax,
                     op.rot_coax);
  BEM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_rot_pad_c<R>, dim3(ceil_div(totc, 256)), dim3(256), 0, s, p, ndist,
                     coax_h, op.rot_coax_h);
  BEM_LAUNCH_CHECK();
  BEM_HIP_TRY(hipStreamSynchronize(s));
  op.rot_n_tiles = nt;
  op.rot_p = p;
  op.rot_ready = true;
  return 0;
}

template <typename R>
int build_rotations(Problem& P, PrecisionData<R>& D, hipStream_t s) {
  for (int l = 2; l <= P.L; ++l) {
    int r = rot_tables<R>(P, D.m2l[l], D.order[l], P.h[l], 7, D.ops, s);
    if (r) return r;
  }
  return 0;
}
template int build_rotations<float>(Problem&, PrecisionData<float>&, hipStream_t);
template int build_rotations<double>(Problem&, PrecisionData<double>&, hipStream_t);

int build_operators(Problem& P, hipStream_t s) {
  DevArena scratch;
  struct Guard {
    DevArena& a;
    ~Guard() { a.release(); }
  } guard{scratch};
  if (P.L >= 2 && !P.direct) {
    int r = build_precision<double>(P, P.f64, true, scratch, s);
    if (r) return r;
    scratch.release();
    r = build_precision<float>(P, P.f32, false, scratch, s);
    if (r) return r;
  }
  // float geometry copy and work vectors
  int64_t cnt = (int64_t)GEO_COUNT * P.n;
  ARENA_ALLOC(P.arena, P.f32.geo, cnt);
  hipLaunchKernelGGL(k_geo_to_float, dim3(ceil_div(cnt, 256)), dim3(256), 0, s, P.geo, cnt, P.f32.geo);
  BEM_LAUNCH_CHECK();
  P.f64.geo = P.geo;
  {
    int r = alloc_exec<double>(P, P.f64, P.f64.X, P.f64.ops);
    if (!r) r = alloc_exec<float>(P, P.f32, P.f32.X, P.f32.ops);
    if (r) return r;
  }
  if (!P.side || !P.side2) {
    P.own_streams = true;
    BEM_HIP_TRY(hipStreamCreateWithFlags(&P.side, hipStreamNonBlocking));
    BEM_HIP_TRY(hipStreamCreateWithFlags(&P.side2, hipStreamNonBlocking));
  }
  // fork/join events order work between this device's streams only: a
  // device-scope release suffices (no system-scope cache write-back)
  const unsigned evf = hipEventDisableTiming | hipEventReleaseToDevice;
  BEM_HIP_TRY(hipEventCreateWithFlags(&P.ev_fork2, evf));
  BEM_HIP_TRY(hipEventCreateWithFlags(&P.ev_join2, evf));
  BEM_HIP_TRY(hipEventCreateWithFlags(&P.ev_fork, evf));
  BEM_HIP_TRY(hipEventCreateWithFlags(&P.ev_join, evf));
  BEM_HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

// ---------------------------------------------------------------------------
// translations into the boxes of evaluation points (off the boundary)
// ---------------------------------------------------------------------------
// The point boxes share the problem's grid, so the translations have the
// problem's form and orders: M2L from the source boxes of level l (offset
// codes over the PT_W^3 table, translation vector = point box centre minus
// source box centre) and L2L from a point box to its children (octant
// codes, as for the problem's tree).  Pairs come from the host lists.
template <typename R>
int build_point_ops(Problem& P, PrecisionData<R>& D, const PointLists& lists, FieldPoints& F,
                    PointOps<R>& O, hipStream_t s) {
  DevArena scratch;
  struct Guard {
    DevArena& a;
    ~Guard() { a.release(); }
  } guard{scratch};
  const int L = P.L;
  const double k = P.k;
  auto upload = [&](const std::vector<int>& h, int** d) -> int {
    ARENA_ALLOC(scratch, *d, std::max<size_t>(1, h.size()));
    if (!h.empty())
      BEM_HIP_TRY(hipMemcpyAsync(*d, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice, s));
    return 0;
  };
  int64_t cbuf_count = 0;
  for (int l = 2; l <= L; ++l) {
    const int p = D.order[l];
    // ---- M2L: one matrix per offset present ----
    {
      const std::vector<int>& hc = lists.m2l_code[l];
      const int np = (int)hc.size();
      std::vector<int> slot(PT_CODES, -1);
      std::vector<double> tv;
      int ns = 0;
      int64_t nfar = 0;
      for (int c : hc) {
        if (slot[c] < 0) slot[c] = 0;
        const int dx = c / (PT_W * PT_W) - PT_OFF, dy = (c / PT_W) % PT_W - PT_OFF,
                  dz = c % PT_W - PT_OFF;
        nfar += std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) >= 3;
      }
      F.n_m2l_far[l] = nfar;
      for (int c = 0; c < PT_CODES; ++c)
        if (slot[c] == 0) {
          slot[c] = ns++;
          const int dx = c / (PT_W * PT_W) - PT_OFF, dy = (c / PT_W) % PT_W - PT_OFF,
                    dz = c % PT_W - PT_OFF;
          tv.push_back(dx * P.h[l]);
          tv.push_back(dy * P.h[l]);
          tv.push_back(dz * P.h[l]);
        }
      GroupedOp<R>& op = O.m2l[l];
      op.rows = op.cols = D.ncoef[l];
      op.n_slots = ns;
      op.group_kc = nullptr;
      if (ns > 0) {
        // L~ = f_n' (S|R) M~ f_n, as for the problem's own boxes
        std::vector<double> rs = coef_scale(p, k * P.h[l], +1), cs = rs;
        int r = make_translations<R>(P, F.arena, ns, tv, 1, p, p, rs, cs, &op.mats, scratch, s);
        // (no input cut: the cut is calibrated on the product, and points
        // off the boundary lose more accuracy to it, up to 3.6 times the
        // float32 error on the 1280-element sphere)
        if (r) return r;
      }
      int *d0, *s0, *c0;
      int r = upload(lists.m2l_dst[l], &d0);
      if (!r) r = upload(lists.m2l_src[l], &s0);
      if (!r) r = upload(hc, &c0);
      if (!r) r = finish_grouped<R>(op, d0, s0, c0, np, PT_CODES, slot, F.arena, scratch, s);
      if (r) return r;
      F.n_m2l[l] = np;
      if (sizeof(R) == 4) {
        r = build_reduce_lists<R>(op, F.nbox[l], F.arena, scratch, s);
        if (r) return r;
        O.cbuf_off[l] = cbuf_count;
        cbuf_count += (int64_t)np * D.ncoef[l];
      }
    }
    // ---- L2L from the parent point boxes (level l - 1) ----
    if (l >= 3) {
      const int pp = D.order[l - 1];
      std::vector<int> slot(8);
      std::vector<double> tv;
      for (int o = 0; o < 8; ++o) {
        slot[o] = o;
        tv.push_back((((o >> 2) & 1) ? 0.5 : -0.5) * P.h[l]);  // child - parent centre
        tv.push_back((((o >> 1) & 1) ? 0.5 : -0.5) * P.h[l]);
        tv.push_back(((o & 1) ? 0.5 : -0.5) * P.h[l]);
      }
      GroupedOp<R>& ll = O.l2l[l];
      ll.rows = D.ncoef[l];
      ll.cols = D.ncoef[l - 1];
      ll.n_slots = 8;
      std::vector<double> rs = coef_scale(p, k * P.h[l], +1), cs = coef_scale(pp, k * P.h[l - 1], -1);
      int r = make_translations<R>(P, F.arena, 8, tv, 0, pp, p, rs, cs, &ll.mats, scratch, s);
      int *d0, *s0, *c0;
      if (!r) r = upload(lists.l2l_dst[l], &d0);
      if (!r) r = upload(lists.l2l_src[l], &s0);
      if (!r) r = upload(lists.l2l_code[l], &c0);
      if (!r)
        r = finish_grouped<R>(ll, d0, s0, c0, (int)lists.l2l_code[l].size(), 8, slot, F.arena,
                              scratch, s);
      if (r) return r;
    }
    ARENA_ALLOC(F.arena, O.Lc[l], std::max<int64_t>(1, (int64_t)F.nbox[l] * D.ncoef[l]));
    ARENA_ALLOC(F.arena, O.X.M[l], std::max<int64_t>(1, (int64_t)P.nbox[l] * D.ncoef[l]));
  }
  if (sizeof(R) == 4) ARENA_ALLOC(F.arena, O.cbuf, std::max<int64_t>(1, cbuf_count));
  ARENA_ALLOC(F.arena, O.X.ps, P.n);
  ARENA_ALLOC(F.arena, O.X.qs, P.n);
  ARENA_ALLOC(F.arena, O.X.p64s, P.n);
  ARENA_ALLOC(F.arena, O.X.q64s, P.n);
  BEM_HIP_TRY(hipStreamSynchronize(s));
  return 0;
}
template int build_point_ops<float>(Problem&, PrecisionData<float>&, const PointLists&,
                                    FieldPoints&, PointOps<float>&, hipStream_t);

// Rotation-based M2L into the point boxes on the levels where the problem's
// own M2L of the precision is rotation-based (or everywhere the order allows,
// as the plan was asked), over the PT_W^3 offset table.
template <typename R>
int build_point_rotations(Problem& P, PrecisionData<R>& D, FieldPoints& F, PointOps<R>& O,
                          hipStream_t s) {
  if (P.m2l_rot_req == 1) return 0;
  for (int l = 2; l <= P.L; ++l) {
    if (P.m2l_rot_req != 2 && !D.m2l[l].rot_on) continue;
    int r = rot_tables<R>(P, O.m2l[l], D.order[l], P.h[l], PT_W, F.arena, s);
    if (r) return r;
    O.m2l[l].rot_on = O.m2l[l].rot_ready;
  }
  return 0;
}
template int build_point_rotations<float>(Problem&, PrecisionData<float>&, FieldPoints&,
                                          PointOps<float>&, hipStream_t);
template int build_point_rotations<double>(Problem&, PrecisionData<double>&, FieldPoints&,
                                           PointOps<double>&, hipStream_t);
template int build_point_ops<double>(Problem&, PrecisionData<double>&, const PointLists&,
                                     FieldPoints&, PointOps<double>&, hipStream_t);

}  // namespace bemfmm
