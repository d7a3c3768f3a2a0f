// Radial parts of the spherical wave functions, shared by the operator build
// and the evaluation at points off the boundary.
#pragma once

#include <hip/hip_runtime.h>

namespace bemfmm {

// spherical Bessel j_n(x), n = 0..nmax, by downward (Miller) recurrence of
// the scaled values jt_n = j_n (2n+1)!! / x^n, normalised by j_0 = sin x / x;
// returns j_n in out[n * stride].
__device__ inline void sph_jn(int nmax, double x, double* out, int stride = 1) {
  if (x == 0.0) {
    out[0] = 1.0;
    for (int n = 1; n <= nmax; ++n) out[n * stride] = 0.0;
    return;
  }
  int top = nmax + 24 + (int)(1.5 * x);
  double x2 = x * x;
  double jp1 = 1.0 - x2 / (2.0 * (2 * top + 5)), jn = 1.0 - x2 / (2.0 * (2 * top + 3));
  // jt_{n-1} = jt_n - jt_{n+1} x^2 / ((2n+1)(2n+3))
  for (int n = top; n >= 1; --n) {
    double jm1 = jn - jp1 * x2 / ((2.0 * n + 1.0) * (2.0 * n + 3.0));
    jp1 = jn;
    jn = jm1;
    if (n - 1 <= nmax) out[(n - 1) * stride] = jm1;
  }
  // normalise on j_0 or j_1, whichever is larger (they never vanish together)
  double j0 = (fabs(x) < 1e-4) ? 1.0 - x2 / 6.0 + x2 * x2 / 120.0 : sin(x) / x;
  double scale;
  if (nmax >= 1 && fabs(x) > 1.0) {
    double j1 = (sin(x) / x - cos(x)) / x;
    scale = (fabs(j0) >= fabs(j1)) ? j0 / out[0] : j1 / (out[stride] * x / 3.0);
  } else {
    scale = j0 / out[0];
  }
  double f = 1.0;  // x^n / (2n+1)!!
  for (int n = 0; n <= nmax; ++n) {
    if (n > 0) f *= x / (2.0 * n + 1.0);
    out[n * stride] *= scale * f;
  }
}

}  // namespace bemfmm
