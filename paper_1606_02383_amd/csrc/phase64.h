// Double-precision sine/cosine for the float64 near field (arguments k r
// between neighbouring leaves, well inside |x| < 2^20).
//
// Reduction: x = q pi/2 + r with q the nearest integer to x (2/pi) and pi/2
// split into three parts of 30 significant bits each (Cody and Waite's
// method), so that each q * part is exact for |q| < 2^23 and r carries no
// cancellation error beyond the third part (~1e-35).  On |r| <= pi/4 the
// Taylor series truncated after r^15 (sine) and r^16 (cosine) are accurate
// to below 5e-17; the quadrant q mod 4 then permutes and negates them.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace bemfmm {

__host__ __device__ inline void sincos_reduced(double x, double* s, double* c) {
  const double q = rint(x * 0.63661977236758134);  // nearest multiple of pi/2
  double r = fma(-q, 1.570796325802803, x);
  r = fma(-q, 9.920935791635221e-10, r);
  r = fma(-q, 5.170182981794105e-19, r);
  const double r2 = r * r;
  double ps = -1.0 / 1307674368000.0;
  ps = fma(ps, r2, 1.0 / 6227020800.0);
  ps = fma(ps, r2, -1.0 / 39916800.0);
  ps = fma(ps, r2, 1.0 / 362880.0);
  ps = fma(ps, r2, -1.0 / 5040.0);
  ps = fma(ps, r2, 1.0 / 120.0);
  ps = fma(ps, r2, -1.0 / 6.0);
  const double sr = fma(ps * r2, r, r);
  double pc = 1.0 / 20922789888000.0;
  pc = fma(pc, r2, -1.0 / 87178291200.0);
  pc = fma(pc, r2, 1.0 / 479001600.0);
  pc = fma(pc, r2, -1.0 / 3628800.0);
  pc = fma(pc, r2, 1.0 / 40320.0);
  pc = fma(pc, r2, -1.0 / 720.0);
  pc = fma(pc, r2, 1.0 / 24.0);
  pc = fma(pc, r2, -0.5);
  const double cr = fma(pc, r2, 1.0);
  const int quad = ((int)q) & 3;  // two's complement: also right for q < 0
  const double sv = (quad & 1) ? cr : sr, cv = (quad & 1) ? sr : cr;
  *s = (quad & 2) ? -sv : sv;
  *c = ((quad + 1) & 2) ? -cv : cv;
}

}  // namespace bemfmm
