// Pointwise kernel arithmetic of the direct sums: the phase e^{ikr} and
// 1/sqrt, per precision.
#pragma once

#include <hip/hip_runtime.h>

#include "phase64.h"

namespace bemfmm {

// e^{i k r}: float32 uses the hardware sine/cosine, which take the phase in
// turns (k r / 2 pi; here a few radians at most, absolute error ~1e-6, far
// below the float32 operator's tolerance); float64 the reduced Taylor
// evaluation of phase64.h (error < 2e-16, branch-free).
template <typename R>
__device__ __forceinline__ void phase(R r, R k, R k_turns, R* s, R* c);
template <>
__device__ __forceinline__ void phase<float>(float r, float, float k_turns, float* s, float* c) {
  const float t = r * k_turns;
  *s = __builtin_amdgcn_sinf(t);
  *c = __builtin_amdgcn_cosf(t);
}
template <>
__device__ __forceinline__ void phase<double>(double r, double k, double, double* s, double* c) {
  sincos_reduced(k * r, s, c);
}
// 1/sqrt(x) for x well inside the normal range (squared distances between
// distinct rule points and collocation points)
template <typename R>
__device__ __forceinline__ R rsqrt_r(R x);
template <>
__device__ __forceinline__ float rsqrt_r<float>(float x) {
  return __builtin_amdgcn_rsqf(x);
}
// float64: hardware estimate refined by two Newton steps
// y <- y + (y/2)(1 - x y^2) (each doubles the correct bits)
template <>
__device__ __forceinline__ double rsqrt_r<double>(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

}  // namespace bemfmm
