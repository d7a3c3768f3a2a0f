// Shared device helpers: complex arithmetic on (re, im) pairs of float or
// double, launch checks and atomics.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

namespace bemfmm {

template <typename T>
struct cplx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T r, T i) {
  cplx<T> c;
  c.re = r;
  c.im = i;
  return c;
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
  return mk<T>(a.re + b.re, a.im + b.im);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) {
  return mk<T>(a.re - b.re, a.im - b.im);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mk<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return mk<T>(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) {
  return mk<T>(a.re * s, a.im * s);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cconj(cplx<T> a) {
  return mk<T>(a.re, -a.im);
}
// acc += a * b
template <typename T>
__host__ __device__ __forceinline__ void cfma(cplx<T>& acc, cplx<T> a, cplx<T> b) {
  // two fused multiply-adds per component (acc += x*y - z*w would take a
  // product, a fused multiply-add and an add)
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ void cfmac(cplx<T>& acc, cplx<T> a, cplx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}

typedef cplx<double> c64;  // complex128
typedef cplx<float> c32;   // complex64

__device__ __forceinline__ void atomic_add_real(float* p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_real(double* p, double v) { unsafeAtomicAdd(p, v); }

template <typename T>
__device__ __forceinline__ void atomic_cadd(cplx<T>* p, cplx<T> v) {
  atomic_add_real(&p->re, v.re);
  atomic_add_real(&p->im, v.im);
}

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace bemfmm

// Launch/return-code helper for host code inside the library: records the
// message and returns BEM_E_HIP from the enclosing function.
#define BEM_HIP_TRY(expr)                                                     \
  do {                                                                        \
    hipError_t _e = (expr);                                                   \
    if (_e != hipSuccess) {                                                   \
      bemfmm::set_error(std::string("HIP error '") + hipGetErrorString(_e) + \
                        "' at " + __FILE__ + ":" + std::to_string(__LINE__)); \
      return -3;                                                              \
    }                                                                         \
  } while (0)

#define BEM_LAUNCH_CHECK() BEM_HIP_TRY(hipGetLastError())

namespace bemfmm {
void set_error(const std::string& msg);
}
