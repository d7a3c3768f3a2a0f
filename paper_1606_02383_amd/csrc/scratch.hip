// The allocation-free product: bem_fmm_matvec with the product buffers (the
// sorted densities and their float64 copies, the near-field sums, the
// multipole and local expansions of every level and the per-pair M2L
// results) laid out in one static device array instead of the plan's own
// buffers.  For callers that cannot allocate device memory (code under HIP
// graph capture, serving loops, harnesses that forbid it).
//
// In host code the array's name stands for a host-side shadow, not a device
// address: its device address is looked up once per device with
// hipGetSymbolAddress (at plan creation, with the plan's device current) and
// only that address is used.  Every call on a device shares that device's
// array, which keeps the last call's contents; the product clears what it
// accumulates into, and calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <type_traits>

#include "plan.h"

namespace bemfmm {

constexpr size_t SCRATCH_BYTES = size_t(64) << 20;  // 64 MiB per device
constexpr int SCRATCH_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// Device address of the current device's array (looked up once per device).
int scratch_init_current_device() {
  int dev = 0;
  BEM_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) {
    set_error("device index beyond the scratch table");
    return -1;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[dev]) return 0;
  void* ptr = nullptr;
  BEM_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) {
    set_error("no device address for the scratch array");
    return -3;
  }
  g_scratch_ptr[dev] = ptr;
  return 0;
}

// The product buffers of precision R laid out from `base` (256-byte aligned
// pieces, the order of exec_buffers); returns the bytes needed.  With base
// null only the size is computed.
template <typename R>
static size_t layout(const Problem& P, const PrecisionData<R>& D, ExecBuf<R>& X,
                     unsigned char* base) {
  size_t off = 0;
  exec_buffers(P, D, X, [&](auto*& ptr, int64_t count) {
    const size_t bytes = ((sizeof(*ptr) * (size_t)count + 255) / 256) * 256;
    ptr = base ? reinterpret_cast<std::remove_reference_t<decltype(ptr)>>(base + off) : nullptr;
    off += bytes;
  });
  return off;
}

template <typename R>
static int apply_noalloc(Problem& P, PrecisionData<R>& D, unsigned char* base, const c64* p,
                         const c64* q, c64* y, int nrhs, hipStream_t s) {
  ExecBuf<R> X;
  const size_t need = layout<R>(P, D, X, nullptr);
  if (need > SCRATCH_BYTES) {
    set_error("problem too large for the allocation-free product: its buffers need " +
              std::to_string(need) + " bytes, the static scratch holds " +
              std::to_string(SCRATCH_BYTES));
    return -1;
  }
  layout<R>(P, D, X, base);
  // no timing events (their creation would allocate): profiling is off for
  // this call
  const bool on = P.prof_on, leaf = P.prof_leaf;
  P.prof_on = P.prof_leaf = false;
  int r = 0;
  for (int c = 0; c < nrhs && !r; ++c) {
    const c64* pc = p ? p + (int64_t)c * P.n : nullptr;
    const c64* qc = q ? q + (int64_t)c * P.n : nullptr;
    r = fmm_apply_x<R>(P, D, X, pc, qc, y + (int64_t)c * P.n, s);
  }
  P.prof_on = on;
  P.prof_leaf = leaf;
  return r;
}

int fmm_matvec_noalloc(Problem& P, int prec, const c64* p, const c64* q, c64* y, int nrhs,
                       hipStream_t s) {
  int dev = 0;
  BEM_HIP_TRY(hipGetDevice(&dev));
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (dev >= 0 && dev < SCRATCH_MAX_DEVICES) base = g_scratch_ptr[dev];
  }
  if (!base) {  // a device the plan was not created on: look it up now
    int r = scratch_init_current_device();
    if (r) return r;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    base = g_scratch_ptr[dev];
  }
  return prec == 0 ? apply_noalloc<double>(P, P.f64, (unsigned char*)base, p, q, y, nrhs, s)
                   : apply_noalloc<float>(P, P.f32, (unsigned char*)base, p, q, y, nrhs, s);
}

}  // namespace bemfmm
