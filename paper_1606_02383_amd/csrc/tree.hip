// Element geometry, Morton keys, stable radix sort, uniform-depth octree and
// its neighbour (U) and multipole-to-local (V) lists, on the device.
//
// Geometry follows the paper's discretisation (Sec. 2.3): flat triangles,
// constant densities, one collocation point per element (its centroid, our
// reading), unit normal into the fluid (Sec. 2.1), and the 3-point
// degree-2 rule (barycentric (2/3,1/6,1/6) and permutations) for regular
// pairs.  The tree is not specified by the paper (it names an FMM, Sec. 2.3);
// the reading implemented here (bounding cube, 21-bit quantisation, key bit
// layout, stable order, uniform leaf level) is stated in the header of the
// Morton kernels below and must agree bit for bit with the CPU reference.
#include <algorithm>
#include <cmath>
#include <vector>

#include "plan.h"

namespace bemfmm {

int DevArena::alloc(void** p, size_t n) {
  if (n == 0) n = 8;
  n = (n + 255) & ~size_t(255);
  if (hipMalloc(p, n) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    set_error("device allocation of " + std::to_string(n) + " bytes failed");
    return -2;
  }
  ptrs.push_back(*p);
  bytes += (int64_t)n;
  return 0;
}

void DevArena::release() {
  for (void* p : ptrs) (void)hipFree(p);
  ptrs.clear();
  bytes = 0;
}

#define ARENA_ALLOC(arena, ptr, count)                                              \
  do {                                                                              \
    int _r = (arena).alloc((void**)&(ptr), sizeof(*(ptr)) * (size_t)(count));      \
    if (_r) return _r;                                                              \
  } while (0)

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
__global__ void k_geometry(const double* __restrict__ V, const int* __restrict__ T, int64_t n,
                           int64_t n_vert, double* __restrict__ g, int* __restrict__ bad) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  int ia = T[3 * e], ib = T[3 * e + 1], ic = T[3 * e + 2];
  if (ia < 0 || ib < 0 || ic < 0 || ia >= n_vert || ib >= n_vert || ic >= n_vert) {
    atomicOr(bad, 1);
    return;
  }
  double a[3], b[3], c[3];
  for (int d = 0; d < 3; ++d) {
    a[d] = V[3 * ia + d];
    b[d] = V[3 * ib + d];
    c[d] = V[3 * ic + d];
  }
  double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
  double cr[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
  double nrm = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  bool finite = isfinite(nrm);
  for (int d = 0; d < 3; ++d) finite = finite && isfinite(a[d]) && isfinite(b[d]) && isfinite(c[d]);
  if (!finite) atomicOr(bad, 2);
  if (!(nrm > 0.0)) atomicOr(bad, 4);
  double e1 = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  double e2 = sqrt((c[0] - b[0]) * (c[0] - b[0]) + (c[1] - b[1]) * (c[1] - b[1]) +
                   (c[2] - b[2]) * (c[2] - b[2]));
  double e3 = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  double ell = fmax(fmax(e1, e2), e3);
  for (int d = 0; d < 3; ++d) {
    g[(GEO_CX + d) * n + e] = (a[d] + b[d] + c[d]) / 3.0;
    g[(GEO_NX + d) * n + e] = cr[d] / nrm;
    g[(GEO_AX + d) * n + e] = a[d];
    g[(GEO_BX + d) * n + e] = b[d];
    g[(GEO_CXV + d) * n + e] = c[d];
  }
  g[GEO_AREA * n + e] = 0.5 * nrm;
  g[GEO_ELL * n + e] = ell;
  // 3-point rule: barycentric (2/3,1/6,1/6), (1/6,2/3,1/6), (1/6,1/6,2/3)
  const double big = 2.0 / 3.0, sm = 1.0 / 6.0;
  for (int d = 0; d < 3; ++d) {
    g[(GEO_QX0 + d) * n + e] = big * a[d] + sm * b[d] + sm * c[d];
    g[(GEO_QX1 + d) * n + e] = sm * a[d] + big * b[d] + sm * c[d];
    g[(GEO_QX2 + d) * n + e] = sm * a[d] + sm * b[d] + big * c[d];
  }
}

// min/max of the centroids and the largest element edge (one block)
__global__ void k_bbox(const double* __restrict__ g, int64_t n, double* __restrict__ out) {
  __shared__ double smin[3][256], smax[3][256], sell[256];
  int t = threadIdx.x;
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  double el = 0.0;
  for (int64_t i = t; i < n; i += blockDim.x) {
    for (int d = 0; d < 3; ++d) {
      double v = g[(GEO_CX + d) * n + i];
      mn[d] = fmin(mn[d], v);
      mx[d] = fmax(mx[d], v);
    }
    el = fmax(el, g[GEO_ELL * n + i]);
  }
  for (int d = 0; d < 3; ++d) {
    smin[d][t] = mn[d];
    smax[d][t] = mx[d];
  }
  sell[t] = el;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) {
      for (int d = 0; d < 3; ++d) {
        smin[d][t] = fmin(smin[d][t], smin[d][t + s]);
        smax[d][t] = fmax(smax[d][t], smax[d][t + s]);
      }
      sell[t] = fmax(sell[t], sell[t + s]);
    }
    __syncthreads();
  }
  if (t == 0) {
    for (int d = 0; d < 3; ++d) {
      out[d] = smin[d][0];
      out[3 + d] = smax[d][0];
    }
    out[6] = sell[0];
  }
}

// Bounding cube and quantisation scale, each float64 operation rounded on
// its own (no contraction):  R0 = (0.5 * max_a(mx_a - mn_a)) * (1 + 2^-10),
// lo_a = (mn_a + mx_a) / 2 - R0,  s = 2^20 / R0.
__global__ void k_morton_params(const double* __restrict__ bb, double* __restrict__ prm) {
#pragma clang fp contract(off)
  double ext = 0.0;
  for (int d = 0; d < 3; ++d) ext = fmax(ext, bb[3 + d] - bb[d]);
  double R0 = (0.5 * ext) * (1.0 + 0x1p-10);
  for (int d = 0; d < 3; ++d) prm[d] = (bb[d] + bb[3 + d]) / 2.0 - R0;
  prm[3] = 0x1p20 / R0;
  prm[4] = R0;
}

__device__ __forceinline__ uint64_t spread3(uint64_t v) {
  // bit b of v -> bit 3b
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__device__ __forceinline__ uint32_t compact3(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
  v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
  v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
  v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
  v = (v ^ (v >> 32)) & 0x1fffffull;
  return (uint32_t)v;
}

// Morton key of each centroid: q_a = clamp(floor((x_a - lo_a) * s), 0, 2^21-1),
// key bit 3b+2 <- q_x bit b, 3b+1 <- q_y bit b, 3b <- q_z bit b.
__global__ void k_morton_keys(const double* __restrict__ g, int64_t n,
                              const double* __restrict__ prm, uint64_t* __restrict__ keys,
                              int* __restrict__ idx) {
#pragma clang fp contract(off)
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t q[3];
  for (int d = 0; d < 3; ++d) {
    double t = g[(GEO_CX + d) * n + i] - prm[d];
    double u = t * prm[3];
    double f = floor(u);
    int64_t qi = (int64_t)f;
    if (!(f >= 0.0)) qi = 0;
    if (f > 2097151.0) qi = 2097151;
    q[d] = (uint64_t)qi;
  }
  keys[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
  idx[i] = (int)i;
}

// ---------------------------------------------------------------------------
// scans and a stable LSD radix sort (4-bit digits)
// ---------------------------------------------------------------------------
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__device__ int block_exclusive_scan_256(int v, int* sh) {
  // returns exclusive prefix of v over the 256 threads; sh has 256 ints
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int add = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  int incl = sh[t];
  __syncthreads();
  return incl - v;
}

__global__ void k_scan_tiles(const int* __restrict__ in, int* __restrict__ out, int n,
                             int* __restrict__ tile_sums) {
  __shared__ int sh[SCAN_BLOCK];
  int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int vals[SCAN_ITEMS];
  int s = 0;
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    int i = base + j;
    vals[j] = (i < n) ? in[i] : 0;
    s += vals[j];
  }
  int pre = block_exclusive_scan_256(s, sh);
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    int i = base + j;
    if (i < n) out[i] = pre;
    pre += vals[j];
  }
  if (threadIdx.x == SCAN_BLOCK - 1) tile_sums[blockIdx.x] = pre;
}

__global__ void k_scan_add(int* __restrict__ out, int n, const int* __restrict__ tile_off) {
  int i = blockIdx.x * SCAN_TILE + threadIdx.x;
  int add = tile_off[blockIdx.x];
  for (int j = 0; j < SCAN_ITEMS; ++j, i += SCAN_BLOCK)
    if (i < n) out[i] += add;
}

static int scan_rec(const int* in, int* out, int n, DevArena& scratch, hipStream_t s) {
  int ntiles = ceil_div(n, SCAN_TILE);
  int* sums;
  int* offs;
  ARENA_ALLOC(scratch, sums, ntiles + 1);
  ARENA_ALLOC(scratch, offs, ntiles + 1);
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(SCAN_BLOCK), 0, s, in, out, n, sums);
  BEM_LAUNCH_CHECK();
  if (ntiles > 1) {
    int r = scan_rec(sums, offs, ntiles, scratch, s);
    if (r) return r;
    hipLaunchKernelGGL(k_scan_add, dim3(ntiles), dim3(SCAN_BLOCK), 0, s, out, n, offs);
    BEM_LAUNCH_CHECK();
  }
  return 0;
}

// out = exclusive scan of in (n entries); *total (host) = sum of in.
int exclusive_scan(const int* in, int* out, int n, int* total, DevArena& scratch, hipStream_t s) {
  if (n <= 0) {
    if (total) *total = 0;
    return 0;
  }
  int r = scan_rec(in, out, n, scratch, s);
  if (r) return r;
  if (total) {
    int last_in = 0, last_out = 0;
    BEM_HIP_TRY(hipMemcpyAsync(&last_in, in + n - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    BEM_HIP_TRY(hipMemcpyAsync(&last_out, out + n - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    BEM_HIP_TRY(hipStreamSynchronize(s));
    *total = last_in + last_out;
  }
  return 0;
}

constexpr int RADIX_BLOCK = 256;

__global__ void k_radix_hist(const uint64_t* __restrict__ keys, int n, int shift,
                             int* __restrict__ hist, int nblk) {
  __shared__ int cnt[16];
  if (threadIdx.x < 16) cnt[threadIdx.x] = 0;
  __syncthreads();
  int i = blockIdx.x * RADIX_BLOCK + threadIdx.x;
  if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 15], 1);
  __syncthreads();
  if (threadIdx.x < 16) hist[threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void k_radix_scatter(const uint64_t* __restrict__ keys, const int* __restrict__ vals,
                                int n, int shift, const int* __restrict__ offs, int nblk,
                                uint64_t* __restrict__ keys_out, int* __restrict__ vals_out) {
  __shared__ int wave_cnt[RADIX_BLOCK / 64][16];
  int i = blockIdx.x * RADIX_BLOCK + threadIdx.x;
  int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  bool valid = i < n;
  uint64_t key = valid ? keys[i] : 0;
  int digit = valid ? (int)((key >> shift) & 15) : 16;
  unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int rank_in_wave = 0;
  for (int v = 0; v < 16; ++v) {
    unsigned long long m = __ballot(digit == v);
    if (digit == v) rank_in_wave = __popcll(m & lt);
    if (lane == 0) wave_cnt[wave][v] = __popcll(m);
  }
  __syncthreads();
  if (valid) {
    int before = 0;
    for (int w = 0; w < wave; ++w) before += wave_cnt[w][digit];
    int dst = offs[digit * nblk + blockIdx.x] + before + rank_in_wave;
    keys_out[dst] = key;
    vals_out[dst] = vals[i];
  }
}

// Stable sort of (key, val) by the low nbits of key (ties keep input order).
int sort_pairs_u64(uint64_t* keys, int* vals, int n, int nbits, DevArena& scratch,
                   hipStream_t s) {
  if (n <= 1) return 0;
  int nblk = ceil_div(n, RADIX_BLOCK);
  uint64_t* k2;
  int *v2, *hist, *offs;
  ARENA_ALLOC(scratch, k2, n);
  ARENA_ALLOC(scratch, v2, n);
  ARENA_ALLOC(scratch, hist, 16 * nblk);
  ARENA_ALLOC(scratch, offs, 16 * nblk);
  int passes = (nbits + 3) / 4;
  uint64_t *ka = keys, *kb = k2;
  int *va = vals, *vb = v2;
  for (int ps = 0; ps < passes; ++ps) {
    int shift = 4 * ps;
    hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(RADIX_BLOCK), 0, s, ka, n, shift, hist,
                       nblk);
    BEM_LAUNCH_CHECK();
    int r = exclusive_scan(hist, offs, 16 * nblk, nullptr, scratch, s);
    if (r) return r;
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(RADIX_BLOCK), 0, s, ka, va, n, shift,
                       offs, nblk, kb, vb);
    BEM_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys) {
    BEM_HIP_TRY(hipMemcpyAsync(keys, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
    BEM_HIP_TRY(hipMemcpyAsync(vals, va, sizeof(int) * n, hipMemcpyDeviceToDevice, s));
  }
  return 0;
}

// ---------------------------------------------------------------------------
// tree
// ---------------------------------------------------------------------------
__global__ void k_gather_geo(const double* __restrict__ g, const int* __restrict__ perm,
                             int64_t n, double* __restrict__ gs) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int src = perm[i];
  for (int c = 0; c < GEO_COUNT; ++c) gs[c * n + i] = g[c * n + src];
}

__global__ void k_keys_orig(const uint64_t* __restrict__ ks, const int* __restrict__ perm,
                            int64_t n, uint64_t* __restrict__ ko) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) ko[perm[i]] = ks[i];
}

__global__ void k_box_flags(const uint64_t* __restrict__ ks, int n, int shift,
                            int* __restrict__ flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flags[i] = (i == 0 || (ks[i] >> shift) != (ks[i - 1] >> shift)) ? 1 : 0;
}

__global__ void k_box_fill(const uint64_t* __restrict__ ks, int n, int shift,
                           const int* __restrict__ flags, const int* __restrict__ idx,
                           uint64_t* __restrict__ bkeys, int* __restrict__ bstart,
                           int* __restrict__ elem_box, int nbox) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int b = idx[i] + flags[i] - 1;
  if (elem_box) elem_box[i] = b;
  if (flags[i]) {
    bkeys[b] = ks[i] >> shift;
    bstart[b] = i;
  }
  if (i == 0) bstart[nbox] = n;
}

__global__ void k_max_run(const int* __restrict__ bstart, int nbox, int* __restrict__ out) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbox) return;
  atomicMax(out, bstart[b + 1] - bstart[b]);
}

__global__ void k_parent(const int* __restrict__ bstart, int nbox,
                         const int* __restrict__ elem_box_parent, int* __restrict__ parent) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbox) return;
  parent[b] = elem_box_parent[bstart[b]];
}

__device__ __forceinline__ int find_key(const uint64_t* __restrict__ keys, int n, uint64_t key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (keys[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < n && keys[lo] == key) ? lo : -1;
}

__device__ __forceinline__ uint64_t key_of(int x, int y, int z) {
  return (spread3((uint64_t)x) << 2) | (spread3((uint64_t)y) << 1) | spread3((uint64_t)z);
}

// U lists: the non-empty leaves adjacent to (or equal to) each leaf, ascending.
__global__ void k_ulist(const uint64_t* __restrict__ lkeys, int nleaf, int L,
                        const int* __restrict__ ptr, int* __restrict__ cnt_or_idx, int fill) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  uint64_t key = lkeys[b];
  int x = compact3(key >> 2), y = compact3(key >> 1), z = compact3(key);
  int side = 1 << L;
  int found[27];
  int nf = 0;
  for (int dx = -1; dx <= 1; ++dx)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dz = -1; dz <= 1; ++dz) {
        int cx = x + dx, cy = y + dy, cz = z + dz;
        if (cx < 0 || cy < 0 || cz < 0 || cx >= side || cy >= side || cz >= side) continue;
        int f = find_key(lkeys, nleaf, key_of(cx, cy, cz));
        if (f >= 0) found[nf++] = f;
      }
  if (!fill) {
    cnt_or_idx[b] = nf;
    return;
  }
  // insertion sort (ascending leaf index)
  for (int i = 1; i < nf; ++i) {
    int v = found[i], j = i - 1;
    while (j >= 0 && found[j] > v) {
      found[j + 1] = found[j];
      --j;
    }
    found[j + 1] = v;
  }
  int o = ptr[b];
  for (int i = 0; i < nf; ++i) cnt_or_idx[o + i] = found[i];
}

// V lists at level l: children of the parent's colleagues that are not
// colleagues themselves.  Pass 0 counts; pass 1 writes (dst, src, offset
// code) with code = (dx+3)*49 + (dy+3)*7 + (dz+3), d = target - source in box
// units.
__global__ void k_vlist(const uint64_t* __restrict__ bkeys, int nbox,
                        const uint64_t* __restrict__ pkeys, int npbox, int l,
                        const int* __restrict__ ptr, int* __restrict__ cnt, int* __restrict__ dst,
                        int* __restrict__ src, int* __restrict__ code, int fill) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbox) return;
  uint64_t key = bkeys[b];
  int x = compact3(key >> 2), y = compact3(key >> 1), z = compact3(key);
  int px = x >> 1, py = y >> 1, pz = z >> 1;
  int pside = 1 << (l - 1);
  int nf = 0;
  int o = fill ? ptr[b] : 0;
  for (int dx = -1; dx <= 1; ++dx)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dz = -1; dz <= 1; ++dz) {
        int qx = px + dx, qy = py + dy, qz = pz + dz;
        if (qx < 0 || qy < 0 || qz < 0 || qx >= pside || qy >= pside || qz >= pside) continue;
        uint64_t pk = key_of(qx, qy, qz);
        if (find_key(pkeys, npbox, pk) < 0) continue;
        for (int ch = 0; ch < 8; ++ch) {
          int cx = 2 * qx + ((ch >> 2) & 1), cy = 2 * qy + ((ch >> 1) & 1), cz = 2 * qz + (ch & 1);
          int ddx = x - cx, ddy = y - cy, ddz = z - cz;
          int m = max(abs(ddx), max(abs(ddy), abs(ddz)));
          if (m <= 1) continue;
          int f = find_key(bkeys, nbox, (pk << 3) | (uint64_t)ch);
          if (f < 0) continue;
          if (fill) {
            dst[o + nf] = b;
            src[o + nf] = f;
            code[o + nf] = (ddx + 3) * 49 + (ddy + 3) * 7 + (ddz + 3);
          }
          ++nf;
        }
      }
  if (!fill) cnt[b] = nf;
}

__global__ void k_elem_leaf(const int* __restrict__ bstart, int nleaf, int* __restrict__ el) {
  int b = blockIdx.x;
  for (int i = bstart[b] + threadIdx.x; i < bstart[b + 1]; i += blockDim.x) el[i] = b;
}

__global__ void k_u_pairs(const int* __restrict__ u_ptr, const int* __restrict__ u_idx,
                          const int* __restrict__ bstart, int nleaf,
                          unsigned long long* __restrict__ out) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  long long s = 0;
  for (int t = u_ptr[b]; t < u_ptr[b + 1]; ++t) {
    int c = u_idx[t];
    s += (long long)(bstart[c + 1] - bstart[c]);
  }
  atomicAdd(out, (unsigned long long)(s * (bstart[b + 1] - bstart[b])));
}

static int box_level(Problem& P, int l, DevArena& scratch, hipStream_t s, int* elem_box,
                     int* nbox_out) {
  int n = (int)P.n;
  int shift = 3 * (NBITS - l);
  int *flags, *idx;
  ARENA_ALLOC(scratch, flags, n);
  ARENA_ALLOC(scratch, idx, n);
  int nb = ceil_div(n, 256);
  hipLaunchKernelGGL(k_box_flags, dim3(nb), dim3(256), 0, s, P.keys_sorted, n, shift, flags);
  BEM_LAUNCH_CHECK();
  int nbox = 0;
  int r = exclusive_scan(flags, idx, n, &nbox, scratch, s);
  if (r) return r;
  uint64_t* bkeys;
  int* bstart;
  ARENA_ALLOC(P.arena, bkeys, nbox);
  ARENA_ALLOC(P.arena, bstart, nbox + 1);
  hipLaunchKernelGGL(k_box_fill, dim3(nb), dim3(256), 0, s, P.keys_sorted, n, shift, flags, idx,
                     bkeys, bstart, elem_box, nbox);
  BEM_LAUNCH_CHECK();
  P.box_keys[l] = bkeys;
  P.box_start[l] = bstart;
  P.nbox[l] = nbox;
  *nbox_out = nbox;
  return 0;
}

static int max_occupancy(Problem& P, int l, DevArena& scratch, hipStream_t s, int* out) {
  int* dmax;
  ARENA_ALLOC(scratch, dmax, 1);
  BEM_HIP_TRY(hipMemsetAsync(dmax, 0, sizeof(int), s));
  int n = (int)P.n, shift = 3 * (NBITS - l);
  int *flags, *idx, *bstart;
  ARENA_ALLOC(scratch, flags, n);
  ARENA_ALLOC(scratch, idx, n);
  int nb = ceil_div(n, 256);
  hipLaunchKernelGGL(k_box_flags, dim3(nb), dim3(256), 0, s, P.keys_sorted, n, shift, flags);
  BEM_LAUNCH_CHECK();
  int nbox = 0;
  int r = exclusive_scan(flags, idx, n, &nbox, scratch, s);
  if (r) return r;
  uint64_t* bkeys;
  ARENA_ALLOC(scratch, bkeys, nbox);
  ARENA_ALLOC(scratch, bstart, nbox + 1);
  hipLaunchKernelGGL(k_box_fill, dim3(nb), dim3(256), 0, s, P.keys_sorted, n, shift, flags, idx,
                     bkeys, bstart, (int*)nullptr, nbox);
  BEM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_max_run, dim3(ceil_div(nbox, 256)), dim3(256), 0, s, bstart, nbox, dmax);
  BEM_LAUNCH_CHECK();
  BEM_HIP_TRY(hipMemcpyAsync(out, dmax, sizeof(int), hipMemcpyDeviceToHost, s));
  BEM_HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

int build_geometry_and_tree(Problem& P, const double* vert, int64_t n_vert, const int32_t* tri,
                            hipStream_t s) {
  const int64_t n = P.n;
  DevArena scratch;
  struct Guard {
    DevArena& a;
    ~Guard() { a.release(); }
  } guard{scratch};
  double* dV;
  int* dT;
  ARENA_ALLOC(scratch, dV, 3 * n_vert);
  ARENA_ALLOC(scratch, dT, 3 * n);
  BEM_HIP_TRY(hipMemcpyAsync(dV, vert, sizeof(double) * 3 * n_vert, hipMemcpyHostToDevice, s));
  BEM_HIP_TRY(hipMemcpyAsync(dT, tri, sizeof(int) * 3 * n, hipMemcpyHostToDevice, s));
  double* g_orig;
  int* bad;
  ARENA_ALLOC(scratch, g_orig, GEO_COUNT * n);
  ARENA_ALLOC(scratch, bad, 1);
  BEM_HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int), s));
  int nb = ceil_div(n, 256);
  hipLaunchKernelGGL(k_geometry, dim3(nb), dim3(256), 0, s, dV, dT, n, n_vert, g_orig, bad);
  BEM_LAUNCH_CHECK();
  int hbad = 0;
  BEM_HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  BEM_HIP_TRY(hipStreamSynchronize(s));
  if (hbad) {
    set_error(std::string("invalid mesh:") + ((hbad & 1) ? " vertex index out of range" : "") +
              ((hbad & 2) ? " non-finite coordinates" : "") +
              ((hbad & 4) ? " zero-area triangle" : ""));
    return -1;
  }
  // bounding cube and keys
  double *bb, *prm;
  ARENA_ALLOC(scratch, bb, 8);
  ARENA_ALLOC(scratch, prm, 8);
  hipLaunchKernelGGL(k_bbox, dim3(1), dim3(256), 0, s, g_orig, n, bb);
  BEM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_morton_params, dim3(1), dim3(1), 0, s, bb, prm);
  BEM_LAUNCH_CHECK();
  double hb[8], hp[8];
  BEM_HIP_TRY(hipMemcpyAsync(hb, bb, sizeof(double) * 8, hipMemcpyDeviceToHost, s));
  BEM_HIP_TRY(hipMemcpyAsync(hp, prm, sizeof(double) * 8, hipMemcpyDeviceToHost, s));
  BEM_HIP_TRY(hipStreamSynchronize(s));
  for (int d = 0; d < 3; ++d) P.lo[d] = hp[d];
  P.scale = hp[3];
  P.R0 = hp[4];
  P.ell_max = hb[6];
  if (!(P.R0 > 0.0)) {
    set_error("degenerate mesh: all collocation points coincide");
    return -1;
  }
  ARENA_ALLOC(P.arena, P.keys_sorted, n);
  ARENA_ALLOC(P.arena, P.keys_orig, n);
  ARENA_ALLOC(P.arena, P.perm, n);
  hipLaunchKernelGGL(k_morton_keys, dim3(nb), dim3(256), 0, s, g_orig, n, prm, P.keys_sorted,
                     P.perm);
  BEM_LAUNCH_CHECK();
  int r = sort_pairs_u64(P.keys_sorted, P.perm, (int)n, 3 * NBITS, scratch, s);
  if (r) return r;
  hipLaunchKernelGGL(k_keys_orig, dim3(nb), dim3(256), 0, s, P.keys_sorted, P.perm, n,
                     P.keys_orig);
  BEM_LAUNCH_CHECK();
  ARENA_ALLOC(P.arena, P.geo, GEO_COUNT * n);
  hipLaunchKernelGGL(k_gather_geo, dim3(nb), dim3(256), 0, s, g_orig, P.perm, n, P.geo);
  BEM_LAUNCH_CHECK();

  // leaf level: smallest L >= 2 with max occupancy <= cap, but leaves must
  // stay wider than the near-pair radius eta * max edge so that every near
  // pair lies in adjacent leaves.
  for (int l = 0; l <= MAX_LEVEL; ++l) P.h[l] = 2.0 * P.R0 / (double)(1 << l);
  int L_near = 2;
  for (int l = 2; l <= MAX_LEVEL; ++l)
    if (P.h[l] > P.eta * P.ell_max) L_near = l;
  int L = 0;
  if (P.leaf_level_req > 0) {
    L = std::min(std::max(P.leaf_level_req, 2), MAX_LEVEL);
  } else {
    L = MAX_LEVEL;
    for (int l = 2; l <= MAX_LEVEL; ++l) {
      int occ = 0;
      r = max_occupancy(P, l, scratch, s, &occ);
      if (r) return r;
      if (occ <= P.leaf_cap) {
        L = l;
        break;
      }
    }
  }
  if (L > L_near) L = L_near;
  P.L = L;
  r = max_occupancy(P, L, scratch, s, &P.max_leaf);
  if (r) return r;
  P.direct = !(P.h[L] > P.eta * P.ell_max);

  // boxes of every level 0..L and parents
  std::vector<int*> elem_box(L + 1, nullptr);
  for (int l = 0; l <= L; ++l) {
    ARENA_ALLOC(scratch, elem_box[l], n);
    int nbx = 0;
    r = box_level(P, l, scratch, s, elem_box[l], &nbx);
    if (r) return r;
    if (l > 0) {
      ARENA_ALLOC(P.arena, P.box_parent[l], nbx);
      hipLaunchKernelGGL(k_parent, dim3(ceil_div(nbx, 256)), dim3(256), 0, s, P.box_start[l], nbx,
                         elem_box[l - 1], P.box_parent[l]);
      BEM_LAUNCH_CHECK();
    }
  }
  const int nleaf = P.nbox[L];
  ARENA_ALLOC(P.arena, P.elem_leaf, n);
  hipLaunchKernelGGL(k_elem_leaf, dim3(nleaf), dim3(64), 0, s, P.box_start[L], nleaf, P.elem_leaf);
  BEM_LAUNCH_CHECK();
  // U lists
  int* ucnt;
  ARENA_ALLOC(scratch, ucnt, nleaf);
  ARENA_ALLOC(P.arena, P.u_ptr, nleaf + 1);
  hipLaunchKernelGGL(k_ulist, dim3(ceil_div(nleaf, 128)), dim3(128), 0, s, P.box_keys[L], nleaf, L,
                     (const int*)nullptr, ucnt, 0);
  BEM_LAUNCH_CHECK();
  int nu = 0;
  r = exclusive_scan(ucnt, P.u_ptr, nleaf, &nu, scratch, s);
  if (r) return r;
  BEM_HIP_TRY(hipMemcpyAsync(P.u_ptr + nleaf, &nu, sizeof(int), hipMemcpyHostToDevice, s));
  ARENA_ALLOC(P.arena, P.u_idx, nu);
  hipLaunchKernelGGL(k_ulist, dim3(ceil_div(nleaf, 128)), dim3(128), 0, s, P.box_keys[L], nleaf, L,
                     P.u_ptr, P.u_idx, 1);
  BEM_LAUNCH_CHECK();
  P.n_u = nu;
  unsigned long long* dpairs;
  ARENA_ALLOC(scratch, dpairs, 1);
  BEM_HIP_TRY(hipMemsetAsync(dpairs, 0, sizeof(unsigned long long), s));
  hipLaunchKernelGGL(k_u_pairs, dim3(ceil_div(nleaf, 128)), dim3(128), 0, s, P.u_ptr, P.u_idx,
                     P.box_start[L], nleaf, dpairs);
  BEM_LAUNCH_CHECK();
  unsigned long long hpairs = 0;
  BEM_HIP_TRY(hipMemcpyAsync(&hpairs, dpairs, sizeof(hpairs), hipMemcpyDeviceToHost, s));
  BEM_HIP_TRY(hipStreamSynchronize(s));
  P.n_p2p_pairs = (int64_t)hpairs;
  return 0;
}

// V-list pairs of level l, sorted by (offset code, dst, src); returns device
// arrays allocated in P.arena.
int build_vlist(Problem& P, int l, int** dst, int** src, int** code, int* npairs,
                DevArena& scratch, hipStream_t s) {
  int nbox = P.nbox[l], npbox = P.nbox[l - 1];
  int *cnt, *ptr;
  ARENA_ALLOC(scratch, cnt, nbox);
  ARENA_ALLOC(scratch, ptr, nbox);
  hipLaunchKernelGGL(k_vlist, dim3(ceil_div(nbox, 128)), dim3(128), 0, s, P.box_keys[l], nbox,
                     P.box_keys[l - 1], npbox, l, (const int*)nullptr, cnt, (int*)nullptr,
                     (int*)nullptr, (int*)nullptr, 0);
  BEM_LAUNCH_CHECK();
  int np = 0;
  int r = exclusive_scan(cnt, ptr, nbox, &np, scratch, s);
  if (r) return r;
  int *d0, *s0, *c0;
  ARENA_ALLOC(scratch, d0, np);
  ARENA_ALLOC(scratch, s0, np);
  ARENA_ALLOC(scratch, c0, np);
  hipLaunchKernelGGL(k_vlist, dim3(ceil_div(nbox, 128)), dim3(128), 0, s, P.box_keys[l], nbox,
                     P.box_keys[l - 1], npbox, l, ptr, cnt, d0, s0, c0, 1);
  BEM_LAUNCH_CHECK();
  *npairs = np;
  *dst = d0;
  *src = s0;
  *code = c0;
  return 0;
}

}  // namespace bemfmm
