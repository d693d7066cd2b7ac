// Bin stage: exclusive scan of per-primitive tile counts, emission of one
// (global tile << 32 | depth bits, record id) pair per overlapped tile, and
// per-tile [start, end) ranges of the sorted pairs.
#include "internal.h"

namespace umgs {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// Block-wide exclusive scan of one value per thread; returns the block total.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T x, T &total) {
  __shared__ T wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T incl = wave_incl_scan(x);
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kScanThreads / 64; ++k) {
    if (k < w) base += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();
  total = tot;
  return base + incl - x;
}

template <typename T>
__global__ void scan_reduce_kernel(const T *__restrict__ in, int64_t n, T *__restrict__ partial) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + (int64_t)k * kScanThreads + threadIdx.x;
    if (idx < n) s += in[idx];
  }
  T total;
  block_excl_scan(s, total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Exclusive scan of a tile, each thread owning kScanItems consecutive items.
template <typename T>
__global__ void scan_apply_kernel(T *__restrict__ data, int64_t n, const T *__restrict__ offs) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    v[k] = idx < n ? data[idx] : T(0);
    s += v[k];
  }
  T total;
  T run = block_excl_scan(s, total) + (offs ? offs[blockIdx.x] : T(0));
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    if (idx < n) data[idx] = run;
    run += v[k];
  }
}

template <typename T>
hipError_t excl_scan(hipStream_t s, T *data, int64_t n, T *tmp) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    hipLaunchKernelGGL(scan_apply_kernel<T>, dim3(1), dim3(kScanThreads), 0, s, data, n,
                       (const T *)nullptr);
    return hipGetLastError();
  }
  T *partial = tmp;
  hipLaunchKernelGGL(scan_reduce_kernel<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s,
                     (const T *)data, n, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = excl_scan<T>(s, partial, nb, tmp + nb);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_apply_kernel<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data,
                     n, (const T *)partial);
  return hipGetLastError();
}

// One thread per record: write one key/value pair per overlapped tile.
__global__ void emit_keys_kernel(const ViewParams *__restrict__ views, int V, int per_view,
                                 int64_t n_records, const uint32_t *__restrict__ depth,
                                 const uint2 *__restrict__ rects,
                                 const uint64_t *__restrict__ offs,
                                 uint64_t *__restrict__ keys_out,
                                 uint32_t *__restrict__ vals_out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_records) return;
  const uint64_t o0 = offs[r], o1 = offs[r + 1];
  if (o0 == o1) return;
  const int v = (int)(r / per_view);
  const ViewParams &vp = views[v];
  const uint2 rc = rects[r];
  const int tx0 = rc.x & 0xFFFF, ty0 = rc.x >> 16, tx1 = rc.y & 0xFFFF, ty1 = rc.y >> 16;
  const uint64_t d = depth[r];
  uint64_t o = o0;
  for (int ty = ty0; ty < ty1; ++ty) {
    const uint64_t row = (uint64_t)vp.tile_base + (uint64_t)ty * vp.ntx;
    for (int tx = tx0; tx < tx1; ++tx) {
      keys_out[o] = ((row + tx) << 32) | d;
      vals_out[o] = (uint32_t)r;
      ++o;
    }
  }
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void tile_ranges_kernel(const uint64_t *__restrict__ keys, uint64_t n,
                                   uint2 *__restrict__ ranges) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t t = (uint32_t)(keys[i] >> 32);
  if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != t) ranges[t].x = (uint32_t)i;
  if (i == n - 1 || (uint32_t)(keys[i + 1] >> 32) != t) ranges[t].y = (uint32_t)(i + 1);
}

}  // namespace

size_t scan_tmp_bytes(int64_t n) {
  size_t total = 0;
  int64_t m = n;
  while (m > kScanTile) {
    m = (m + kScanTile - 1) / kScanTile;
    total += (size_t)m;
  }
  return (total + 16) * sizeof(uint64_t);
}

hipError_t launch_exclusive_scan_u64(Ctx *c, uint64_t *data, int64_t n, uint64_t *tmp) {
  ScopedTimer t(c, K_SCAN);
  return excl_scan<uint64_t>(c->stream, data, n, tmp);
}

hipError_t launch_exclusive_scan_u32(Ctx *c, uint32_t *data, int64_t n, uint32_t *tmp) {
  ScopedTimer t(c, K_SORT_SCAN);
  return excl_scan<uint32_t>(c->stream, data, n, tmp);
}

hipError_t launch_emit_keys(Ctx *c) {
  if (c->n_dup == 0) return hipSuccess;
  ScopedTimer t(c, K_EMIT);
  hipLaunchKernelGGL(emit_keys_kernel, dim3(ceil_div(c->n_records, 256)), dim3(256), 0,
                     c->stream, (const ViewParams *)c->d_views.p, c->V, c->N + c->T,
                     c->n_records, (const uint32_t *)c->keys.p, (const uint2 *)c->rects.p,
                     (const uint64_t *)c->counts.p, (uint64_t *)c->k0.p, (uint32_t *)c->v0.p);
  return hipGetLastError();
}

hipError_t launch_fill_u32(Ctx *c, uint32_t *p, int64_t n, uint32_t v) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, c->stream, p, n, v);
  return hipGetLastError();
}

hipError_t launch_tile_ranges(Ctx *c) {
  ScopedTimer t(c, K_RANGES);
  hipError_t e = launch_fill_u32(c, (uint32_t *)c->ranges.p, 2 * c->n_tiles, 0u);
  if (e != hipSuccess || c->n_dup == 0) return e;
  const uint64_t *k = (const uint64_t *)(c->sorted_in ? c->k1.p : c->k0.p);
  hipLaunchKernelGGL(tile_ranges_kernel, dim3(ceil_div(c->n_dup, 256)), dim3(256), 0, c->stream,
                     k, c->n_dup, (uint2 *)c->ranges.p);
  return hipGetLastError();
}

}  // namespace umgs
