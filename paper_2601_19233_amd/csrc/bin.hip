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

// One thread per record: write one key/value pair per overlapped tile.  The
// key is (global tile << depth_bits) | (depth key - depth_base): the order of
// (tile, depth) with the depth range of the frame in as few bits as it needs.
__global__ void emit_keys_kernel(const ViewParams *__restrict__ views, int V, int per_view,
                                 int64_t n_records, const uint32_t *__restrict__ depth,
                                 const uint2 *__restrict__ rects,
                                 const uint64_t *__restrict__ offs,
                                 const FrameInfo *__restrict__ fi,
                                 uint64_t *__restrict__ keys_out,
                                 uint32_t *__restrict__ vals_out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_records) return;
  const uint64_t o0 = offs[r], o1 = offs[r + 1];
  const uint64_t cap = fi->n_dup;          // pairs beyond the key capacity are dropped
  if (o0 == o1 || o0 >= cap) return;
  const uint32_t depth_base = fi->depth_base;
  const int depth_bits = fi->depth_bits;
  const int v = (int)(r / per_view);
  const ViewParams &vp = views[v];
  const uint2 rc = rects[r];
  const int tx0 = rc.x & 0xFFFF, ty0 = rc.x >> 16, tx1 = rc.y & 0xFFFF, ty1 = rc.y >> 16;
  const uint64_t d = depth[r] - depth_base;
  uint64_t o = o0;
  for (int ty = ty0; ty < ty1; ++ty) {
    const uint64_t row = (uint64_t)vp.tile_base + (uint64_t)ty * vp.ntx;
    for (int tx = tx0; tx < tx1 && o < cap; ++tx) {
      keys_out[o] = ((row + tx) << depth_bits) | d;
      vals_out[o] = (uint32_t)r;
      ++o;
    }
  }
}

// Load-balanced emission: each block owns kEmitSpan consecutive output
// positions and writes them with consecutive lanes on consecutive addresses.
// The records covering the block's range are found by binary search in the
// scanned offsets and staged in LDS; every lane then finds its position's
// record by binary search in LDS and derives the tile from the position's
// rank inside the record's tile rectangle (row-major, as the scan counted).
constexpr int kEmitThreads = 256;
constexpr int kEmitPer = 8;
constexpr int kEmitSpan = kEmitThreads * kEmitPer;
constexpr int kEmitRecCap = 1024;

// last r in [lo, hi] with offs[r] <= d (offs is non-decreasing)
__device__ __forceinline__ int64_t last_record_at(const uint64_t *__restrict__ offs, int64_t lo,
                                                  int64_t hi, uint64_t d) {
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= d) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ uint64_t tile_key(const ViewParams *__restrict__ views, int v, uint2 rc,
                                             uint64_t j, uint32_t dep, int bits) {
  const uint32_t tx0 = rc.x & 0xFFFF, ty0 = rc.x >> 16, tx1 = rc.y & 0xFFFF;
  const uint32_t w = tx1 - tx0;
  const uint32_t jj = (uint32_t)j;
  const uint32_t ty = ty0 + jj / w, tx = tx0 + jj % w;
  const uint64_t tile = (uint64_t)views[v].tile_base + (uint64_t)ty * views[v].ntx + tx;
  return (tile << bits) | dep;
}

__global__ __launch_bounds__(kEmitThreads) void emit_balanced_kernel(
    const ViewParams *__restrict__ views, int per_view, int64_t n_records,
    const uint32_t *__restrict__ depth, const uint2 *__restrict__ rects,
    const uint64_t *__restrict__ offs, const FrameInfo *__restrict__ fi,
    uint64_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out) {
  __shared__ uint64_t s_off[kEmitRecCap];
  __shared__ uint2 s_rect[kEmitRecCap];
  __shared__ uint32_t s_dep[kEmitRecCap];
  __shared__ int32_t s_view[kEmitRecCap];
  __shared__ int64_t s_lo, s_hi;
  const uint64_t n = fi->n_dup;
  const uint64_t d0 = (uint64_t)blockIdx.x * kEmitSpan;
  if (d0 >= n) return;
  const uint64_t d1 = min(d0 + (uint64_t)kEmitSpan, n);
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_lo = last_record_at(offs, 0, n_records, d0);
    s_hi = last_record_at(offs, s_lo, n_records, d1 - 1);
  }
  __syncthreads();
  const int64_t rlo = s_lo, rhi = s_hi;
  const int64_t nr = rhi - rlo + 1;
  const uint32_t base = fi->depth_base;
  const int bits = fi->depth_bits;
  if (nr <= kEmitRecCap) {
    for (int64_t i = tid; i < nr; i += kEmitThreads) {
      const int64_t r = rlo + i;
      s_off[i] = offs[r];
      s_rect[i] = rects[r];
      s_dep[i] = depth[r] - base;
      s_view[i] = (int32_t)(r / per_view);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kEmitPer; ++k) {
      const uint64_t d = d0 + (uint64_t)k * kEmitThreads + tid;
      if (d >= d1) break;
      int lo = 0, hi = (int)nr - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= d) lo = mid; else hi = mid - 1;
      }
      keys_out[d] = tile_key(views, s_view[lo], s_rect[lo], d - s_off[lo], s_dep[lo], bits);
      vals_out[d] = (uint32_t)(rlo + lo);
    }
  } else {
    // many empty records inside the range: search the offsets in memory
    for (int k = 0; k < kEmitPer; ++k) {
      const uint64_t d = d0 + (uint64_t)k * kEmitThreads + tid;
      if (d >= d1) break;
      const int64_t r = last_record_at(offs, rlo, rhi, d);
      keys_out[d] = tile_key(views, (int)(r / per_view), rects[r], d - offs[r], depth[r] - base, bits);
      vals_out[d] = (uint32_t)r;
    }
  }
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Turns the scanned total and the depth range into the frame's sizes.
__global__ void frame_info_kernel(const uint64_t *__restrict__ total,
                                  const uint32_t *__restrict__ minmax, uint64_t cap,
                                  int tile_bits, FrameInfo *__restrict__ fi) {
  const uint64_t raw = *total;
  fi->n_dup = (uint32_t)(raw < cap ? raw : cap);
  if (raw > cap) fi->overflow = 1u;
  const uint32_t lo = minmax[0], hi = minmax[1];
  const bool any = lo <= hi;
  fi->depth_base = any ? lo : 0u;
  int db = 1;
  while (any && db < 32 && (uint64_t)(hi - lo) >= (1ull << db)) ++db;
  fi->depth_bits = db;
  fi->total_bits = db + tile_bits;
  fi->sorted_in = ((db + tile_bits + 7) / 8) & 1;
  fi->queue = 0u;
}

__global__ void tile_ranges_kernel(const uint64_t *__restrict__ k0, const uint64_t *__restrict__ k1,
                                   const FrameInfo *__restrict__ fi, uint2 *__restrict__ ranges) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t n = fi->n_dup;
  if (i >= n) return;
  const int shift = fi->depth_bits;
  const uint64_t *keys = fi->sorted_in ? k1 : k0;
  const uint32_t t = (uint32_t)(keys[i] >> shift);
  if (i == 0 || (uint32_t)(keys[i - 1] >> shift) != t) ranges[t].x = (uint32_t)i;
  if (i == n - 1 || (uint32_t)(keys[i + 1] >> shift) != t) ranges[t].y = (uint32_t)(i + 1);
}

// Sorted keys back in the exported (tile << 32 | depth key bits) form.
__global__ void expand_keys_kernel(const uint64_t *__restrict__ k0, const uint64_t *__restrict__ k1,
                                   const FrameInfo *__restrict__ fi, uint64_t *__restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= fi->n_dup) return;
  const int shift = fi->depth_bits;
  const uint32_t base = fi->depth_base;
  const uint64_t k = (fi->sorted_in ? k1 : k0)[i];
  const uint64_t mask = shift >= 64 ? ~0ull : ((1ull << shift) - 1ull);
  out[i] = ((k >> shift) << 32) | (uint64_t)((uint32_t)(k & mask) + base);
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
  hipLaunchKernelGGL(frame_info_kernel, dim3(1), dim3(1), 0, c->stream,
                     (const uint64_t *)c->counts.p + c->n_records, (const uint32_t *)c->minmax.p,
                     (uint64_t)c->key_cap, c->tile_bits, (FrameInfo *)c->finfo.p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || c->n_records == 0) return e;
  if (c->n_launch == 0) return hipSuccess;
  ScopedTimer t(c, K_EMIT);
  hipLaunchKernelGGL(emit_balanced_kernel, dim3(ceil_div(c->n_launch, kEmitSpan)),
                     dim3(kEmitThreads), 0, c->stream, c->cur_views,
                     c->N + c->T, c->n_records, (const uint32_t *)c->keys.p,
                     (const uint2 *)c->rects.p, (const uint64_t *)c->counts.p,
                     (const FrameInfo *)c->finfo.p, (uint64_t *)c->k0.p, (uint32_t *)c->v0.p);
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
  if (e != hipSuccess || c->n_launch == 0) return e;
  hipLaunchKernelGGL(tile_ranges_kernel, dim3(ceil_div(c->n_launch, 256)), dim3(256), 0, c->stream,
                     (const uint64_t *)c->k0.p, (const uint64_t *)c->k1.p,
                     (const FrameInfo *)c->finfo.p, (uint2 *)c->ranges.p);
  return hipGetLastError();
}

hipError_t launch_expand_keys(Ctx *c, uint64_t *dst) {
  if (c->n_launch == 0) return hipSuccess;
  hipLaunchKernelGGL(expand_keys_kernel, dim3(ceil_div(c->n_launch, 256)), dim3(256), 0, c->stream,
                     (const uint64_t *)c->k0.p, (const uint64_t *)c->k1.p,
                     (const FrameInfo *)c->finfo.p, dst);
  return hipGetLastError();
}

}  // namespace umgs
