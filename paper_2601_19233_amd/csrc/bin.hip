// Bin stage.  The records are put in depth order first (a radix sort of
// 1 key per record), their tile counts scanned in that order, and one
// (global tile id, record id) pair emitted per overlapped tile at the
// record's scanned offset.  Duplicates thus leave the bin stage in depth
// order, and a stable sort by tile id alone (sort.hip) yields every tile's
// front-to-back list; per-tile [start, end) ranges are then read off the
// sorted tile ids.
#include "support.h"

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

// Per-view duplicate totals (records are view-major): one partial sum per
// block, one atomic per block.
__global__ void view_sum_kernel(const uint64_t *__restrict__ counts, int64_t per_view,
                                unsigned long long *__restrict__ sums) {
  const int v = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kScanTile;
  uint64_t s = 0;
  for (int k = threadIdx.x; k < kScanTile; k += kScanThreads)
    if (i + k < per_view) s += counts[(int64_t)v * per_view + i + k];
  uint64_t total;
  block_excl_scan(s, total);
  if (threadIdx.x == 0 && total) atomicAdd(sums + v, (unsigned long long)total);
}

// Depth range of the frame: sort keys hold (depth key - base) in depth_bits.
// One wave folds the slot pairs the projection kernels filled.
__global__ void depth_range_kernel(const uint32_t *__restrict__ minmax, FrameInfo *__restrict__ fi) {
  const uint32_t lo = wave_min_u32(minmax[threadIdx.x]);
  const uint32_t hi = wave_max_u32(minmax[kMinMaxSlots + threadIdx.x]);
  if (threadIdx.x != 0) return;
  const bool any = lo <= hi;
  fi->depth_base = any ? lo : 0u;
  int db = 1;
  while (any && db < 32 && (uint64_t)(hi - lo) >= (1ull << db)) ++db;
  fi->depth_bits = db;
}

// Depth-sort input: relative depth keys (culled records get all ones, after
// every visible one) and record ids in id order.
__global__ void depth_prep_kernel(const uint32_t *__restrict__ depth, int64_t n,
                                  const FrameInfo *__restrict__ fi, uint32_t *__restrict__ dk,
                                  uint32_t *__restrict__ dv) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const uint32_t k = depth[r];
  dk[r] = k == kCulled ? 0xFFFFFFFFu : k - fi->depth_base;
  dv[r] = (uint32_t)r;
}

// Tile counts in depth order (the count scan then gives each record's first
// output position); the entry past the end receives the total.
__global__ void gather_counts_kernel(const uint32_t *__restrict__ order, int64_t n,
                                     const uint64_t *__restrict__ counts,
                                     uint64_t *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = counts[order[i]];
  else if (i == n) out[n] = 0;
}

// Load-balanced emission: each block owns kEmitSpan consecutive output
// positions and writes them with consecutive lanes on consecutive addresses.
// Positions follow the depth order of the records; inside a record, its
// tiles in row-major order, each row cut to the record's support
// (support.h) exactly as the projection counted them.
//
// The block finds the records covering its range by binary search in the
// scanned offsets and stages them in LDS; one thread per record then lays
// out the record's tile rows in LDS (first column, first output position),
// so every lane finds its position's row, hence record and column, by one
// binary search in LDS.  Output: global tile id (the tile sort's key) and
// record id.
constexpr int kEmitThreads = 256;
constexpr int kEmitPer = 8;
constexpr int kEmitSpan = kEmitThreads * kEmitPer;
constexpr int kEmitRecCap = 256;
constexpr int kEmitRowCap = 1024;
constexpr int kEmitRowPer = kEmitRowCap / kEmitThreads;

// last r in [lo, hi] with offs[r] <= d (offs is non-decreasing)
__device__ __forceinline__ int64_t last_record_at(const uint64_t *__restrict__ offs, int64_t lo,
                                                  int64_t hi, uint64_t d) {
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= d) lo = mid; else hi = mid - 1;
  }
  return lo;
}

struct EmitArgs {
  const ViewParams *views;
  int per_view, N, tile_w, tile_h;
  int64_t n_records;
  const uint32_t *order;
  const uint2 *rects;
  const uint64_t *offs;
  const GaussRec *grec;
  const FrameInfo *fi;
  const uint32_t *blk_first;   // per block: the (depth-order) record holding its first position,
                               // then one entry: the record holding the last position
  void *keys_out;              // K (uint16_t or uint32_t) global tile ids
  uint32_t *vals_out;
};

// For every emit block, the record (in depth order) that holds the block's
// first output position, found by the records themselves: record i covers
// the positions [offs[i], offs[i+1]) and writes its index for each block
// starting inside that range, so no block searches the offsets.  The
// record holding the frame's last position is stored after the blocks.
__global__ void emit_blocks_kernel(const uint64_t *__restrict__ offs, int64_t n_records,
                                   const FrameInfo *__restrict__ fi, uint32_t nblocks,
                                   uint32_t *__restrict__ blk_first) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_records) return;
  const uint64_t n = fi->n_dup;
  const uint64_t o0 = offs[i], o1 = min(offs[i + 1], n);
  if (o0 >= o1) return;
  const uint64_t b0 = (o0 + kEmitSpan - 1) / kEmitSpan, b1 = (o1 + kEmitSpan - 1) / kEmitSpan;
  for (uint64_t b = b0; b < b1 && b < nblocks; ++b) blk_first[b] = (uint32_t)i;
  if (o1 == n) blk_first[nblocks] = (uint32_t)i;
}

// (clamps keep a tile inside its record's rectangle, hence inside its view,
// whatever the counts say)
__device__ __forceinline__ int clampi(int x, int lo, int hi) { return max(lo, min(x, hi)); }

__device__ __forceinline__ uint32_t global_tile(const EmitArgs &e, uint32_t r, int ty, int tx) {
  const ViewParams &vp = e.views[r / (uint32_t)e.per_view];
  return vp.tile_base + (uint32_t)ty * (uint32_t)vp.ntx + (uint32_t)tx;
}

// Block-wide exclusive scan of LDS values [0, n) (n <= per * kEmitThreads,
// each thread a contiguous chunk of `per`); returns the total.
template <int PER>
__device__ __forceinline__ uint32_t block_scan_lds(uint32_t *vals, int n, uint32_t *wsum) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint32_t v[PER], sum = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int q = tid * PER + j;
    v[j] = q < n ? vals[q] : 0u;
    sum += v[j];
  }
  uint32_t incl = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  __syncthreads();                       // vals fully read, wsum free
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t base = 0, total = 0;
#pragma unroll
  for (int k = 0; k < kEmitThreads / 64; ++k) {
    if (k < w) base += wsum[k];
    total += wsum[k];
  }
  uint32_t run = base + incl - sum;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int q = tid * PER + j;
    if (q < n) vals[q] = run;
    run += v[j];
  }
  __syncthreads();
  return total;
}

template <typename K>
__global__ __launch_bounds__(kEmitThreads) void emit_balanced_kernel(EmitArgs e) {
  K *const keys_out = (K *)e.keys_out;
  // staged records
  __shared__ uint32_t s_rec[kEmitRecCap];        // record id
  __shared__ int32_t s_off[kEmitRecCap];         // first output position, relative to d0
  __shared__ uint2 s_rect[kEmitRecCap];          // tile rectangle
  __shared__ uint32_t s_tb[kEmitRecCap];         // global id of its view's tile (0, 0)
  __shared__ uint32_t s_ntx[kEmitRecCap];        // tiles per row of its view
  __shared__ int2 s_wh[kEmitRecCap];             // its view's width and height
  __shared__ Support s_sup[kEmitRecCap];         // support of a Gaussian (exact = false: triangle)
  __shared__ uint32_t s_row0[kEmitRecCap + 1];   // rows, scanned to the first row slot
  __shared__ uint32_t s_pbase[kEmitRecCap];      // scanned tile count at the first row slot
  // row slots: one per tile row of a staged record
  __shared__ int32_t q_start[kEmitRowCap];       // first output position (relative to d0)
  __shared__ uint32_t q_tile0[kEmitRowCap];      // global tile id of the row's first tile
  __shared__ uint16_t q_k[kEmitRowCap];          // staged record index
  __shared__ uint16_t q_cnt[kEmitRowCap];        // tiles in the row
  __shared__ uint32_t s_wsum[kEmitThreads / 64];
  const uint64_t n = e.fi->n_dup;
  const uint64_t d0 = (uint64_t)blockIdx.x * kEmitSpan;
  if (d0 >= n) return;
  const uint64_t d1 = min(d0 + (uint64_t)kEmitSpan, n);
  const int tid = threadIdx.x;
  // records [rlo, rhi] cover the block: rhi is the next block's first record
  // (possibly one record too many, which no position maps to) or, for the
  // frame's last block, the record holding the last position
  const int64_t rlo = e.blk_first[blockIdx.x];
  const int64_t rhi = d1 < n ? (int64_t)e.blk_first[blockIdx.x + 1] : (int64_t)e.blk_first[gridDim.x];
  const int nr = (int)min<int64_t>(rhi - rlo + 1, (int64_t)kEmitRecCap + 1);
  int R = kEmitRowCap + 1;
  if (nr <= kEmitRecCap) {
    // records (strided over the threads, so their loads overlap)
    for (int k = tid; k < nr; k += kEmitThreads) {
      const uint32_t r = e.order[rlo + k];
      const uint2 rc = e.rects[r];
      const uint32_t v = r / (uint32_t)e.per_view;
      const int i = (int)(r - v * (uint32_t)e.per_view);
      s_rec[k] = r;
      s_off[k] = (int32_t)((int64_t)e.offs[rlo + k] - (int64_t)d0);
      s_rect[k] = rc;
      s_tb[k] = e.views[v].tile_base;
      s_ntx[k] = (uint32_t)e.views[v].ntx;
      s_wh[k] = make_int2(e.views[v].W, e.views[v].H);
      Support sup;
      sup.exact = false;
      if (i < e.N) sup = make_support(e.grec[(int64_t)v * e.N + i]);
      s_sup[k] = sup;
      s_row0[k] = (rc.y >> 16) - (rc.x >> 16);
    }
    __syncthreads();
    R = (int)block_scan_lds<kEmitRecCap / kEmitThreads>(s_row0, nr, s_wsum);
    if (tid == 0) s_row0[nr] = (uint32_t)R;
    __syncthreads();
  }
  if (R <= kEmitRowCap) {
    // row slot -> staged record
    for (int k = tid; k < nr; k += kEmitThreads)
      for (uint32_t q = s_row0[k]; q < s_row0[k + 1]; ++q) q_k[q] = (uint16_t)k;
    __syncthreads();
    // each row slot's columns (strided), then a block scan of the tile counts
    for (int q = tid; q < R; q += kEmitThreads) {
      const int k = q_k[q];
      const uint2 rc = s_rect[k];
      const int tx0 = rc.x & 0xFFFF, tx1 = rc.y & 0xFFFF;
      const int ty = (int)(rc.x >> 16) + (q - (int)s_row0[k]);
      int a, b;
      const int2 wh = s_wh[k];
      support_row(s_sup[k], ty, e.tile_w, e.tile_h, wh.x, wh.y, tx0, tx1, a, b);
      q_tile0[q] = s_tb[k] + (uint32_t)ty * s_ntx[k] + (uint32_t)a;
      q_cnt[q] = (uint16_t)(b - a);
      q_start[q] = b - a;
    }
    __syncthreads();
    block_scan_lds<kEmitRowPer>((uint32_t *)q_start, R, s_wsum);
    for (int q = tid; q < R; q += kEmitThreads) {
      const int k = q_k[q];
      if ((uint32_t)q == s_row0[k]) s_pbase[k] = (uint32_t)q_start[q];
    }
    __syncthreads();
    for (int q = tid; q < R; q += kEmitThreads) {
      const int k = q_k[q];
      q_start[q] = s_off[k] + (int32_t)((uint32_t)q_start[q] - s_pbase[k]);
    }
    __syncthreads();
    // each thread writes kEmitPer consecutive positions: one search for the
    // row slot of its first position (the last slot starting at or before
    // it; slots without tiles share their start with the next slot, which
    // the search then picks), then a forward walk, and 16-byte stores
    const int p0 = tid * kEmitPer;
    if (d0 + (uint64_t)p0 < d1) {
      int q = 0, hi = R - 1;
      while (q < hi) {
        const int mid = (q + hi + 1) >> 1;
        if (q_start[mid] <= p0) q = mid; else hi = mid - 1;
      }
      uint32_t kk[kEmitPer], vv[kEmitPer];
#pragma unroll
      for (int j = 0; j < kEmitPer; ++j) {
        const int p = p0 + j;
        while (q + 1 < R && q_start[q + 1] <= p) ++q;
        const int col = min(p - q_start[q], max((int)q_cnt[q], 1) - 1);
        kk[j] = q_tile0[q] + (uint32_t)max(col, 0);
        vv[j] = s_rec[q_k[q]];
      }
      const uint64_t d = d0 + (uint64_t)p0;
      if (d + kEmitPer <= d1) {
        union { uint4 v[kEmitPer * sizeof(K) / 16]; K k[kEmitPer]; } ku;
#pragma unroll
        for (int j = 0; j < kEmitPer; ++j) ku.k[j] = (K)kk[j];
#pragma unroll
        for (int j = 0; j < (int)(kEmitPer * sizeof(K) / 16); ++j)
          *((uint4 *)(keys_out + d) + j) = ku.v[j];
#pragma unroll
        for (int j = 0; j < kEmitPer; j += 4)
          *(uint4 *)(e.vals_out + d + j) = make_uint4(vv[j], vv[j + 1], vv[j + 2], vv[j + 3]);
      } else {
        for (int j = 0; j < kEmitPer && d + j < d1; ++j) {
          keys_out[d + j] = (K)kk[j];
          e.vals_out[d + j] = vv[j];
        }
      }
    }
  } else {
    // more records or rows than LDS holds: search the offsets in memory and
    // walk the record's rows
    for (int k = 0; k < kEmitPer; ++k) {
      const uint64_t d = d0 + (uint64_t)k * kEmitThreads + tid;
      if (d >= d1) break;
      const int64_t i = last_record_at(e.offs, rlo, rhi, d);
      const uint32_t r = e.order[i];
      const uint2 rc = e.rects[r];
      uint32_t j = (uint32_t)(d - e.offs[i]);
      const int ty0 = (int)(rc.x >> 16), ty1 = (int)(rc.y >> 16);
      const int v = (int)(r / (uint32_t)e.per_view);
      const int li = (int)(r - (uint32_t)v * (uint32_t)e.per_view);
      const int tx0 = rc.x & 0xFFFF, tx1 = rc.y & 0xFFFF;
      const bool gauss = li < e.N;
      Support sup;
      if (gauss) sup = make_support(e.grec[(int64_t)v * e.N + li]);
      const ViewParams &vp = e.views[v];
      int ty = ty0, a = tx0, b = tx1;
      for (; ty < ty1; ++ty) {
        a = tx0;
        b = tx1;
        if (gauss) support_row(sup, ty, e.tile_w, e.tile_h, vp.W, vp.H, tx0, tx1, a, b);
        if (j < (uint32_t)(b - a)) break;
        j -= (uint32_t)(b - a);
      }
      ty = clampi(ty, ty0, ty1 - 1);
      const int tx = clampi(a + (int)min(j, 0xFFFFu), tx0, tx1 - 1);
      keys_out[d] = (K)global_tile(e, r, ty, tx);
      e.vals_out[d] = r;
    }
  }
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Turns the scanned total into the frame's duplicate count (clamped to the
// key capacity, overflow flagged) and resets the persistent blend's queue.
__global__ void frame_info_kernel(const uint64_t *__restrict__ total, uint64_t cap,
                                  int sorted_in, FrameInfo *__restrict__ fi) {
  const uint64_t raw = *total;
  fi->n_dup = (uint32_t)(raw < cap ? raw : cap);
  if (raw > cap) fi->overflow = 1u;
  fi->sorted_in = sorted_in;
  fi->queue = 0u;
}

// Tile ranges from the sorted tile ids: 4 consecutive ids per thread, a
// range starts or ends where the id changes.
template <typename K>
__global__ void tile_ranges_kernel(const K *__restrict__ k0, const K *__restrict__ k1,
                                   const FrameInfo *__restrict__ fi, uint2 *__restrict__ ranges) {
  const uint64_t i0 = 4 * ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x);
  const uint64_t n = fi->n_dup;
  if (i0 >= n) return;
  const K *keys = fi->sorted_in ? k1 : k0;
  uint32_t k[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) k[j] = i0 + j < n ? (uint32_t)keys[i0 + j] : 0xFFFFFFFFu;
  uint32_t prev = i0 > 0 ? (uint32_t)keys[i0 - 1] : 0xFFFFFFFFu;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint64_t i = i0 + j;
    if (i >= n) break;
    const uint32_t t = k[j];
    if (i == 0 || prev != t) ranges[t].x = (uint32_t)i;
    if (i == n - 1 || k[j + 1] != t) ranges[t].y = (uint32_t)(i + 1);
    prev = t;
  }
}

// Sorted pairs in the exported (tile << 32 | depth key bits) form.
template <typename K>
__global__ void expand_keys_kernel(const K *__restrict__ k0, const K *__restrict__ k1,
                                   const uint32_t *__restrict__ v0, const uint32_t *__restrict__ v1,
                                   const uint32_t *__restrict__ depth,
                                   const FrameInfo *__restrict__ fi, uint64_t *__restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= fi->n_dup) return;
  const uint32_t t = (uint32_t)(fi->sorted_in ? k1 : k0)[i];
  const uint32_t r = (fi->sorted_in ? v1 : v0)[i];
  out[i] = ((uint64_t)t << 32) | (uint64_t)depth[r];
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
  return excl_scan<uint64_t>(c->stream, data, n, tmp);
}

hipError_t launch_exclusive_scan_u32(Ctx *c, uint32_t *data, int64_t n, uint32_t *tmp) {
  return excl_scan<uint32_t>(c->stream, data, n, tmp);
}

size_t emit_blocks_bytes(uint64_t n) { return (size_t)((n + kEmitSpan - 1) / kEmitSpan + 2) * 4; }

hipError_t launch_fill_u32(Ctx *c, uint32_t *p, int64_t n, uint32_t v) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, c->stream, p, n, v);
  return hipGetLastError();
}

hipError_t launch_view_sums(Ctx *c, unsigned long long *sums) {
  hipError_t e = launch_fill_u32(c, (uint32_t *)sums, 2 * (int64_t)c->V, 0u);
  const int64_t per = (int64_t)c->N + c->T;
  if (e != hipSuccess || per == 0) return e;
  hipLaunchKernelGGL(view_sum_kernel, dim3(ceil_div(per, kScanTile), c->V), dim3(kScanThreads), 0,
                     c->stream, (const uint64_t *)c->counts.p, per, sums);
  return hipGetLastError();
}

// Records in (depth key, record id) order, then their tile counts in that
// order scanned into output offsets (total at index n_records).  The depth
// sort runs four 8-bit passes; those beyond the frame's depth bits (known on
// the device) copy through, so the order lands in dk[0]/dv[0].
hipError_t launch_depth_order(Ctx *c) {
  const int64_t n = c->n_records;
  FrameInfo *fi = (FrameInfo *)c->finfo.p;
  hipError_t e;
  {
    ScopedTimer t(c, K_DEPTH_SORT);
    static_assert(kMinMaxSlots == 64, "one wave folds the slots");
    hipLaunchKernelGGL(depth_range_kernel, dim3(1), dim3(kMinMaxSlots), 0, c->stream,
                       (const uint32_t *)c->minmax.p, fi);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (n == 0) return launch_fill_u32(c, (uint32_t *)c->offs.p, 2, 0u);   // total: 0
    hipLaunchKernelGGL(depth_prep_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, c->stream,
                       (const uint32_t *)c->keys.p, n, (const FrameInfo *)fi,
                       (uint32_t *)c->dk[0].p, (uint32_t *)c->dv[0].p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    uint32_t *k[2] = {(uint32_t *)c->dk[0].p, (uint32_t *)c->dk[1].p};
    uint32_t *v[2] = {(uint32_t *)c->dv[0].p, (uint32_t *)c->dv[1].p};
    e = launch_radix_sort_u32(c, k, v, (uint64_t)n, nullptr, &fi->depth_bits, 32, -1, -1, -1);
    if (e != hipSuccess) return e;
  }
  ScopedTimer t(c, K_SCAN);
  hipLaunchKernelGGL(gather_counts_kernel, dim3(ceil_div(n + 1, 256)), dim3(256), 0, c->stream,
                     (const uint32_t *)c->dv[0].p, n, (const uint64_t *)c->counts.p,
                     (uint64_t *)c->offs.p);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return excl_scan<uint64_t>(c->stream, (uint64_t *)c->offs.p, n + 1, (uint64_t *)c->scan_tmp.p);
}

hipError_t launch_emit_keys(Ctx *c) {
  hipLaunchKernelGGL(frame_info_kernel, dim3(1), dim3(1), 0, c->stream,
                     (const uint64_t *)c->offs.p + c->n_records, (uint64_t)c->key_cap,
                     c->sort_passes & 1, (FrameInfo *)c->finfo.p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || c->n_records == 0) return e;
  if (c->n_launch == 0) return hipSuccess;
  ScopedTimer t(c, K_EMIT);
  const uint32_t nblocks = ceil_div(c->n_launch, kEmitSpan);
  hipLaunchKernelGGL(emit_blocks_kernel, dim3(ceil_div(c->n_records, 256)), dim3(256), 0, c->stream,
                     (const uint64_t *)c->offs.p, c->n_records, (const FrameInfo *)c->finfo.p,
                     nblocks, (uint32_t *)c->blk_first.p);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  EmitArgs a;
  a.views = c->cur_views;
  a.per_view = c->N + c->T;
  a.N = c->N;
  a.tile_w = c->tile_w;
  a.tile_h = c->tile_h;
  a.n_records = c->n_records;
  a.order = (const uint32_t *)c->dv[0].p;
  a.rects = (const uint2 *)c->rects.p;
  a.offs = (const uint64_t *)c->offs.p;
  a.grec = (const GaussRec *)c->grec.p;
  a.fi = (const FrameInfo *)c->finfo.p;
  a.blk_first = (const uint32_t *)c->blk_first.p;
  a.keys_out = c->k0.p;
  a.vals_out = (uint32_t *)c->v0.p;
  if (c->key16)
    hipLaunchKernelGGL(emit_balanced_kernel<uint16_t>, dim3(nblocks), dim3(kEmitThreads), 0,
                       c->stream, a);
  else
    hipLaunchKernelGGL(emit_balanced_kernel<uint32_t>, dim3(nblocks), dim3(kEmitThreads), 0,
                       c->stream, a);
  return hipGetLastError();
}

// Duplicates by global tile id: radix passes over the tile bits, element
// count read on the device.
hipError_t launch_tile_sort(Ctx *c) {
  uint32_t *v[2] = {(uint32_t *)c->v0.p, (uint32_t *)c->v1.p};
  const uint32_t *n_dev = &((const FrameInfo *)c->finfo.p)->n_dup;
  if (c->key16) {
    uint16_t *k[2] = {(uint16_t *)c->k0.p, (uint16_t *)c->k1.p};
    return launch_radix_sort_u16(c, k, v, c->n_launch, n_dev, c->tile_bits, K_SORT_UPSWEEP,
                                 K_SORT_SCAN, K_SORT_DOWNSWEEP);
  }
  uint32_t *k[2] = {(uint32_t *)c->k0.p, (uint32_t *)c->k1.p};
  return launch_radix_sort_u32(c, k, v, c->n_launch, n_dev, nullptr, c->tile_bits, K_SORT_UPSWEEP,
                               K_SORT_SCAN, K_SORT_DOWNSWEEP);
}

hipError_t launch_tile_ranges(Ctx *c) {
  ScopedTimer t(c, K_RANGES);
  hipError_t e = launch_fill_u32(c, (uint32_t *)c->ranges.p, 2 * c->n_tiles, 0u);
  if (e != hipSuccess || c->n_launch == 0) return e;
  if (c->key16)
    hipLaunchKernelGGL(tile_ranges_kernel<uint16_t>, dim3(ceil_div(c->n_launch, 1024)), dim3(256),
                       0, c->stream, (const uint16_t *)c->k0.p, (const uint16_t *)c->k1.p,
                       (const FrameInfo *)c->finfo.p, (uint2 *)c->ranges.p);
  else
    hipLaunchKernelGGL(tile_ranges_kernel<uint32_t>, dim3(ceil_div(c->n_launch, 1024)), dim3(256),
                       0, c->stream, (const uint32_t *)c->k0.p, (const uint32_t *)c->k1.p,
                       (const FrameInfo *)c->finfo.p, (uint2 *)c->ranges.p);
  return hipGetLastError();
}

hipError_t launch_expand_keys(Ctx *c, uint64_t *dst) {
  if (c->n_launch == 0) return hipSuccess;
  if (c->key16)
    hipLaunchKernelGGL(expand_keys_kernel<uint16_t>, dim3(ceil_div(c->n_launch, 256)), dim3(256), 0,
                       c->stream, (const uint16_t *)c->k0.p, (const uint16_t *)c->k1.p,
                       (const uint32_t *)c->v0.p, (const uint32_t *)c->v1.p,
                       (const uint32_t *)c->keys.p, (const FrameInfo *)c->finfo.p, dst);
  else
    hipLaunchKernelGGL(expand_keys_kernel<uint32_t>, dim3(ceil_div(c->n_launch, 256)), dim3(256), 0,
                       c->stream, (const uint32_t *)c->k0.p, (const uint32_t *)c->k1.p,
                       (const uint32_t *)c->v0.p, (const uint32_t *)c->v1.p,
                       (const uint32_t *)c->keys.p, (const FrameInfo *)c->finfo.p, dst);
  return hipGetLastError();
}

}  // namespace umgs
