// Bin and sort stages: every tile's list of the records whose support
// reaches it, front to back, built as a two-digit MSD counting sort whose
// digits are the supertile (8 x 8 tiles) and the tile inside it.
//
//  1. The records are put in depth order (a radix sort of one key per
//     record, values = record ids, so equal depths keep id order).
//  2. First level: every record emits one (supertile, record) entry per
//     supertile its support reaches, in depth order at its scanned offset,
//     and a stable radix sort by supertile id (sort.hip) leaves each
//     supertile's entries front to back.
//     Each entry carries a 64-bit mask of the supertile's tiles its support
//     reaches (the support rows the projection counted), sorted with it.
//  3. Second level, per chunk of a supertile's entries: per-chunk tile
//     counts, their prefix over the supertile's chunks and over all tiles,
//     then each entry's record id written to every tile of its mask at its
//     rank there.
//
// No per-duplicate key is ever stored: each duplicate's record id is written
// once, to its final place, and the tile ranges come out of the tile scan.
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

// Single-launch exclusive scan (at most kLbMaxTiles tiles; 64-bit data with
// tile totals below 2^63).  Tiles take tickets in launch order; each
// publishes its total with a ready flag (bit 63) in one 64-bit word, then
// adds the totals of all earlier tiles, read
// in parallel (one thread per earlier tile), so no tile waits on a chain of
// prefixes -- only on its predecessors having published, and those hold
// earlier tickets, so they are running or done.  The wait is bounded: past
// the limit the tile records a fault and goes on, so every wave exits.  The
// last tile to finish zeroes the state for the next scan.
constexpr uint32_t kLbSpinLimit = 1u << 20;
constexpr unsigned long long kLbReady = 1ull << 63;

// Scan input: the data in place (0 past the end).
template <typename T>
struct LoadPlain {
  const T *d;
  __device__ T operator()(int64_t i, int64_t n) const { return i < n ? d[i] : T(0); }
};

// zero_p[0, zero_n) is cleared by the grid on the side (may be empty).
template <typename T, typename L>
__global__ __launch_bounds__(kScanThreads) void scan_lookback_kernel(
    T *__restrict__ data, int64_t n, L load, uint32_t ntiles, LbState *__restrict__ st,
    uint32_t *__restrict__ fault, uint32_t *__restrict__ zero_p, int64_t zero_n) {
  __shared__ uint32_t s_tile;
  __shared__ bool s_last;
  if (threadIdx.x == 0) s_tile = atomicAdd(&st->ticket, 1u);
  __syncthreads();
  const uint32_t t = s_tile;
  const int64_t base = (int64_t)t * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = load(base + k, n);
    s += v[k];
  }
  for (int64_t k = (int64_t)t * kScanThreads + threadIdx.x; k < zero_n;
       k += (int64_t)ntiles * kScanThreads)
    zero_p[k] = 0u;
  T total;
  const T excl = block_excl_scan(s, total);
  if (threadIdx.x == 0)
    __hip_atomic_store(&st->status[t], kLbReady | (unsigned long long)total, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  T pre = 0;
  for (uint32_t k = threadIdx.x; k < t; k += kScanThreads) {
    unsigned long long w =
        __hip_atomic_load(&st->status[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (uint32_t spin = 0; !(w & kLbReady) && spin < kLbSpinLimit; ++spin) {
      __builtin_amdgcn_s_sleep(1);
      w = __hip_atomic_load(&st->status[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!(w & kLbReady)) atomicOr(fault, 1u);
    pre += (T)(w & ~kLbReady);
  }
  T pre_total;
  block_excl_scan(pre, pre_total);
  T run = excl + pre_total;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    if (idx < n) data[idx] = run;
    run += v[k];
  }
  // every thread of this tile is past its reads of the state
  if (threadIdx.x == 0) s_last = atomicAdd(&st->done, 1u) == ntiles - 1;
  __syncthreads();
  if (s_last) {
    for (uint32_t k = threadIdx.x; k < ntiles; k += kScanThreads)
      __hip_atomic_store(&st->status[k], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0) {
      __hip_atomic_store(&st->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&st->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// The entry offsets of the bin stage in one launch: the look-back scan above
// over the supertile-entry counts (high 32 bits of a record's count)
// gathered in depth order, which also sums the tile counts (low 32 bits) and
// leaves both frame totals: each tile's status word carries its entry total
// (bits 0-31) and its tile total (bits 32-62; a tile of 4096 records stays
// far below 2^31), and the last tile to finish adds up every status.  It
// clears the supertile ranges on the side.
__global__ __launch_bounds__(kScanThreads) void entry_offsets_kernel(
    const uint32_t *__restrict__ order, const uint64_t *__restrict__ counts, int64_t n_rec,
    uint64_t *__restrict__ offs, uint32_t ntiles, LbState *__restrict__ st,
    uint32_t *__restrict__ fault, uint32_t *__restrict__ st_rng, int64_t n_rng,
    uint64_t *__restrict__ totals) {
  __shared__ uint32_t s_tile;
  __shared__ bool s_last;
  if (threadIdx.x == 0) s_tile = atomicAdd(&st->ticket, 1u);
  __syncthreads();
  const uint32_t t = s_tile;
  const int64_t base = (int64_t)t * kScanTile + (int64_t)threadIdx.x * kScanItems;
  const int64_t n = n_rec + 1;
  uint32_t v[kScanItems];
  uint32_t s = 0, tl = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    const uint64_t c = idx < n_rec ? counts[order[idx]] : 0ull;
    v[k] = (uint32_t)(c >> 32);
    s += v[k];
    tl += (uint32_t)c;
  }
  for (int64_t k = (int64_t)t * kScanThreads + threadIdx.x; k < n_rng;
       k += (int64_t)ntiles * kScanThreads)
    st_rng[k] = 0u;
  uint32_t total, tl_total;
  const uint32_t excl = block_excl_scan(s, total);
  block_excl_scan(tl, tl_total);
  if (threadIdx.x == 0)
    __hip_atomic_store(&st->status[t],
                       kLbReady | ((unsigned long long)tl_total << 32) | (unsigned long long)total,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // one thread per earlier tile (bounded wait, as in scan_lookback_kernel)
  auto status_of = [&](uint32_t k) {
    unsigned long long w =
        __hip_atomic_load(&st->status[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (uint32_t spin = 0; !(w & kLbReady) && spin < kLbSpinLimit; ++spin) {
      __builtin_amdgcn_s_sleep(1);
      w = __hip_atomic_load(&st->status[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!(w & kLbReady)) atomicOr(fault, 1u);
    return w;
  };
  uint64_t pre = 0;
  for (uint32_t k = threadIdx.x; k < t; k += kScanThreads) pre += status_of(k) & 0xFFFFFFFFull;
  uint64_t pre_total;
  block_excl_scan(pre, pre_total);
  uint64_t run = pre_total + excl;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    if (idx < n) offs[idx] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) s_last = atomicAdd(&st->done, 1u) == ntiles - 1;
  __syncthreads();
  if (s_last) {
    // the frame totals: tiles of the records' rectangles, entries
    uint64_t a = 0, b = 0;
    for (uint32_t k = threadIdx.x; k < ntiles; k += kScanThreads) {
      const unsigned long long w = status_of(k);
      a += (w >> 32) & 0x7FFFFFFFull;
      b += w & 0xFFFFFFFFull;
    }
    uint64_t ta, tb;
    block_excl_scan(a, ta);
    block_excl_scan(b, tb);
    if (threadIdx.x == 0) {
      totals[0] = ta;
      totals[1] = tb;
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < ntiles; k += kScanThreads)
      __hip_atomic_store(&st->status[k], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0) {
      __hip_atomic_store(&st->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&st->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
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

// Per-view duplicate totals (records are view-major; the low 32 bits of a
// record's count are its tiles): one partial sum per block, one atomic per
// block.
__global__ void view_sum_kernel(const uint64_t *__restrict__ counts, int64_t per_view,
                                unsigned long long *__restrict__ sums) {
  const int v = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kScanTile;
  uint64_t s = 0;
  for (int k = threadIdx.x; k < kScanTile; k += kScanThreads)
    if (i + k < per_view) s += counts[(int64_t)v * per_view + i + k] & 0xFFFFFFFFull;
  uint64_t total;
  block_excl_scan(s, total);
  if (threadIdx.x == 0 && total) atomicAdd(sums + v, (unsigned long long)total);
}

// Frame totals: duplicates (sum of the view totals) and supertile entries
// (the scanned entry counts' total).
__global__ void frame_totals_kernel(const unsigned long long *__restrict__ view_sums, int V,
                                    const uint64_t *__restrict__ st_total,
                                    uint64_t *__restrict__ totals) {
  uint64_t s = 0;
  for (int v = threadIdx.x; v < V; v += 64) s += view_sums[v];
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if (threadIdx.x == 0) {
    totals[0] = s;
    totals[1] = *st_total;
  }
}

// Depth range of the frame: sort keys hold (depth key - base) in depth_bits.
// One wave folds the slot pairs the projection kernels filled.
// It also clears the per-view duplicate sums (V x uint64) the count stage
// adds into.
constexpr int kRangeThreads = 1024;

// Folds the projection's depth-key range slots into the frame info and
// resets them for the next projection (each thread reads and resets its own
// slots); also clears the per-view sums.
__global__ __launch_bounds__(kRangeThreads) void depth_range_kernel(
    uint32_t *__restrict__ minmax, FrameInfo *__restrict__ fi,
    uint32_t *__restrict__ view_sums, int V) {
  __shared__ uint32_t wlo[kRangeThreads / 64], whi[kRangeThreads / 64];
  for (int k = threadIdx.x; k < 2 * V; k += blockDim.x) view_sums[k] = 0u;
  uint32_t l = kCulled, h = 0u;
  for (int k = threadIdx.x; k < kMinMaxSlots; k += kRangeThreads) {
    l = min(l, minmax[k]);
    h = max(h, minmax[kMinMaxSlots + k]);
    minmax[k] = kCulled;
    minmax[kMinMaxSlots + k] = 0u;
  }
  l = wave_min_u32(l);
  h = wave_max_u32(h);
  if ((threadIdx.x & 63) == 0) {
    wlo[threadIdx.x >> 6] = l;
    whi[threadIdx.x >> 6] = h;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  uint32_t lo = wlo[0], hi = whi[0];
  for (int k = 1; k < kRangeThreads / 64; ++k) {
    lo = min(lo, wlo[k]);
    hi = max(hi, whi[k]);
  }
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

// Supertile-entry counts (high 32 bits of a record's count) in depth order;
// the entry past the end receives 0, so the scan leaves the total there.
// The grid also clears the supertile ranges (empty supertiles keep [0, 0)).
__global__ void gather_st_counts_kernel(const uint32_t *__restrict__ order, int64_t n,
                                        const uint64_t *__restrict__ counts,
                                        uint64_t *__restrict__ out, uint32_t *__restrict__ st_rng,
                                        int64_t n_rng) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = counts[order[i]] >> 32;
  else if (i == n) out[n] = 0;
  for (int64_t k = i; k < n_rng; k += (int64_t)gridDim.x * blockDim.x) st_rng[k] = 0u;
}

// Resets the depth-key range slots the projection folds into.
__global__ void minmax_reset_kernel(uint32_t *__restrict__ minmax) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < 2 * kMinMaxSlots) minmax[k] = k < kMinMaxSlots ? kCulled : 0u;
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// The frame's sizes on the device, each clamped to its buffer's capacity
// (overflow flagged, sticky).  The
// duplicates are bounded by the records' rectangles here; the tile scan
// replaces the bound by the exact count (ranges_kernel).
__global__ void frame_info_kernel(const uint64_t *__restrict__ totals, uint64_t cap,
                                  uint64_t st_cap, FrameInfo *__restrict__ fi) {
  const uint64_t nd = totals[0], n1 = totals[1];
  fi->n_dup = (uint32_t)(nd < cap ? nd : cap);
  fi->n1 = (uint32_t)(n1 < st_cap ? n1 : st_cap);
  if (n1 > st_cap || nd >= 0xFFFF0000ull) fi->overflow = 1u;
  fi->sorted_in = 0;
  fi->queue = 0u;
}

// ---- first level: supertile entries -----------------------------------------

struct StEmitArgs {
  const ViewParams *views;
  int per_view, N, tile_w, tile_h;
  int64_t n_records;
  const uint32_t *order;   // records in depth order
  const uint2 *rects;
  const uint64_t *offs;    // scanned entry counts in depth order
  const GaussRec *grec;
  const FrameInfo *fi;
  void *keys;              // K global supertile ids
  uint32_t *vals;          // record ids
  uint64_t *masks;         // tiles of the supertile the record reaches (mask kernel)
};

__device__ __forceinline__ void unpack_rect(uint2 rc, int &tx0, int &ty0, int &tx1, int &ty1) {
  tx0 = rc.x & 0xFFFF;
  ty0 = rc.x >> 16;
  tx1 = rc.y & 0xFFFF;
  ty1 = rc.y >> 16;
}

// Entries of a record: one per supertile of its tile rectangle, rows top to
// bottom, columns left to right (their order within a record does not
// matter; the sort by supertile is stable over records in depth order).
// A wave takes 64 consecutive records and writes their entries -- one
// contiguous run of the output -- with consecutive lanes on consecutive
// entries: each lane finds its entry's record by binary search over the 64
// records' first entries (LDS), so a record with many supertiles does not
// hold the others' lanes, and every store is coalesced.
template <typename K>
__global__ __launch_bounds__(256) void st_emit_kernel(StEmitArgs e) {
  __shared__ uint32_t s_p0[4][64], s_rec[4][64], s_base[4][64], s_dim[4][64];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + tid;
  const uint32_t n1 = e.fi->n1;
  uint32_t p0 = 0xFFFFFFFFu, p1 = 0u, r = 0u, base = 0u, dim = 1u;
  if (i < e.n_records) {
    p0 = (uint32_t)min(e.offs[i], (uint64_t)n1);
    p1 = (uint32_t)min(e.offs[i + 1], (uint64_t)n1);
    if (p1 > p0) {
      r = e.order[i];
      int tx0, ty0, tx1, ty1;
      unpack_rect(e.rects[r], tx0, ty0, tx1, ty1);
      const uint32_t v = r / (uint32_t)e.per_view;
      const ViewParams &vp = e.views[v];
      const uint32_t nstx = (uint32_t)(vp.ntx + kST - 1) >> kSTLog;
      const uint32_t sx0 = (uint32_t)tx0 >> kSTLog, sy0 = (uint32_t)ty0 >> kSTLog;
      const uint32_t nsx = (((uint32_t)tx1 - 1) >> kSTLog) - sx0 + 1;
      base = vp.st_base + sy0 * nstx + sx0;
      dim = nsx | (nstx << 16);
    }
  }
  s_p0[w][lane] = p0;
  s_rec[w][lane] = r;
  s_base[w][lane] = base;
  s_dim[w][lane] = dim;
  // the wave's entries: [first entry of its first record, last end)
  const uint32_t first = (uint32_t)__builtin_amdgcn_readfirstlane((int)p0);
  const uint32_t last = wave_max_u32(p1);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  K *keys = (K *)e.keys;
  for (uint32_t en = first + lane; en < last; en += 64) {
    // the last record (lane) whose first entry is at or before en
    int lo = 0, hi = 64;
#pragma unroll
    for (int step = 0; step < 6; ++step) {
      const int mid = (lo + hi) >> 1;
      if (s_p0[w][mid] <= en) lo = mid; else hi = mid;
    }
    const uint32_t k = en - s_p0[w][lo];
    const uint32_t dm = s_dim[w][lo], nsx = dm & 0xFFFFu, nstx = dm >> 16;
    const uint32_t q = k / nsx;
    keys[en] = (K)(s_base[w][lo] + q * nstx + (k - q * nsx));
    e.vals[en] = s_rec[w][lo];
  }
}

// One thread per entry (in emit order, so neighbouring threads mostly share
// a record): the mask of the supertile's tiles the record reaches -- the
// support rows of the projection's count, cut to the supertile.
template <typename K>
__global__ void st_mask_kernel(StEmitArgs e) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= e.fi->n1) return;
  const uint32_t s = (uint32_t)((const K *)e.keys)[i];
  const uint32_t r = e.vals[i];
  int tx0, ty0, tx1, ty1;
  unpack_rect(e.rects[r], tx0, ty0, tx1, ty1);
  const uint32_t v = r / (uint32_t)e.per_view;
  const int li = (int)(r - v * (uint32_t)e.per_view);
  const ViewParams &vp = e.views[v];
  Support sup;
  sup.exact = false;
  if (li < e.N) sup = make_support(e.grec[(int64_t)v * e.N + li]);
  const uint32_t nstx = (uint32_t)(vp.ntx + kST - 1) >> kSTLog;
  const uint32_t sl = s - vp.st_base;
  const uint32_t sy = sl / nstx;
  e.masks[i] = st_mask(sup, (int)(sl - sy * nstx), (int)sy, tx0, ty0, tx1, ty1,
                       __builtin_ctz((unsigned)e.tile_w), __builtin_ctz((unsigned)e.tile_h), vp.W,
                       vp.H);
}

// Per-supertile [start, end) of the sorted entries: 4 consecutive ids per
// thread, a range starts or ends where the id changes.
template <typename K>
__global__ void st_ranges_kernel(const K *__restrict__ keys, const FrameInfo *__restrict__ fi,
                                 uint2 *__restrict__ rng) {
  const uint64_t i0 = 4 * ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x);
  const uint64_t n = fi->n1;
  if (i0 >= n) return;
  uint32_t k[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) k[j] = i0 + j < n ? (uint32_t)keys[i0 + j] : 0xFFFFFFFFu;
  uint32_t prev = i0 > 0 ? (uint32_t)keys[i0 - 1] : 0xFFFFFFFFu;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint64_t i = i0 + j;
    if (i >= n) break;
    const uint32_t s = k[j];
    if (i == 0 || prev != s) rng[s].x = (uint32_t)i;
    if (i == n - 1 || k[j + 1] != s) rng[s].y = (uint32_t)(i + 1);
    prev = s;
  }
}

// ---- second level: tiles inside a supertile ---------------------------------

constexpr int kChunk = 1024;          // entries of one supertile's list per workgroup
constexpr int kL2Threads = 256;
constexpr int kL2Waves = kL2Threads / 64;

// Chunks per supertile (the entry past the end receives 0 for the scan).
__global__ void st_chunks_kernel(const uint2 *__restrict__ rng, int64_t n_st,
                                 uint32_t *__restrict__ chunk_base) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n_st) {
    const uint2 r = rng[s];
    chunk_base[s] = r.y > r.x ? (r.y - r.x + kChunk - 1) / kChunk : 0u;
  } else if (s == n_st) {
    chunk_base[n_st] = 0;
  }
}

__global__ void chunk_total_kernel(const uint32_t *__restrict__ chunk_base, int64_t n_st,
                                   FrameInfo *__restrict__ fi) {
  fi->n_chunks = chunk_base[n_st];
}

// A second-level chunk: entries [e0, e0 + n) of the supertile whose first
// tile is (cxy & 0xFFFF, cxy >> 16) in view v, the supertile's chunk k
// (nk = n | k << 11; n <= kChunk = 1024).
struct __align__(16) ChunkRec {
  uint32_t e0, nk, v, cxy;
};

// The view whose supertiles [st_base, next st_base) hold s.
__device__ __forceinline__ int view_of_st(const ViewParams *views, int V, uint32_t s) {
  int lo = 0, hi = V - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].st_base <= s) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// One thread per supertile writes the records of its chunks.
__global__ void chunk_table_kernel(const ViewParams *__restrict__ views, int V,
                                   const uint2 *__restrict__ rng, const uint32_t *__restrict__ chunk_base,
                                   int64_t n_st, ChunkRec *__restrict__ tab) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_st) return;
  const uint32_t c0 = chunk_base[s], c1 = chunk_base[s + 1];
  if (c0 >= c1) return;
  const uint2 r = rng[s];
  const int v = view_of_st(views, V, (uint32_t)s);
  const ViewParams &vp = views[v];
  const uint32_t sl = (uint32_t)s - vp.st_base;
  const uint32_t nstx = (uint32_t)(vp.ntx + kST - 1) >> kSTLog;
  const uint32_t cxy = ((sl % nstx) << kSTLog) | ((sl / nstx) << (kSTLog + 16));
  for (uint32_t c = c0; c < c1; ++c) {
    ChunkRec k;
    k.e0 = r.x + (c - c0) * (uint32_t)kChunk;
    k.nk = (min(k.e0 + (uint32_t)kChunk, r.y) - k.e0) | ((c - c0) << 11);
    k.v = (uint32_t)v;
    k.cxy = cxy;
    tab[c] = k;
  }
}

// The three steps above in one launch, for frames of at most kScanTile - 1
// supertiles: every workgroup takes the chunk counts and their exclusive
// scan (in LDS; workgroup 0 also leaves it in chunk_base and the total in
// the frame info), then builds the table entries of its own chunks, one
// thread per chunk (its supertile found by binary search in the scanned
// counts), so no thread waits on more than one chain of loads.
__global__ __launch_bounds__(kScanThreads) void chunk_plan_kernel(
    const ViewParams *__restrict__ views, int V, const uint2 *__restrict__ rng, int64_t n_st,
    uint32_t *__restrict__ chunk_base, FrameInfo *__restrict__ fi, ChunkRec *__restrict__ tab) {
  __shared__ uint32_t cb[kScanTile];
  __shared__ uint32_t s_total;
  const int64_t s0 = (int64_t)threadIdx.x * kScanItems;
  uint32_t cnt[kScanItems];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t s = s0 + k;
    uint32_t n = 0;
    if (s < n_st) {
      const uint2 r = rng[s];
      n = r.y > r.x ? (r.y - r.x + kChunk - 1) / kChunk : 0u;
    }
    cnt[k] = n;
    sum += n;
  }
  uint32_t total;
  uint32_t run = block_excl_scan(sum, total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t s = s0 + k;
    if (s <= n_st) {
      if (blockIdx.x == 0) chunk_base[s] = run;
      cb[s] = run;
    }
    run += cnt[k];
  }
  if (threadIdx.x == 0) {
    if (blockIdx.x == 0) fi->n_chunks = total;
    s_total = total;
  }
  __syncthreads();
  const uint32_t nc = s_total;
  for (uint32_t c = blockIdx.x * kScanThreads + threadIdx.x; c < nc; c += gridDim.x * kScanThreads) {
    // last supertile s with cb[s] <= c (cb is non-decreasing, cb[0] = 0)
    uint32_t lo = 0, hi = (uint32_t)n_st;   // cb[lo] <= c < cb[hi]
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (cb[mid] <= c) lo = mid; else hi = mid;
    }
    const uint32_t s = lo;
    const uint2 r = rng[s];
    const int v = view_of_st(views, V, s);
    const ViewParams &vp = views[v];
    const uint32_t sl = s - vp.st_base;
    const uint32_t nstx = (uint32_t)(vp.ntx + kST - 1) >> kSTLog;
    const uint32_t k = c - cb[s];
    ChunkRec ck;
    ck.e0 = r.x + k * (uint32_t)kChunk;
    ck.nk = (min(ck.e0 + (uint32_t)kChunk, r.y) - ck.e0) | (k << 11);
    ck.v = (uint32_t)v;
    ck.cxy = ((sl % nstx) << kSTLog) | ((sl / nstx) << (kSTLog + 16));
    tab[c] = ck;
  }
}

struct L2Args {
  const ViewParams *views;
  int V, per_view, N, tile_w, tile_h;
  int64_t n_st, n_tiles;
  const uint2 *st_rng;         // per supertile [start, end) of its sorted entries
  const uint32_t *chunk_base;  // scanned chunks per supertile (n_st + 1)
  const ChunkRec *chunks;      // per chunk: its entries, view and supertile
  const uint32_t *rec;         // sorted entries' record ids
  const FrameInfo *fi;
  const uint64_t *masks;       // sorted entries' masks: tiles of the supertile they reach
  uint32_t *cnt;               // per chunk 64 tile counts
  uint32_t *tstart;            // per tile: count, then (scanned) first position
  uint32_t *out;               // record ids in tile order
  uint32_t cap;                // record ids out holds
};

// The wave's 64 x 64 bit matrix (row i = lane i's m) transposed: lane j's
// result has bit i set iff lane i's m has bit j set.  Six stages swap the
// off-diagonal blocks of 32, 16, ..., 1 bits between lanes i and i ^ s; in
// the 32-bit stages the lower lane of a pair keeps the bit positions of
// mask_s (positions whose bit s is clear) and takes the rest from the upper
// lane's word rotated left by s, the upper lane keeps the other positions
// and takes the lower lane's word rotated right by s (one alignbit and one
// bitfield insert per word and stage).
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t m) {
  const int lane = (int)__lane_id();
  uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
  {
    const bool low = lane < 32;
    const uint32_t r = (uint32_t)__shfl_xor((int)(low ? hi : lo), 32, 64);
    hi = low ? r : hi;
    lo = low ? lo : r;
  }
  constexpr uint32_t kMask[5] = {0x0000FFFFu, 0x00FF00FFu, 0x0F0F0F0Fu, 0x33333333u, 0x55555555u};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int s = 16 >> k;
    const bool low = (lane & s) == 0;
    const uint32_t keep = low ? kMask[k] : ~kMask[k];
    const uint32_t rot = low ? 32u - (uint32_t)s : (uint32_t)s;   // rotate right by this
    const uint32_t plo = (uint32_t)__shfl_xor((int)lo, s, 64);
    const uint32_t phi = (uint32_t)__shfl_xor((int)hi, s, 64);
    lo = (keep & lo) | (~keep & __builtin_amdgcn_alignbit(plo, plo, rot));
    hi = (keep & hi) | (~keep & __builtin_amdgcn_alignbit(phi, phi, rot));
  }
  return ((uint64_t)hi << 32) | lo;
}

// Lane j's result: how many lanes of the wave have bit j of m set (every
// lane of the wave must be active).
__device__ __forceinline__ uint32_t wave_bit_counts(uint64_t m) {
  return (uint32_t)__popcll(wave_transpose64(m));
}

// A chunk's per-tile counts (bit counts of its entries' masks).
constexpr int kL2Rounds = kChunk / kL2Threads;   // rounds of a chunk: 4 per wave
static_assert(kChunk % kL2Threads == 0, "a chunk is whole rounds of the workgroup");

__global__ __launch_bounds__(kL2Threads) void tile_count_kernel(L2Args a) {
  // consecutive chunks (mostly of one supertile) on one XCD
  const uint32_t c = xcd_block_n(blockIdx.x, a.fi->n_chunks);
  if (c >= a.fi->n_chunks) return;
  __shared__ uint32_t wc[kL2Waves][64];
  const ChunkRec ck = a.chunks[c];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t e1 = ck.e0 + (ck.nk & 0x7FFu);
  // every round's masks in flight at once
  uint64_t m[kL2Rounds];
#pragma unroll
  for (int k = 0; k < kL2Rounds; ++k) {
    const uint32_t e = ck.e0 + (uint32_t)(k * kL2Threads + tid);
    m[k] = e < e1 ? a.masks[e] : 0ull;
  }
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < kL2Rounds; ++k) acc += wave_bit_counts(m[k]);
  wc[w][lane] = acc;
  __syncthreads();
  if (tid < 64) {
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kL2Waves; ++k) s += wc[k][tid];
    a.cnt[(uint64_t)c * 64 + tid] = s;
  }
}

// Per (supertile, tile j): the tile's total over the supertile's chunks, at
// its global tile id (every tile of every view is one (supertile, j) pair),
// and each chunk's count replaced by the sum over the supertile's earlier
// chunks (the chunk's first position inside the tile's part of the lists).
__global__ void tile_prefix_kernel(L2Args a) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0) a.tstart[a.n_tiles] = 0;
  const int64_t s = g >> 6;
  const int j = (int)(g & 63);
  if (s >= a.n_st) return;
  const uint32_t c0 = a.chunk_base[s], c1 = a.chunk_base[s + 1];
  uint32_t run = 0;
  uint32_t c = c0;
  for (; c + 8 <= c1; c += 8) {
    uint32_t x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = a.cnt[(uint64_t)(c + i) * 64 + j];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      a.cnt[(uint64_t)(c + i) * 64 + j] = run;
      run += x[i];
    }
  }
  for (; c < c1; ++c) {
    const uint32_t x = a.cnt[(uint64_t)c * 64 + j];
    a.cnt[(uint64_t)c * 64 + j] = run;
    run += x;
  }
  const int v = view_of_st(a.views, a.V, (uint32_t)s);
  const ViewParams &vp = a.views[v];
  const uint32_t sl = (uint32_t)s - vp.st_base;
  const uint32_t nstx = (uint32_t)(vp.ntx + kST - 1) >> kSTLog;
  const int tx = (int)(sl % nstx) * kST + (j & (kST - 1));
  const int ty = (int)(sl / nstx) * kST + (j >> kSTLog);
  if (tx < vp.ntx && ty < vp.nty) a.tstart[vp.tile_base + (uint32_t)ty * vp.ntx + tx] = run;
}

// Tile ranges from the scanned tile counts, clamped to the capacity of the
// lists; the first thread stores the frame's exact duplicate count (flagging
// an overflow of the capacity).
__global__ void ranges_kernel(const uint32_t *__restrict__ tstart, int64_t n_tiles, uint32_t cap,
                              FrameInfo *__restrict__ fi, uint2 *__restrict__ ranges) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    const uint32_t total = tstart[n_tiles];
    fi->n_dup = min(total, cap);
    if (total > cap) fi->overflow = 1u;
  }
  if (t >= n_tiles) return;
  ranges[t] = make_uint2(min(tstart[t], cap), min(tstart[t + 1], cap));
}

// Each entry's record id to every tile of its mask, at the tile's first
// position + the counts of the supertile's earlier chunks + the entry's rank
// among the chunk's entries with that bit (earlier rounds, earlier waves,
// earlier lanes).
// Stores go tile by tile, so the lanes of a store write consecutive words.
// One round of a wave's 64 entries: for tile j, the lanes whose mask has
// bit j write consecutive positions (rank among them = set bits of the
// ballot below the lane).  CHECKED: some positions may reach the capacity.
template <bool CHECKED>
__device__ __forceinline__ void scatter_round(uint64_t m, uint32_t r, uint32_t off, uint32_t cap,
                                              uint32_t *__restrict__ out) {
  const uint32_t mw[2] = {(uint32_t)m, (uint32_t)(m >> 32)};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll 4
    for (int jj = 0; jj < 32; ++jj) {
      const bool bit = __builtin_amdgcn_ubfe(mw[h], jj, 1) != 0u;
      const uint64_t b = __builtin_amdgcn_ballot_w64(bit);
      if (b == 0) continue;
      const int j = 32 * h + jj;
      // the tile's next position (scalar) and the lane's rank among the
      // lanes with the bit: a scalar base and a 32-bit lane offset
      const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)off, j);
      const uint32_t rank =
          __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
      __builtin_assume(rank < 64u);
      uint32_t *__restrict__ dst = out + o;
      if (bit && (!CHECKED || o + rank < cap)) dst[rank] = r;
    }
  }
}

__global__ __launch_bounds__(kL2Threads) void tile_scatter_kernel(L2Args a) {
  const uint32_t c = xcd_block_n(blockIdx.x, a.fi->n_chunks);
  if (c >= a.fi->n_chunks) return;
  // every list fits (the usual case): no per-position capacity test
  const bool fits = a.tstart[a.n_tiles] <= a.cap;
  __shared__ uint32_t base[64];
  __shared__ uint32_t wc[kL2Rounds * kL2Waves][64];
  const ChunkRec ck = a.chunks[c];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t e1 = ck.e0 + (ck.nk & 0x7FFu);
  // every round's entries in flight at once
  uint64_t m[kL2Rounds];
  uint32_t r[kL2Rounds];
#pragma unroll
  for (int k = 0; k < kL2Rounds; ++k) {
    const uint32_t e = ck.e0 + (uint32_t)(k * kL2Threads + tid);
    const bool valid = e < e1;
    m[k] = valid ? a.masks[e] : 0ull;
    r[k] = valid ? a.rec[e] : 0u;
  }
  if (tid < 64) {
    // the tile's first position + the supertile's earlier chunks' counts
    const ViewParams &vp = a.views[ck.v];
    const int tx = (int)(ck.cxy & 0xFFFF) + (tid & (kST - 1));
    const int ty = (int)(ck.cxy >> 16) + (tid >> kSTLog);
    uint32_t b = 0;
    if (tx < vp.ntx && ty < vp.nty)
      b = a.tstart[vp.tile_base + (uint32_t)ty * vp.ntx + tx] + a.cnt[(uint64_t)c * 64 + tid];
    base[tid] = b;
  }
  // wave-round q = k * waves + w holds entries [e0 + 64 q, e0 + 64 q + 64)
#pragma unroll
  for (int k = 0; k < kL2Rounds; ++k) wc[k * kL2Waves + w][lane] = wave_bit_counts(m[k]);
  __syncthreads();
  // lane j: tile j's first position for each of this wave's rounds (the
  // counts of every earlier wave-round added)
  uint32_t off[kL2Rounds];
  uint32_t run = base[lane];
#pragma unroll
  for (int q = 0; q < kL2Rounds * kL2Waves; ++q) {
    if ((q % kL2Waves) == w) off[q / kL2Waves] = run;
    run += wc[q][lane];
  }
  const uint32_t cap = a.cap;
#pragma unroll
  for (int k = 0; k < kL2Rounds; ++k) {
    if (ck.e0 + (uint32_t)(k * kL2Threads + w * 64) >= e1) break;   // no entries left for this wave
    if (fits)
      scatter_round<false>(m[k], r[k], off[k], cap, a.out);
    else
      scatter_round<true>(m[k], r[k], off[k], cap, a.out);
  }
}

// Sorted pairs in the exported (tile << 32 | depth key bits) form, one block
// per tile.
__global__ void expand_keys_kernel(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
                                   const uint32_t *__restrict__ depth, uint64_t *__restrict__ out) {
  const uint32_t t = blockIdx.x;
  const uint2 r = ranges[t];
  for (uint32_t i = r.x + threadIdx.x; i < r.y; i += blockDim.x)
    out[i] = ((uint64_t)t << 32) | (uint64_t)depth[vals[i]];
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

// Exclusive scans: one launch (look-back) where the state is set up and the
// tile count allows, else reduce, scan of the tile totals, apply.
template <typename T>
hipError_t scan_any(Ctx *c, T *data, int64_t n, T *tmp) {
  const int64_t nt = (n + kScanTile - 1) / kScanTile;
  if (nt <= 1 || nt > kLbMaxTiles || !c->lb_zeroed) return excl_scan<T>(c->stream, data, n, tmp);
  FrameInfo *fi = (FrameInfo *)c->finfo.p;
  hipLaunchKernelGGL((scan_lookback_kernel<T, LoadPlain<T>>), dim3((unsigned)nt),
                     dim3(kScanThreads), 0, c->stream, data, n, LoadPlain<T>{data}, (uint32_t)nt,
                     (LbState *)c->lb.p, &fi->fault, (uint32_t *)nullptr, (int64_t)0);
  return hipGetLastError();
}

hipError_t launch_exclusive_scan_u64(Ctx *c, uint64_t *data, int64_t n, uint64_t *tmp) {
  return scan_any<uint64_t>(c, data, n, tmp);
}

hipError_t launch_exclusive_scan_u32(Ctx *c, uint32_t *data, int64_t n, uint32_t *tmp) {
  return scan_any<uint32_t>(c, data, n, tmp);
}

hipError_t launch_minmax_reset(Ctx *c) {
  hipLaunchKernelGGL(minmax_reset_kernel, dim3(ceil_div(2 * kMinMaxSlots, 256)), dim3(256), 0,
                     c->stream, (uint32_t *)c->minmax.p);
  return hipGetLastError();
}

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

uint64_t max_chunks(uint64_t n1, int64_t n_st) { return n1 / kChunk + (uint64_t)n_st + 1; }
size_t chunk_rec_bytes() { return sizeof(ChunkRec); }

// Records in (depth key, record id) order, their supertile-entry counts in
// that order scanned into entry offsets (total at index n_records), and the
// frame totals (duplicates, entries) in c->totals.  The depth sort runs four
// 8-bit passes; those beyond the frame's depth bits (known on the device)
// copy through, so the order lands in dk[0]/dv[0].
hipError_t launch_depth_order(Ctx *c) {
  const int64_t n = c->n_records;
  FrameInfo *fi = (FrameInfo *)c->finfo.p;
  hipError_t e;
  {
    ScopedTimer t(c, K_DEPTH_SORT);
    hipLaunchKernelGGL(depth_range_kernel, dim3(1), dim3(kRangeThreads), 0, c->stream,
                       (uint32_t *)c->minmax.p, fi, (uint32_t *)c->view_sums.p, c->V);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (n > 0) {
      hipLaunchKernelGGL(depth_prep_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, c->stream,
                         (const uint32_t *)c->keys.p, n, (const FrameInfo *)fi,
                         (uint32_t *)c->dk[0].p, (uint32_t *)c->dv[0].p);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      uint32_t *k[2] = {(uint32_t *)c->dk[0].p, (uint32_t *)c->dk[1].p};
      uint32_t *v[2] = {(uint32_t *)c->dv[0].p, (uint32_t *)c->dv[1].p};
      e = launch_radix_sort_u32(c, k, v, (uint64_t)n, nullptr, &fi->depth_bits, 32, -1, -1, -1);
      if (e != hipSuccess) return e;
    }
  }
  ScopedTimer t(c, K_SCAN);
  const int64_t nt = (n + 1 + kScanTile - 1) / kScanTile;
  if (nt > 1 && nt <= kLbMaxTiles && c->lb_zeroed) {
    // one launch: gather in depth order, scan, both frame totals, clear the
    // supertile ranges
    hipLaunchKernelGGL(entry_offsets_kernel, dim3((unsigned)nt), dim3(kScanThreads), 0, c->stream,
                       (const uint32_t *)c->dv[0].p, (const uint64_t *)c->counts.p, n,
                       (uint64_t *)c->offs.p, (uint32_t)nt, (LbState *)c->lb.p, &fi->fault,
                       (uint32_t *)c->st_rng.p, 2 * c->n_st, (uint64_t *)c->totals.p);
    return hipGetLastError();
  } else {
    hipLaunchKernelGGL(gather_st_counts_kernel, dim3(ceil_div(n + 1, 256)), dim3(256), 0,
                       c->stream, (const uint32_t *)c->dv[0].p, n, (const uint64_t *)c->counts.p,
                       (uint64_t *)c->offs.p, (uint32_t *)c->st_rng.p, 2 * c->n_st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_any<uint64_t>(c, (uint64_t *)c->offs.p, n + 1, (uint64_t *)c->scan_tmp.p)) !=
        hipSuccess)
      return e;
  }
  // the view sums were cleared by depth_range_kernel
  const int64_t per = (int64_t)c->N + c->T;
  if (per > 0) {
    hipLaunchKernelGGL(view_sum_kernel, dim3(ceil_div(per, kScanTile), c->V), dim3(kScanThreads), 0,
                       c->stream, (const uint64_t *)c->counts.p, per,
                       (unsigned long long *)c->view_sums.p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(frame_totals_kernel, dim3(1), dim3(64), 0, c->stream,
                     (const unsigned long long *)c->view_sums.p, c->V,
                     (const uint64_t *)c->offs.p + n, (uint64_t *)c->totals.p);
  return hipGetLastError();
}

// Frame sizes on the device, then the first level: supertile entries in
// depth order, sorted by supertile, and the supertiles' ranges and chunks.
hipError_t launch_st_bin(Ctx *c) {
  FrameInfo *fi = (FrameInfo *)c->finfo.p;
  hipLaunchKernelGGL(frame_info_kernel, dim3(1), dim3(1), 0, c->stream,
                     (const uint64_t *)c->totals.p, (uint64_t)c->key_cap, (uint64_t)c->st_cap, fi);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  uint32_t *cb = (uint32_t *)c->chunk_base.p;
  if (c->n_records == 0 || c->st_launch == 0) {
    if ((e = launch_fill_u32(c, cb, c->n_st + 1, 0u)) != hipSuccess) return e;
    hipLaunchKernelGGL(chunk_total_kernel, dim3(1), dim3(1), 0, c->stream, (const uint32_t *)cb,
                       c->n_st, fi);
    return hipGetLastError();
  }
  {
    ScopedTimer t(c, K_EMIT);
    StEmitArgs a;
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
    a.fi = fi;
    a.keys = c->sk[0].p;
    a.vals = (uint32_t *)c->sv[0].p;
    a.masks = (uint64_t *)c->masks[0].p;
    if (c->st_key16)
      hipLaunchKernelGGL(st_emit_kernel<uint16_t>, dim3(ceil_div(c->n_records, 256)), dim3(256), 0,
                         c->stream, a);
    else
      hipLaunchKernelGGL(st_emit_kernel<uint32_t>, dim3(ceil_div(c->n_records, 256)), dim3(256), 0,
                         c->stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    ScopedTimer t(c, K_ST_MASK);
    StEmitArgs a;
    a.views = c->cur_views;
    a.per_view = c->N + c->T;
    a.N = c->N;
    a.tile_w = c->tile_w;
    a.tile_h = c->tile_h;
    a.n_records = c->n_records;
    a.rects = (const uint2 *)c->rects.p;
    a.grec = (const GaussRec *)c->grec.p;
    a.fi = fi;
    a.keys = c->sk[0].p;
    a.vals = (uint32_t *)c->sv[0].p;
    a.masks = (uint64_t *)c->masks[0].p;
    if (c->st_key16)
      hipLaunchKernelGGL(st_mask_kernel<uint16_t>, dim3(ceil_div(c->st_launch, 256)), dim3(256), 0,
                         c->stream, a);
    else
      hipLaunchKernelGGL(st_mask_kernel<uint32_t>, dim3(ceil_div(c->st_launch, 256)), dim3(256), 0,
                         c->stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  uint32_t *v[2] = {(uint32_t *)c->sv[0].p, (uint32_t *)c->sv[1].p};
  uint64_t *m[2] = {(uint64_t *)c->masks[0].p, (uint64_t *)c->masks[1].p};
  const uint32_t *n_dev = &fi->n1;
  const int out = radix_passes(c->st_bits) & 1;
  if (c->st_key16) {
    uint16_t *k[2] = {(uint16_t *)c->sk[0].p, (uint16_t *)c->sk[1].p};
    e = launch_radix_sort_pay_u16(c, k, v, m, c->st_launch, n_dev, c->st_bits, K_SORT_UPSWEEP,
                                  K_SORT_SCAN, K_SORT_DOWNSWEEP);
  } else {
    uint32_t *k[2] = {(uint32_t *)c->sk[0].p, (uint32_t *)c->sk[1].p};
    e = launch_radix_sort_pay_u32(c, k, v, m, c->st_launch, n_dev, c->st_bits, K_SORT_UPSWEEP,
                                  K_SORT_SCAN, K_SORT_DOWNSWEEP);
  }
  if (e != hipSuccess) return e;
  c->st_sorted = out;
  ScopedTimer t(c, K_RANGES);
  uint2 *rng = (uint2 *)c->st_rng.p;   // cleared by gather_st_counts_kernel
  if (c->st_key16)
    hipLaunchKernelGGL(st_ranges_kernel<uint16_t>, dim3(ceil_div(c->st_launch, 1024)), dim3(256), 0,
                       c->stream, (const uint16_t *)c->sk[out].p, (const FrameInfo *)fi, rng);
  else
    hipLaunchKernelGGL(st_ranges_kernel<uint32_t>, dim3(ceil_div(c->st_launch, 1024)), dim3(256), 0,
                       c->stream, (const uint32_t *)c->sk[out].p, (const FrameInfo *)fi, rng);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (c->n_st + 1 <= kScanTile) {
    // the grid covers the most chunks the frame can have
    const unsigned nwg = (unsigned)ceil_div((int64_t)max_chunks(c->st_launch, c->n_st), kScanThreads);
    hipLaunchKernelGGL(chunk_plan_kernel, dim3(nwg), dim3(kScanThreads), 0, c->stream, c->cur_views,
                       c->V, (const uint2 *)rng, c->n_st, cb, fi, (ChunkRec *)c->chunk_tab.p);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(st_chunks_kernel, dim3(ceil_div(c->n_st + 1, 256)), dim3(256), 0, c->stream,
                     (const uint2 *)rng, c->n_st, cb);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = excl_scan<uint32_t>(c->stream, cb, c->n_st + 1, (uint32_t *)c->scan_tmp.p)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(chunk_total_kernel, dim3(1), dim3(1), 0, c->stream, (const uint32_t *)cb,
                     c->n_st, fi);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(chunk_table_kernel, dim3(ceil_div(c->n_st, 256)), dim3(256), 0, c->stream,
                     c->cur_views, c->V, (const uint2 *)rng, (const uint32_t *)cb, c->n_st,
                     (ChunkRec *)c->chunk_tab.p);
  return hipGetLastError();
}

// Second level: tile masks and counts per chunk, the tile scan, the tile
// ranges, and the record ids in tile order (into v0).
hipError_t launch_tile_lists(Ctx *c) {
  L2Args a;
  a.views = c->cur_views;
  a.V = c->V;
  a.per_view = c->N + c->T;
  a.N = c->N;
  a.tile_w = c->tile_w;
  a.tile_h = c->tile_h;
  a.n_st = c->n_st;
  a.n_tiles = c->n_tiles;
  a.st_rng = (const uint2 *)c->st_rng.p;
  a.chunk_base = (const uint32_t *)c->chunk_base.p;
  a.chunks = (const ChunkRec *)c->chunk_tab.p;
  a.rec = (const uint32_t *)c->sv[c->st_sorted].p;
  a.fi = (const FrameInfo *)c->finfo.p;
  a.masks = (const uint64_t *)c->masks[c->st_sorted].p;
  a.cnt = (uint32_t *)c->cnt2.p;
  a.tstart = (uint32_t *)c->tstart.p;
  a.out = (uint32_t *)c->v0.p;
  a.cap = (uint32_t)std::min<uint64_t>(c->key_cap, 0xFFFFFFFFull);
  const unsigned nchunks = (unsigned)max_chunks(c->st_launch, c->n_st);
  hipError_t e;
  {
    ScopedTimer t(c, K_TILE_COUNT);
    if (c->st_launch > 0) {
      hipLaunchKernelGGL(tile_count_kernel, dim3(nchunks), dim3(kL2Threads), 0, c->stream, a);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(tile_prefix_kernel, dim3(ceil_div(c->n_st * 64, 256)), dim3(256), 0,
                       c->stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_exclusive_scan_u32(c, a.tstart, c->n_tiles + 1,
                                 (uint32_t *)c->scan_tmp.p)) != hipSuccess)
      return e;
  }
  {
    ScopedTimer t(c, K_RANGES);
    hipLaunchKernelGGL(ranges_kernel, dim3(ceil_div(c->n_tiles, 256)), dim3(256), 0, c->stream,
                       (const uint32_t *)a.tstart, c->n_tiles, a.cap, (FrameInfo *)c->finfo.p,
                       (uint2 *)c->ranges.p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (c->st_launch == 0) return hipSuccess;
  ScopedTimer t(c, K_TILE_SCATTER);
  hipLaunchKernelGGL(tile_scatter_kernel, dim3(nchunks), dim3(kL2Threads), 0, c->stream, a);
  return hipGetLastError();
}

hipError_t launch_expand_keys(Ctx *c, uint64_t *dst) {
  if (c->n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(expand_keys_kernel, dim3((unsigned)c->n_tiles), dim3(256), 0, c->stream,
                     (const uint2 *)c->ranges.p, (const uint32_t *)c->v0.p,
                     (const uint32_t *)c->keys.p, dst);
  return hipGetLastError();
}

}  // namespace umgs
