// Stable LSD radix sort of 32- or 16-bit keys with 32-bit values (and, for
// the second use, a 64-bit payload), at most 8 bits a pass.  Two sorts use
// it: the records by depth key (values: record ids, so equal depths stay in
// id order), and the supertile entries -- emitted in that depth order -- by
// supertile id (16-bit keys while a frame has at most 2^16 supertiles;
// payload: the entry's tile mask), which leaves every supertile's entries
// ordered by (depth key, record id).
//
// Each pass is reduce-then-scan: an upsweep writes per-block digit counts in
// digit-major order, one workgroup per digit scans its row over the blocks
// and stores the digit's total (every row at once, no look-back; the
// downsweep adds the scan of the 256 totals itself), and a downsweep ranks
// every key stably inside its block (wave ballots build the
// equal-digit lane masks, per-wave running counts order the rounds), stages
// the block's keys in LDS in digit order and writes each digit's run with
// consecutive lanes on consecutive addresses.  A block covers 256 R keys:
// 4 waves x R rounds x 64 lanes, wave-major, so block order is key order.
// R (4, 8 or 16) is chosen per sort so that the grid has about a thousand
// blocks or more: a 1M-key sort in 4096-key blocks runs one block per CU,
// four waves, and waits on latency.
// Logical blocks are laid out contiguously per XCD, so the digit runs that
// neighbouring blocks write side by side are merged in the same L2.
//
// The element count may live on the device (a captured frame does not know
// it on the host), and so may the number of significant key bits: a pass
// whose shift reaches them copies its input through unchanged.
#include "internal.h"

namespace umgs {

hipError_t launch_exclusive_scan_u32(Ctx *c, uint32_t *data, int64_t n, uint32_t *tmp);
hipError_t launch_fill_u32(Ctx *c, uint32_t *p, int64_t n, uint32_t v);

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMinRounds = 4;
constexpr int kBins = 256;

struct PassArgs {
  uint32_t n_host;           // element count if n_dev is null
  const uint32_t *n_dev;     // element count on the device (clamped to n_host)
  const int32_t *bits_dev;   // significant key bits on the device, or null
  int shift;
  uint32_t mask;             // digit mask (2^bits - 1)
  uint32_t nblocks;
  // nonzero: only the blocks that hold elements run (spread over the XCDs
  // by their count on the device) and write counts, which the per-digit
  // scans read; zero: every block writes its column (the generic scan reads
  // them all)
  uint32_t spread;
};

// Logical block of this workgroup, or a value >= nblocks when it has none.
template <int R>
__device__ __forceinline__ uint32_t pass_block(const PassArgs &a, uint32_t n) {
  if (!a.spread) return xcd_block(blockIdx.x, a.nblocks);
  constexpr uint32_t kTile = kThreads * R;
  const uint32_t nb = min(a.nblocks, (n + kTile - 1) / kTile);
  const uint32_t b = xcd_block_n(blockIdx.x, nb);
  return b < nb ? b : 0xFFFFFFFFu;
}

__device__ __forceinline__ uint32_t pass_count(const PassArgs &a) {
  return a.n_dev ? min(*a.n_dev, a.n_host) : a.n_host;
}

__device__ __forceinline__ bool pass_through(const PassArgs &a) {
  return a.bits_dev && a.shift >= *a.bits_dev;
}

// Equal-digit lane mask of the wave (8 ballots over the digit's bits).
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint64_t bb = __ballot((d >> b) & 1);
    m &= ((d >> b) & 1) ? bb : ~bb;
  }
  return m;
}

// Per-block digit counts.  Order does not matter here, so each thread reads
// R consecutive keys with wide loads and counts them with LDS atomics into
// its wave's histogram (neighbouring keys -- a record's tiles -- mostly carry
// different digits, so lanes rarely collide on an address).
template <typename K, int R>
__global__ __launch_bounds__(kThreads) void rs_upsweep(const K *__restrict__ keys, PassArgs a,
                                                       uint32_t *__restrict__ hist) {
  if (pass_through(a)) return;
  constexpr int kTile = kThreads * R;
  const uint32_t n = pass_count(a);
  __shared__ uint32_t h[kWaves][kBins];
  const int tid = threadIdx.x, w = tid >> 6;
  for (int k = tid; k < kWaves * kBins; k += kThreads) (&h[0][0])[k] = 0;
  const uint32_t blk = pass_block<R>(a, n);
  if (blk >= a.nblocks) return;
  __syncthreads();
  const uint32_t i0 = blk * kTile + tid * R;
  constexpr int kBytes = R * (int)sizeof(K);   // 8 .. 64, a multiple of 8
  if (i0 + R <= n) {
    if constexpr (kBytes >= 16) {
      constexpr int kPerLoad = 16 / sizeof(K);
#pragma unroll
      for (int q = 0; q < R / kPerLoad; ++q) {
        union { uint4 v; K k[kPerLoad]; } u;
        u.v = *(const uint4 *)(keys + i0 + kPerLoad * q);
#pragma unroll
        for (int j = 0; j < kPerLoad; ++j) atomicAdd(&h[w][((uint32_t)u.k[j] >> a.shift) & a.mask], 1u);
      }
    } else {
      union { uint2 v; K k[R]; } u;
      u.v = *(const uint2 *)(keys + i0);
#pragma unroll
      for (int j = 0; j < R; ++j) atomicAdd(&h[w][((uint32_t)u.k[j] >> a.shift) & a.mask], 1u);
    }
  } else {
    for (int r = 0; r < R; ++r)
      if (i0 + r < n) atomicAdd(&h[w][((uint32_t)keys[i0 + r] >> a.shift) & a.mask], 1u);
  }
  __syncthreads();
  const uint32_t s = h[0][tid] + h[1][tid] + h[2][tid] + h[3][tid];
  hist[(uint64_t)tid * a.nblocks + blk] = s;
}

// Exclusive scan of each digit's block counts (row d of the digit-major
// counts, in place), one workgroup per digit, and the digit's total into
// totals[d].  Each thread owns kDigitItems consecutive blocks; a pass with
// more blocks than one workgroup covers takes the generic scan instead.
constexpr int kDigitItems = 16;

__global__ __launch_bounds__(kThreads) void rs_digit_scan(uint32_t *__restrict__ hist, uint32_t stride,
                                                          uint32_t *__restrict__ totals, PassArgs a,
                                                          uint32_t tile) {
  __shared__ uint32_t wsum[kWaves];
  // the blocks that hold elements (the only ones that wrote counts)
  const uint32_t nb = min(stride, (pass_count(a) + tile - 1) / tile);
  uint32_t *row = hist + (uint64_t)blockIdx.x * stride;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t i0 = (uint32_t)tid * kDigitItems;
  uint32_t v[kDigitItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kDigitItems; ++k) {
    v[k] = i0 + k < nb ? row[i0 + k] : 0u;
    s += v[k];
  }
  uint32_t x = s;   // inclusive scan over the wave, then over the waves
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t run = x - s, tot = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) {
    run += k < w ? wsum[k] : 0u;
    tot += wsum[k];
  }
#pragma unroll
  for (int k = 0; k < kDigitItems; ++k) {
    if (i0 + k < nb) row[i0 + k] = run;
    run += v[k];
  }
  if (tid == 0) totals[blockIdx.x] = tot;
}

// With P64, a 64-bit payload per element (pin/pout) moves with its key.
template <typename K, bool P64, int R>
__global__ __launch_bounds__(kThreads) void rs_downsweep(
    const K *__restrict__ kin, const uint32_t *__restrict__ vin, const uint64_t *__restrict__ pin,
    K *__restrict__ kout, uint32_t *__restrict__ vout, uint64_t *__restrict__ pout, PassArgs a,
    const uint32_t *__restrict__ offs, const uint32_t *__restrict__ totals) {
  constexpr int kRounds = R;
  constexpr int kTile = kThreads * R;
  const uint32_t n = pass_count(a);
  const uint32_t blk = pass_block<R>(a, n);
  if (blk >= a.nblocks) return;
  const uint32_t base = blk * kTile;
  if (base >= n) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (pass_through(a)) {
    const uint32_t end = min(base + (uint32_t)kTile, n);
    for (uint32_t i = base + tid; i < end; i += kThreads) {
      kout[i] = kin[i];
      vout[i] = vin[i];
      if (P64) pout[i] = pin[i];
    }
    return;
  }
  __shared__ K sk[kTile];
  __shared__ uint32_t sv[kTile];
  __shared__ uint64_t sp[P64 ? kTile : 1];
  __shared__ uint32_t wcnt[kWaves][kBins];
  __shared__ uint32_t lstart[kBins];
  __shared__ uint32_t gbase[kBins];
  __shared__ uint32_t wscan[kWaves];
  __shared__ uint32_t wscan_g[kWaves];

  for (int k = tid; k < kWaves * kBins; k += kThreads) (&wcnt[0][0])[k] = 0;
  __syncthreads();

  const uint32_t wbase = base + w * (kRounds * 64);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  K key[kRounds];
  uint32_t val[kRounds];
  uint64_t pay[P64 ? kRounds : 1];
  uint32_t rank[kRounds];   // digit | (rank within the wave) << 8
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint32_t idx = wbase + r * 64 + lane;
    const bool valid = idx < n;
    key[r] = valid ? kin[idx] : K(0);
    val[r] = valid ? vin[idx] : 0u;
    if (P64) pay[P64 ? r : 0] = valid ? pin[idx] : 0ull;
  }
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const bool valid = wbase + r * 64 + lane < n;
    const uint32_t d = ((uint32_t)key[r] >> a.shift) & a.mask;
    const uint64_t m = digit_peers(d, valid);
    const uint32_t before = (uint32_t)__popcll(m & lt);
    const uint32_t prev = wcnt[w][d];
    if (valid && before == 0) wcnt[w][d] = prev + (uint32_t)__popcll(m);
    rank[r] = d | ((prev + before) << 8);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();

  // per digit: counts over waves, exclusive prefix over waves, block scan
  // over digits; with per-digit scanned counts, the digit's first position
  // is the scan of the digits' totals (same for every block)
  {
    const int d = tid;
    const uint32_t c0 = wcnt[0][d], c1 = wcnt[1][d], c2 = wcnt[2][d], c3 = wcnt[3][d];
    const uint32_t tot = c0 + c1 + c2 + c3;
    const uint32_t gt = totals ? totals[d] : 0u;
    uint32_t x = tot, xg = gt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64), yg = __shfl_up(xg, o, 64);
      if (lane >= o) {
        x += y;
        xg += yg;
      }
    }
    if (lane == 63) {
      wscan[w] = x;
      wscan_g[w] = xg;
    }
    __syncthreads();
    uint32_t pre = 0, pre_g = 0;
    for (int k = 0; k < w; ++k) {
      pre += wscan[k];
      pre_g += wscan_g[k];
    }
    const uint32_t ls = pre + x - tot;
    lstart[d] = ls;
    gbase[d] = tot ? offs[(uint64_t)d * a.nblocks + blk] + (pre_g + xg - gt) : 0u;
    wcnt[0][d] = ls;
    wcnt[1][d] = ls + c0;
    wcnt[2][d] = ls + c0 + c1;
    wcnt[3][d] = ls + c0 + c1 + c2;
  }
  __syncthreads();

#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint32_t idx = wbase + r * 64 + lane;
    if (idx < n) {
      const uint32_t d = rank[r] & 0xFF;
      const uint32_t pos = wcnt[w][d] + (rank[r] >> 8);
      sk[pos] = key[r];
      sv[pos] = val[r];
      if (P64) sp[P64 ? pos : 0] = pay[P64 ? r : 0];
    }
  }
  __syncthreads();

  const uint32_t cnt = min((uint32_t)kTile, n - base);
  for (uint32_t i = tid; i < cnt; i += kThreads) {
    const K k = sk[i];
    const uint32_t d = ((uint32_t)k >> a.shift) & a.mask;
    const uint32_t o = gbase[d] + (i - lstart[d]);
    kout[o] = k;
    vout[o] = sv[i];
    if (P64) pout[o] = sp[P64 ? i : 0];
  }
}

}  // namespace

// Digit-major block counts (blocks of the smallest size) and the 256 digit
// totals behind them.
size_t radix_hist_bytes(uint64_t n) {
  constexpr uint64_t kSmallest = kThreads * kMinRounds;
  const uint64_t nb = (n + kSmallest - 1) / kSmallest;
  return (size_t)(nb * kBins + kBins + 16) * sizeof(uint32_t);
}

namespace {

// Rounds per thread: 16 while that still gives about a thousand blocks,
// else fewer (at least 4); with a payload at most 8 (its LDS staging
// otherwise allows two blocks per CU).
int choose_rounds(uint64_t n, bool payload) {
  int r = 16;
  while (r > kMinRounds && n < (uint64_t)1024 * kThreads * r) r >>= 1;
  if (payload && r > 8) r = 8;
  return r;
}

template <typename K, int R>
hipError_t launch_pass(Ctx *c, K *keys[2], uint32_t *vals[2], uint64_t *pay[2], int src,
                       PassArgs a, uint32_t *hist, int kid_up, int kid_scan, int kid_down) {
  const int dst = src ^ 1;
  const uint32_t nb = a.nblocks;
  a.spread = nb <= (uint32_t)(kThreads * kDigitItems) ? 1u : 0u;
  hipError_t e;
  {
    ScopedTimer t(c, kid_up);
    hipLaunchKernelGGL((rs_upsweep<K, R>), dim3(nb), dim3(kThreads), 0, c->stream,
                       (const K *)keys[src], a, hist);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  // per-digit scans when one workgroup covers a digit's blocks, else one
  // scan over all counts (global offsets; no totals)
  uint32_t *totals = nb <= (uint32_t)(kThreads * kDigitItems) ? hist + (uint64_t)nb * kBins : nullptr;
  {
    ScopedTimer t(c, kid_scan);
    if (totals) {
      hipLaunchKernelGGL(rs_digit_scan, dim3(kBins), dim3(kThreads), 0, c->stream, hist, nb, totals, a,
                         (uint32_t)(kThreads * R));
      e = hipGetLastError();
    } else {
      e = launch_exclusive_scan_u32(c, hist, (int64_t)nb * kBins, (uint32_t *)c->scan_tmp.p);
    }
  }
  if (e != hipSuccess) return e;
  ScopedTimer t(c, kid_down);
  if (pay)
    hipLaunchKernelGGL((rs_downsweep<K, true, R>), dim3(nb), dim3(kThreads), 0, c->stream,
                       (const K *)keys[src], (const uint32_t *)vals[src],
                       (const uint64_t *)pay[src], keys[dst], vals[dst], pay[dst], a,
                       (const uint32_t *)hist, (const uint32_t *)totals);
  else
    hipLaunchKernelGGL((rs_downsweep<K, false, R>), dim3(nb), dim3(kThreads), 0, c->stream,
                       (const K *)keys[src], (const uint32_t *)vals[src],
                       (const uint64_t *)nullptr, keys[dst], vals[dst], (uint64_t *)nullptr, a,
                       (const uint32_t *)hist, (const uint32_t *)totals);
  return hipGetLastError();
}

}  // namespace

int radix_passes(int bits) { return bits <= 0 ? 0 : (bits + 7) / 8; }

// Sorts keys[0]/vals[0] over `bits` key bits in radix_passes(bits) passes,
// ping-ponging with keys[1]/vals[1]; the result lies in index passes & 1.
// Grids cover n_launch elements; n_dev (if not null) holds the true count
// and bits_dev (if not null) the significant bits, both read on the device.
// The passes split the bits evenly (13 bits: 7 + 6), which keeps the digit
// runs that the downsweep writes long.
template <typename K>
hipError_t launch_radix_sort(Ctx *c, K *keys[2], uint32_t *vals[2], uint64_t *pay[2],
                             uint64_t n_launch, const uint32_t *n_dev, const int32_t *bits_dev,
                             int bits, int kid_up, int kid_scan, int kid_down) {
  if (n_launch == 0 || bits <= 0) return hipSuccess;
  const uint32_t n = (uint32_t)n_launch;
  const int rounds = choose_rounds(n, pay != nullptr);
  const uint32_t nb = (n + kThreads * rounds - 1) / (kThreads * rounds);
  const int passes = radix_passes(bits);
  uint32_t *hist = (uint32_t *)c->hist.p;
  int shift = 0;
  for (int p = 0; p < passes; ++p) {
    const int pb = bits / passes + (p < bits % passes ? 1 : 0);
    PassArgs a;
    a.n_host = n;
    a.n_dev = n_dev;
    a.bits_dev = bits_dev;
    a.shift = shift;
    a.mask = (1u << pb) - 1u;
    a.nblocks = nb;
    const int src = p & 1;
    hipError_t e;
    if (rounds == 16)
      e = launch_pass<K, 16>(c, keys, vals, pay, src, a, hist, kid_up, kid_scan, kid_down);
    else if (rounds == 8)
      e = launch_pass<K, 8>(c, keys, vals, pay, src, a, hist, kid_up, kid_scan, kid_down);
    else
      e = launch_pass<K, 4>(c, keys, vals, pay, src, a, hist, kid_up, kid_scan, kid_down);
    if (e != hipSuccess) return e;
    shift += pb;
  }
  return hipSuccess;
}

hipError_t launch_radix_sort_u32(Ctx *c, uint32_t *keys[2], uint32_t *vals[2], uint64_t n_launch,
                                 const uint32_t *n_dev, const int32_t *bits_dev, int bits,
                                 int kid_up, int kid_scan, int kid_down) {
  return launch_radix_sort<uint32_t>(c, keys, vals, nullptr, n_launch, n_dev, bits_dev, bits,
                                     kid_up, kid_scan, kid_down);
}

hipError_t launch_radix_sort_pay_u32(Ctx *c, uint32_t *keys[2], uint32_t *vals[2],
                                     uint64_t *pay[2], uint64_t n_launch, const uint32_t *n_dev,
                                     int bits, int kid_up, int kid_scan, int kid_down) {
  return launch_radix_sort<uint32_t>(c, keys, vals, pay, n_launch, n_dev, nullptr, bits, kid_up,
                                     kid_scan, kid_down);
}

hipError_t launch_radix_sort_pay_u16(Ctx *c, uint16_t *keys[2], uint32_t *vals[2],
                                     uint64_t *pay[2], uint64_t n_launch, const uint32_t *n_dev,
                                     int bits, int kid_up, int kid_scan, int kid_down) {
  return launch_radix_sort<uint16_t>(c, keys, vals, pay, n_launch, n_dev, nullptr, bits, kid_up,
                                     kid_scan, kid_down);
}

}  // namespace umgs
