// Stable LSD radix sort of 64-bit (tile << 32 | depth) keys with 32-bit
// values, 8-bit digits, over the significant bits only (32 depth bits plus
// the bits of the largest global tile id).
//
// Each pass is reduce-then-scan: an upsweep writes per-block digit counts in
// digit-major order, an exclusive scan turns them into global offsets, and a
// downsweep ranks every key stably inside its block (wave ballots build the
// equal-digit lane masks, per-wave running counts order the rounds), stages
// the block's keys in LDS in digit order and writes each digit's run with
// consecutive lanes on consecutive addresses.  A block covers 4096 keys:
// 4 waves x 16 rounds x 64 lanes, wave-major, so block order is key order.
// Logical blocks are laid out contiguously per XCD, so the digit runs that
// neighbouring blocks write side by side are merged in the same L2.
#include "internal.h"

namespace umgs {

hipError_t launch_exclusive_scan_u32(Ctx *c, uint32_t *data, int64_t n, uint32_t *tmp);

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kRounds = 16;
constexpr int kTile = kThreads * kRounds;   // 4096
constexpr int kBins = 256;

__global__ __launch_bounds__(kThreads) void rs_upsweep(const uint64_t *__restrict__ keys,
                                                       const FrameInfo *__restrict__ fi, int shift,
                                                       uint32_t *__restrict__ hist,
                                                       uint32_t nblocks) {
  if (shift >= fi->total_bits) return;     // pass beyond the significant bits
  const uint32_t n = fi->n_dup;
  __shared__ uint32_t h[kWaves][kBins];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int k = tid; k < kWaves * kBins; k += kThreads) (&h[0][0])[k] = 0;
  __syncthreads();
  const uint32_t blk = xcd_block(blockIdx.x, nblocks);
  const uint32_t wbase = blk * kTile + w * (kRounds * 64);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint64_t key[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint32_t idx = wbase + r * 64 + lane;
    key[r] = idx < n ? keys[idx] : 0ull;
  }
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    // one LDS add per distinct digit of the wave: the lowest lane of each
    // equal-digit lane set adds the set's size
    const bool valid = wbase + r * 64 + lane < n;
    const uint32_t d = (uint32_t)(key[r] >> shift) & 0xFF;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bb = __ballot((d >> b) & 1);
      m &= ((d >> b) & 1) ? bb : ~bb;
    }
    if (valid && (m & lt) == 0) h[w][d] += (uint32_t)__popcll(m);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  const uint32_t s = h[0][tid] + h[1][tid] + h[2][tid] + h[3][tid];
  hist[(uint64_t)tid * nblocks + blk] = s;
}

__global__ __launch_bounds__(kThreads) void rs_downsweep(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, const FrameInfo *__restrict__ fi,
    int shift, const uint32_t *__restrict__ offs, uint32_t nblocks) {
  if (shift >= fi->total_bits) return;
  const uint32_t n = fi->n_dup;
  const uint32_t blk = xcd_block(blockIdx.x, nblocks);
  if (blk * (uint32_t)kTile >= n) return;
  __shared__ uint64_t sk[kTile];
  __shared__ uint32_t sv[kTile];
  __shared__ uint32_t wcnt[kWaves][kBins];
  __shared__ uint32_t lstart[kBins];
  __shared__ uint32_t gbase[kBins];
  __shared__ uint32_t wscan[kWaves];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int k = tid; k < kWaves * kBins; k += kThreads) (&wcnt[0][0])[k] = 0;
  __syncthreads();

  const uint32_t base = blk * kTile;
  const uint32_t wbase = base + w * (kRounds * 64);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint64_t key[kRounds];
  uint32_t val[kRounds];
  uint32_t rank[kRounds];   // digit | (rank within the wave) << 8
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint32_t idx = wbase + r * 64 + lane;
    const bool valid = idx < n;
    key[r] = valid ? kin[idx] : 0ull;
    val[r] = valid ? vin[idx] : 0u;
    const uint32_t d = (uint32_t)(key[r] >> shift) & 0xFF;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bb = __ballot((d >> b) & 1);
      m &= ((d >> b) & 1) ? bb : ~bb;
    }
    const uint32_t before = (uint32_t)__popcll(m & lt);
    const uint32_t prev = wcnt[w][d];
    if (valid && before == 0) wcnt[w][d] = prev + (uint32_t)__popcll(m);
    rank[r] = d | ((prev + before) << 8);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();

  // per digit: counts over waves, exclusive prefix over waves, block scan over digits
  {
    const int d = tid;
    uint32_t c0 = wcnt[0][d], c1 = wcnt[1][d], c2 = wcnt[2][d], c3 = wcnt[3][d];
    const uint32_t tot = c0 + c1 + c2 + c3;
    // inclusive scan of tot over the 256 digits
    uint32_t x = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wscan[w] = x;
    __syncthreads();
    uint32_t pre = 0;
    for (int k = 0; k < w; ++k) pre += wscan[k];
    const uint32_t ls = pre + x - tot;
    lstart[d] = ls;
    gbase[d] = offs[(uint64_t)d * nblocks + blk];
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
    }
  }
  __syncthreads();

  const uint32_t cnt = min((uint32_t)kTile, n - base);
  for (uint32_t i = tid; i < cnt; i += kThreads) {
    const uint64_t k = sk[i];
    const uint32_t d = (uint32_t)(k >> shift) & 0xFF;
    const uint32_t o = gbase[d] + (i - lstart[d]);
    kout[o] = k;
    vout[o] = sv[i];
  }
}

}  // namespace

size_t radix_hist_bytes(uint64_t n) {
  const uint64_t nb = (n + kTile - 1) / kTile;
  return (size_t)(nb * kBins + 16) * sizeof(uint32_t);
}

// Launches c->sort_passes passes over c->n_launch elements; the kernels read
// the frame's true size and significant bits from the device, so passes
// beyond them (launched when the host does not know the frame's sizes, as
// in a captured graph) return immediately.
hipError_t launch_radix_sort(Ctx *c) {
  const uint64_t n64 = c->n_launch;
  if (n64 == 0) return hipSuccess;
  const uint32_t n = (uint32_t)n64;
  const uint32_t nb = (n + kTile - 1) / kTile;
  const int passes = c->sort_passes;
  const FrameInfo *fi = (const FrameInfo *)c->finfo.p;
  uint64_t *ka = (uint64_t *)c->k0.p, *kb = (uint64_t *)c->k1.p;
  uint32_t *va = (uint32_t *)c->v0.p, *vb = (uint32_t *)c->v1.p;
  uint32_t *hist = (uint32_t *)c->hist.p;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    hipError_t e;
    {
      ScopedTimer t(c, K_SORT_UPSWEEP);
      hipLaunchKernelGGL(rs_upsweep, dim3(nb), dim3(kThreads), 0, c->stream,
                         (const uint64_t *)ka, fi, shift, hist, nb);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    e = launch_exclusive_scan_u32(c, hist, (int64_t)nb * kBins, (uint32_t *)c->scan_tmp.p);
    if (e != hipSuccess) return e;
    {
      ScopedTimer t(c, K_SORT_DOWNSWEEP);
      hipLaunchKernelGGL(rs_downsweep, dim3(nb), dim3(kThreads), 0, c->stream,
                         (const uint64_t *)ka, (const uint32_t *)va, kb, vb, fi, shift,
                         (const uint32_t *)hist, nb);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    uint64_t *tk = ka; ka = kb; kb = tk;
    uint32_t *tv = va; va = vb; vb = tv;
  }
  return hipSuccess;
}

}  // namespace umgs
