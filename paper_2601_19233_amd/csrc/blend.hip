// Forward blend: one workgroup per screen tile, one thread per pixel.
//
// The tile's sorted fragments are staged in LDS in batches (one 128-B slot
// per fragment; every pixel then reads the same slot, a broadcast).  Each
// pixel walks the batch front to back:
//   Gaussian (Eq. 1-2): alpha = min(0.99, o exp(power)); skipped below
//     1/255; if T (1 - alpha) < 1e-4 the pixel stops before blending it.
//   Triangle (Eq. 7-9): sub-sample coverage o^j of the 4 rotated-grid samples
//     from exact integer edge functions; consecutive triangles form an entity
//     with entry transmittance T_in and sub-sample transmittances t^j;
//     C += T_in O alpha c with O = mean_j o^j t^j; t^j *= 1 - o^j alpha;
//     T = T_in mean_j t^j; stop after blending once T < 1e-4.
// The background is composited with the final T (Eq. 10-11, opaque
// background).  A wave skips the rest of a batch once all its pixels are
// done; the workgroup stops loading batches once every pixel is done.
//
// Two schedules: one workgroup per tile, or a persistent grid (a few
// workgroups per CU) taking tiles in an order by list length, longest
// first, strided over the grid, which evens out views and tiles of very
// different cost.
//
// Edge functions E = dx (Py - Ya) - dy (Px - Xa) are integers in 1/256-px
// units below 2^52 in magnitude; they are evaluated in FP64, which holds
// them exactly (CDNA executes FP64 FMA at full vector rate).
#include "blend_common.h"

namespace umgs {

namespace {

// First set bit at or after slot f among the first bn slots of the batch's
// triangle mask (bn if none).
__device__ __forceinline__ uint32_t next_set_slot(const uint64_t *m, uint32_t f, uint32_t bn) {
  while (f < bn) {
    const uint64_t w = m[f >> 6] >> (f & 63u);
    if (w) return min(bn, f + (uint32_t)__builtin_ctzll(w));
    f = (f | 63u) + 1u;
  }
  return bn;
}

// COUNT instantiations also count into pairs[0..3]: the (pixel, fragment)
// pairs each pixel evaluates before it is done (Gaussian, triangle), the
// wave iterations of the fragment loop (times 64 lanes: the SIMD slots the
// pairs occupy) and the fragments staged into LDS.
template <int TW, int TH, bool COUNT = false>
__device__ __forceinline__ void blend_tile(
    uint32_t tile, uint32_t *__restrict__ slots, const ViewParams *__restrict__ views, int V,
    int N, int T, int mode, int batch, float bg0, float bg1, float bg2,
    const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
    const GaussRec *__restrict__ grec, const TriRec *__restrict__ trec, const TexView tex,
    float *__restrict__ image, float *__restrict__ Tout, int32_t *__restrict__ ncontrib,
    float *__restrict__ Tent_out, unsigned long long *__restrict__ pairs = nullptr) {
  uint32_t n_gp = 0, n_tp = 0, n_wit = 0;
  constexpr int NT = TW * TH;
  const int v = find_view(views, V, tile);
  const ViewParams &vp = views[v];
  const uint32_t lt = tile - vp.tile_base;
  const int tx = (int)(lt % (uint32_t)vp.ntx), ty = (int)(lt / (uint32_t)vp.ntx);
  const int tid = threadIdx.x;
  const int lx = tid % TW, ly = tid / TW;
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool inside = px < vp.W && py < vp.H;
  const float pcx = (float)px + 0.5f, pcy = (float)py + 0.5f;
  // tile's first pixel centre in 1/256 px
  const int64_t P0x = (int64_t)(tx * TW) * kSubpx + kSubpx / 2;
  const int64_t P0y = (int64_t)(ty * TH) * kSubpx + kSubpx / 2;
  const double rlx = (double)(lx * kSubpx), rly = (double)(ly * kSubpx);
  const bool direct = mode == UMGS_MODE_DIRECT;

  // The tile's range (and below, each run's end) is the same on every lane;
  // taken with readfirstlane, it stays in scalar registers.
  uint2 rg = ranges[tile];
  rg.x = (uint32_t)__builtin_amdgcn_readfirstlane((int)rg.x);
  rg.y = (uint32_t)__builtin_amdgcn_readfirstlane((int)rg.y);
  const int64_t rbase = (int64_t)v * (N + T);

  float C0 = 0.f, C1 = 0.f, C2 = 0.f;
  float Tr = 1.0f, Tin = 1.0f, Tent = 1.0f;
  float t0 = 1.f, t1 = 1.f, t2 = 1.f, t3 = 1.f;
  bool in_entity = false;
  bool done = !inside;
  int32_t last = 0;

  // triangle slots of the staged batch, one bit per slot (batch <= 256)
  __shared__ uint64_t tmask[4];

  for (uint32_t bstart = rg.x; bstart < rg.y; bstart += batch) {
    const uint32_t bn = min((uint32_t)batch, rg.y - bstart);
    if (COUNT && tid == 0) atomicAdd(pairs + 3, (unsigned long long)bn);
    // ---- stage fragments into LDS; each wave records which of its slots
    // hold triangles
    for (uint32_t j0 = 0; j0 < bn; j0 += NT) {
      const uint32_t f = j0 + tid;
      bool is_tri = false;
      if (f < bn) {
        uint32_t *s = slots + f * kSlotWords;
        const int64_t local = (int64_t)vals[bstart + f] - rbase;
        if (local < N) {
          const uint32_t rec = (uint32_t)((int64_t)v * N + local);
          stage_gauss(s, grec[rec], rec);
        } else {
          const TriRec &tr = trec[(int64_t)v * T + (local - N)];
          stage_tri(s, tr, P0x, P0y);
          s[38] = tri_tile_box(tr, tx * TW, ty * TH, TW, TH);
          is_tri = true;
        }
      }
      const uint64_t bits = __ballot(is_tri);
      const uint32_t w0 = j0 + ((uint32_t)tid & ~63u);
      if ((tid & 63) == 0 && w0 < bn) tmask[w0 >> 6] = bits;
    }
    __syncthreads();
    uint64_t any_bits = 0;
    for (uint32_t w = 0; w * 64 < bn; ++w) any_bits |= tmask[w];
    const bool any_tri = any_bits != 0;

    // ---- blend the batch: runs of Gaussians between the triangles (the
    // whole wave walks while one of its pixels is live; a done pixel starts
    // every run with T = 0, where each fragment is a stop and adds nothing,
    // and skips the triangles)
    if (!__all(done)) {
      uint32_t f = 0;
      while (f < bn) {
        const uint32_t fe = (uint32_t)__builtin_amdgcn_readfirstlane(
            (int)(any_tri ? next_set_slot(tmask, f, bn) : bn));
        if (fe > f) {
          // Gaussians [f, fe): alpha of kUnroll fragments evaluated together
          // (they do not depend on the pixel's state), then blended in list
          // order.  Every decision is a per-lane select: a fragment that
          // does not contribute gets alpha 0.  A stop is a fragment whose
          // T (1 - alpha) would fall below 1e-4; Tf keeps the pixel's final
          // T, while Tl, the running product, goes on falling below 1e-4,
          // so every later fragment is a stop too and adds nothing (a live
          // pixel always has T >= 1e-4).
          constexpr int kUnroll = 8;
          float Tl = done ? 0.0f : Tr, Tf = Tr;   // a pixel stopped in an earlier run stays stopped
          const int32_t last0 = last;
          for (; f + kUnroll <= fe; f += kUnroll) {
            if (__all(Tl < kTStop)) break;
            if (COUNT) n_wit += kUnroll;
            float al[kUnroll], cr[kUnroll], cg[kUnroll], cb[kUnroll];
            bool ok[kUnroll];
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
              const uint32_t *s = slots + (f + k) * kSlotWords;
              float a;
              ok[k] = gauss_alpha(s, pcx, pcy, a);
              al[k] = ok[k] ? a : 0.0f;
              cr[k] = __uint_as_float(s[6]);
              cg[k] = __uint_as_float(s[7]);
              cb[k] = __uint_as_float(s[8]);
            }
            // last blended slot of the group, 1-based (0: none): a select of
            // a constant per fragment; the list position is added once per
            // group
            int32_t lastk = 0;
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
              if (COUNT) n_gp += Tl < kTStop ? 0u : 1u;
              const float w = Tl * al[k];
              const float test_T = Tl - w;      // T (1 - alpha)
              const bool stop = test_T < kTStop;
              const bool blend = !stop && ok[k];
              const float wc = stop ? 0.0f : w;
              C0 = fmaf(wc, cr[k], C0);
              C1 = fmaf(wc, cg[k], C1);
              C2 = fmaf(wc, cb[k], C2);
              Tent = blend ? Tl : Tent;
              lastk = blend ? k + 1 : lastk;
              Tf = stop ? Tf : test_T;
              Tl = test_T;
            }
            last = lastk != 0 ? (int32_t)(bstart - rg.x + f) + lastk : last;
          }
          // the rest of the run one at a time, same arithmetic
          for (; f < fe; ++f) {
            if (__all(Tl < kTStop)) break;
            if (COUNT) ++n_wit;
            if (COUNT) n_gp += Tl < kTStop ? 0u : 1u;
            const uint32_t *s = slots + f * kSlotWords;
            float a;
            const bool ok = gauss_alpha(s, pcx, pcy, a);
            const float w = Tl * (ok ? a : 0.0f);
            const float test_T = Tl - w;
            const bool stop = test_T < kTStop;
            const bool blend = !stop && ok;
            const float wc = stop ? 0.0f : w;
            C0 = fmaf(wc, __uint_as_float(s[6]), C0);
            C1 = fmaf(wc, __uint_as_float(s[7]), C1);
            C2 = fmaf(wc, __uint_as_float(s[8]), C2);
            Tent = blend ? Tl : Tent;
            last = blend ? (int32_t)(bstart - rg.x + f + 1) : last;
            Tf = stop ? Tf : test_T;
            Tl = test_T;
          }
          Tr = Tf;
          done = Tl < kTStop;
          // a blended Gaussian ends the run of consecutive triangles
          if (mode != UMGS_MODE_ONE_ENTITY && last != last0) in_entity = false;
          if (__all(done)) break;
          f = fe;
        }
        if (f < bn) {
          // the triangle at slot f
          if (COUNT) ++n_wit;
          if (!done) {
            if (COUNT) ++n_tp;
            const uint32_t *s = slots + f * kSlotWords;
            const int32_t pos = (int32_t)(bstart - rg.x + f + 1);
            double e[3];
            float o[4];
            if (in_tile_box(s[38], lx, ly) && tri_eval(s, rlx, rly, direct, e, o) != 0) {
              float cr, cg, cbl, alpha;
              tri_shade(s, e, tex, cr, cg, cbl, alpha);
              if (direct) {
                const float w = Tr * alpha;
                C0 = fmaf(w, cr, C0); C1 = fmaf(w, cg, C1); C2 = fmaf(w, cbl, C2);
                Tent = Tr;
                Tr = Tr - w;
                last = pos;
                if (Tr < kTStop) done = true;
              } else {
                if (!in_entity) {
                  Tin = Tr;
                  Tent = Tr;
                  t0 = t1 = t2 = t3 = 1.0f;
                  in_entity = true;
                }
                const float O = 0.25f * (o[0] * t0 + o[1] * t1 + o[2] * t2 + o[3] * t3);
                const float w = Tin * O * alpha;
                C0 = fmaf(w, cr, C0); C1 = fmaf(w, cg, C1); C2 = fmaf(w, cbl, C2);
                if (mode == UMGS_MODE_LITERAL_T) Tr = Tr * (1.0f - O * alpha);
                t0 *= 1.0f - o[0] * alpha;
                t1 *= 1.0f - o[1] * alpha;
                t2 *= 1.0f - o[2] * alpha;
                t3 *= 1.0f - o[3] * alpha;
                if (mode != UMGS_MODE_LITERAL_T) Tr = Tin * (0.25f * ((t0 + t1) + (t2 + t3)));
                last = pos;
                if (Tr < kTStop) done = true;
              }
            }
          }
          ++f;
          if (__all(done)) break;
        }
      }
    }
    if (__syncthreads_count(done ? 1 : 0) == NT) break;
  }

  if (inside) {
    const int64_t HW = (int64_t)vp.W * vp.H;
    const int64_t pix = (int64_t)py * vp.W + px;
    float *img = image + 3 * vp.pix_base;
    img[pix] = C0 + Tr * bg0;
    img[HW + pix] = C1 + Tr * bg1;
    img[2 * HW + pix] = C2 + Tr * bg2;
    if (Tout) Tout[vp.pix_base + pix] = Tr;
    if (ncontrib) ncontrib[vp.pix_base + pix] = last;
    if (Tent_out) Tent_out[vp.pix_base + pix] = Tent;
  }
  if (COUNT) {
    unsigned long long g = n_gp, t = n_tp;
    for (int o = 32; o >= 1; o >>= 1) {
      g += __shfl_xor(g, o, 64);
      t += __shfl_xor(t, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(pairs, g);
      atomicAdd(pairs + 1, t);
      atomicAdd(pairs + 2, (unsigned long long)n_wit);
    }
  }
}

struct BlendArgs {
  const ViewParams *views;
  int V, N, T, mode, batch;
  float bg0, bg1, bg2;
  const uint2 *ranges;
  const uint32_t *v0, *v1;
  const GaussRec *grec;
  const TriRec *trec;
  TexView tex;
  FrameInfo *fi;
  const uint32_t *order;
  uint32_t n_tiles;
  float *image, *Tout;
  int32_t *ncontrib;
  float *Tent;
};

// Six waves per SIMD (at most 80 VGPRs, no spills): while one workgroup
// waits for its batch's records at the staging barrier, others blend.
constexpr int kBlendWaves = 6;

template <int TW, int TH>
__global__ __launch_bounds__(TW *TH) __attribute__((amdgpu_waves_per_eu(kBlendWaves, kBlendWaves))) void blend_kernel(BlendArgs a) {
  extern __shared__ uint32_t slots[];   // batch * kSlotWords
  const uint32_t *vals = a.fi->sorted_in ? a.v1 : a.v0;
  blend_tile<TW, TH>(blockIdx.x, slots, a.views, a.V, a.N, a.T, a.mode, a.batch, a.bg0, a.bg1,
                     a.bg2, a.ranges, vals, a.grec, a.trec, a.tex, a.image, a.Tout, a.ncontrib, a.Tent);
}

template <int TW, int TH>
__global__ __launch_bounds__(TW *TH) __attribute__((amdgpu_waves_per_eu(kBlendWaves, kBlendWaves))) void blend_count_kernel(BlendArgs a,
                                                             unsigned long long *pairs) {
  extern __shared__ uint32_t slots[];
  const uint32_t *vals = a.fi->sorted_in ? a.v1 : a.v0;
  blend_tile<TW, TH, true>(blockIdx.x, slots, a.views, a.V, a.N, a.T, a.mode, a.batch, a.bg0,
                           a.bg1, a.bg2, a.ranges, vals, a.grec, a.trec, a.tex, a.image, a.Tout,
                           a.ncontrib, a.Tent, pairs);
}

// Persistent schedule: workgroup g of G takes items g, g + G, g + 2G, ...
// of the longest-first order, so every workgroup gets one tile from each
// band of G and the longest lists start first.  (Taking the next item from
// an atomic counter made every tile wait on one address: atomics to one
// address serialise at the memory side, 1.6 ms for 8160 tiles.)
template <int TW, int TH>
__global__ __launch_bounds__(TW *TH) __attribute__((amdgpu_waves_per_eu(kBlendWaves, kBlendWaves))) void blend_persistent_kernel(BlendArgs a) {
  extern __shared__ uint32_t slots[];
  const uint32_t *vals = a.fi->sorted_in ? a.v1 : a.v0;
  for (uint32_t it = blockIdx.x; it < a.n_tiles; it += gridDim.x)
    blend_tile<TW, TH>(a.order[it], slots, a.views, a.V, a.N, a.T, a.mode, a.batch, a.bg0, a.bg1,
                       a.bg2, a.ranges, vals, a.grec, a.trec, a.tex, a.image, a.Tout, a.ncontrib, a.Tent);
}

// ---- longest-first tile order: bucket tiles by floor(log2(list length)) ----
constexpr int kBuckets = 34;

__device__ __forceinline__ int length_bucket(uint2 r) {
  const uint32_t len = r.y - r.x;
  return len == 0 ? 0 : 33 - __clz(len);      // 1..33, larger = longer
}

__global__ void order_count_kernel(const uint2 *__restrict__ ranges, uint32_t n,
                                   uint32_t *__restrict__ cnt) {
  __shared__ uint32_t h[kBuckets];
  if (threadIdx.x < kBuckets) h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) atomicAdd(&h[length_bucket(ranges[t])], 1u);
  __syncthreads();
  if (threadIdx.x < kBuckets && h[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], h[threadIdx.x]);
}

// cursors: descending bucket order, longest lists first
__global__ void order_scan_kernel(uint32_t *__restrict__ cnt) {
  if (threadIdx.x != 0) return;
  uint32_t run = 0;
  for (int b = kBuckets - 1; b >= 0; --b) {
    const uint32_t c = cnt[b];
    cnt[b] = run;
    run += c;
  }
}

__global__ void order_scatter_kernel(const uint2 *__restrict__ ranges, uint32_t n,
                                     uint32_t *__restrict__ cursor, uint32_t *__restrict__ order) {
  __shared__ uint32_t h[kBuckets], base[kBuckets];
  if (threadIdx.x < kBuckets) h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  int b = 0;
  uint32_t local = 0;
  if (t < n) {
    b = length_bucket(ranges[t]);
    local = atomicAdd(&h[b], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kBuckets && h[threadIdx.x]) base[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], h[threadIdx.x]);
  __syncthreads();
  if (t < n) order[base[b] + local] = t;
}

template <int TW, int TH>
hipError_t launch_tw(Ctx *c, BlendArgs a, bool persistent, unsigned long long *pairs) {
  const size_t lds = (size_t)c->frag_batch * kSlotWords * sizeof(uint32_t);
  if (pairs) {
    hipLaunchKernelGGL((blend_count_kernel<TW, TH>), dim3((unsigned)c->n_tiles), dim3(TW * TH),
                       lds, c->stream, a, pairs);
    return hipGetLastError();
  }
  ScopedTimer t(c, K_BLEND);
  if (persistent) {
    // enough workgroups to fill every CU (LDS and registers allow several per
    // CU); workgroups beyond the tile count exit at once
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, blend_persistent_kernel<TW, TH>,
                                                     TW * TH, lds) != hipSuccess || per_cu < 8)
      per_cu = 8;
    const uint64_t grid = std::min<uint64_t>((uint64_t)c->num_cu * per_cu, (uint64_t)c->n_tiles);
    hipLaunchKernelGGL((blend_persistent_kernel<TW, TH>), dim3((unsigned)grid), dim3(TW * TH), lds,
                       c->stream, a);
  } else {
    hipLaunchKernelGGL((blend_kernel<TW, TH>), dim3((unsigned)c->n_tiles), dim3(TW * TH), lds,
                       c->stream, a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fill_u32(Ctx *c, uint32_t *p, int64_t n, uint32_t v);

hipError_t launch_blend(Ctx *c, float *image, float *T_final, int32_t *n_contrib,
                        float *T_entity_in, unsigned long long *pairs) {
  if (c->n_tiles == 0) return hipSuccess;
  const bool persistent = !pairs && c->opt.schedule == UMGS_SCHEDULE_PERSISTENT;
  uint32_t *cnt = (uint32_t *)c->tile_order.p;
  uint32_t *order = cnt + 64;
  if (persistent) {
    hipError_t e = launch_fill_u32(c, cnt, kBuckets, 0u);
    if (e != hipSuccess) return e;
    const unsigned g = ceil_div(c->n_tiles, 256);
    hipLaunchKernelGGL(order_count_kernel, dim3(g), dim3(256), 0, c->stream,
                       (const uint2 *)c->ranges.p, (uint32_t)c->n_tiles, cnt);
    hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(64), 0, c->stream, cnt);
    hipLaunchKernelGGL(order_scatter_kernel, dim3(g), dim3(256), 0, c->stream,
                       (const uint2 *)c->ranges.p, (uint32_t)c->n_tiles, cnt, order);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  BlendArgs a;
  a.views = c->cur_views;
  a.V = c->V; a.N = c->N; a.T = c->T; a.mode = c->mode; a.batch = c->frag_batch;
  a.bg0 = c->bg[0]; a.bg1 = c->bg[1]; a.bg2 = c->bg[2];
  a.ranges = (const uint2 *)c->ranges.p;
  a.v0 = (const uint32_t *)c->v0.p;
  a.v1 = (const uint32_t *)c->v1.p;
  a.grec = (const GaussRec *)c->grec.p;
  a.trec = (const TriRec *)c->trec.p;
  a.tex = frame_texture(c);
  a.fi = (FrameInfo *)c->finfo.p;
  a.order = order;
  a.n_tiles = (uint32_t)c->n_tiles;
  a.image = image; a.Tout = T_final; a.ncontrib = n_contrib; a.Tent = T_entity_in;
  if (c->tile_w == 16 && c->tile_h == 16) return launch_tw<16, 16>(c, a, persistent, pairs);
  if (c->tile_w == 8 && c->tile_h == 8) return launch_tw<8, 8>(c, a, persistent, pairs);
  if (c->tile_w == 32 && c->tile_h == 8) return launch_tw<32, 8>(c, a, persistent, pairs);
  return hipErrorInvalidValue;
}

}  // namespace umgs
