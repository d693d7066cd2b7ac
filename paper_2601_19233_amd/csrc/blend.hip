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
// Edge functions E = dx (Py - Ya) - dy (Px - Xa) are integers in 1/256-px
// units below 2^52 in magnitude; they are evaluated in FP64, which holds
// them exactly (CDNA executes FP64 FMA at full vector rate).
#include "internal.h"

namespace umgs {

namespace {

constexpr int kSlotWords = 32;   // 128 B per staged fragment

// rotated-grid sample offsets from the pixel centre, 1/256 px
__constant__ int kSampleOX[4] = {-32, 96, -96, 32};
__constant__ int kSampleOY[4] = {-96, -32, 32, 96};

__device__ __forceinline__ int find_view(const ViewParams *views, int V, uint32_t tile) {
  int lo = 0, hi = V - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int TW, int TH>
__global__ __launch_bounds__(TW *TH) void blend_kernel(
    const ViewParams *__restrict__ views, int V, int N, int T, int mode, int batch,
    float bg0, float bg1, float bg2, const uint2 *__restrict__ ranges,
    const uint32_t *__restrict__ vals, const GaussRec *__restrict__ grec,
    const TriRec *__restrict__ trec, float *__restrict__ image, float *__restrict__ Tout,
    int32_t *__restrict__ ncontrib, float *__restrict__ Tent_out) {
  constexpr int NT = TW * TH;
  extern __shared__ uint32_t slots[];   // batch * kSlotWords

  const uint32_t tile = blockIdx.x;
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

  const uint2 rg = ranges[tile];
  const int per_view = N + T;
  const int64_t rbase = (int64_t)v * per_view;

  float C0 = 0.f, C1 = 0.f, C2 = 0.f;
  float Tr = 1.0f, Tin = 1.0f, Tent = 1.0f;
  float t0 = 1.f, t1 = 1.f, t2 = 1.f, t3 = 1.f;
  bool in_entity = false;
  bool done = !inside;
  int32_t last = 0;

  for (uint32_t bstart = rg.x; bstart < rg.y; bstart += batch) {
    const uint32_t bn = min((uint32_t)batch, rg.y - bstart);
    // ---- stage fragments into LDS
    for (uint32_t f = tid; f < bn; f += NT) {
      uint32_t *s = slots + f * kSlotWords;
      const int64_t local = (int64_t)vals[bstart + f] - rbase;
      if (local < N) {
        const GaussRec g = grec[(int64_t)v * N + local];
        const float4 a = make_float4(g.mx, g.my, g.qa, g.qb);
        const float4 b = make_float4(g.qc, g.opacity, g.r, g.g);
        *(float4 *)(s + 0) = a;
        *(float4 *)(s + 4) = b;
        s[8] = __float_as_uint(g.b);
        s[31] = 0u;
      } else {
        const TriRec tr = trec[(int64_t)v * T + (local - N)];
        const int ea[3] = {1, 2, 0}, eb[3] = {2, 0, 1};
        double *dv = (double *)s;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int64_t dx = (int64_t)tr.X[eb[k]] - tr.X[ea[k]];
          const int64_t dy = (int64_t)tr.Y[eb[k]] - tr.Y[ea[k]];
          const int64_t E0 = dx * (P0y - tr.Y[ea[k]]) - dy * (P0x - tr.X[ea[k]]);
          dv[k] = (double)E0;
          dv[3 + k] = 96.0 * (double)((dx < 0 ? -dx : dx) + (dy < 0 ? -dy : dy));
          s[12 + k] = (uint32_t)(int32_t)dx;
          s[15 + k] = (uint32_t)(int32_t)dy;
          s[18 + k] = __float_as_uint(tr.iz[k]);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) s[21 + k] = __float_as_uint(tr.ciz[k]);
        s[30] = __float_as_uint(tr.alpha);
        s[31] = 1u | (tr.owned << 8);
      }
    }
    __syncthreads();

    // ---- blend the batch
    if (!done) {
      for (uint32_t f = 0; f < bn; ++f) {
        if (__all(done)) break;
        const uint32_t *s = slots + f * kSlotWords;
        const uint32_t tag = s[31];
        if (done) continue;
        if ((tag & 1u) == 0u) {
          const float4 a = *(const float4 *)(s + 0);
          const float4 b = *(const float4 *)(s + 4);
          const float dx = a.x - pcx, dy = a.y - pcy;
          const float power = a.z * dx * dx + a.w * dx * dy + b.x * dy * dy;
          if (power > 0.0f) continue;
          const float alpha = fminf(kAlphaMax, b.y * __expf(power));
          if (alpha < kAlphaMin) continue;
          const float test_T = Tr * (1.0f - alpha);
          if (test_T < kTStop) { done = true; continue; }
          const float w = Tr * alpha;
          C0 += w * b.z;
          C1 += w * b.w;
          C2 += w * __uint_as_float(s[8]);
          Tent = Tr;
          Tr = test_T;
          if (mode != UMGS_MODE_ONE_ENTITY) in_entity = false;
          last = (int32_t)(bstart - rg.x + f + 1);
        } else {
          const double *dv = (const double *)s;
          const uint32_t owned = tag >> 8;
          double e[3];
          bool any = true;
          bool full = true;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const double dxk = (double)(int32_t)s[12 + k];
            const double dyk = (double)(int32_t)s[15 + k];
            e[k] = fma(dxk, rly, fma(-dyk, rlx, dv[k]));
            const double own = (double)((owned >> k) & 1u);
            any = any && (e[k] + dv[3 + k] + own > 0.0);
            full = full && (e[k] - dv[3 + k] > 0.0);
          }
          if (!any) continue;
          float o[4];
          if (mode == UMGS_MODE_DIRECT) {
            bool c = true;
#pragma unroll
            for (int k = 0; k < 3; ++k) c = c && (e[k] + (double)((owned >> k) & 1u) > 0.0);
            if (!c) continue;
          } else if (full) {
            o[0] = o[1] = o[2] = o[3] = 1.0f;
          } else {
            bool anyc = false;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              bool c = true;
#pragma unroll
              for (int k = 0; k < 3; ++k) {
                const double dxk = (double)(int32_t)s[12 + k];
                const double dyk = (double)(int32_t)s[15 + k];
                const double ej = fma(dxk, (double)kSampleOY[j], fma(-dyk, (double)kSampleOX[j], e[k]));
                c = c && (ej + (double)((owned >> k) & 1u) > 0.0);
              }
              o[j] = c ? 1.0f : 0.0f;
              anyc = anyc || c;
            }
            if (!anyc) continue;
          }
          // perspective-correct colour at the pixel centre (clamped barycentrics)
          const float b0 = fmaxf((float)e[0], 0.0f), b1 = fmaxf((float)e[1], 0.0f),
                      b2 = fmaxf((float)e[2], 0.0f);
          const float iz0 = __uint_as_float(s[18]), iz1 = __uint_as_float(s[19]),
                      iz2 = __uint_as_float(s[20]);
          const float den = 1.0f / (b0 * iz0 + b1 * iz1 + b2 * iz2);
          const float cr = (b0 * __uint_as_float(s[21]) + b1 * __uint_as_float(s[24]) +
                            b2 * __uint_as_float(s[27])) * den;
          const float cg = (b0 * __uint_as_float(s[22]) + b1 * __uint_as_float(s[25]) +
                            b2 * __uint_as_float(s[28])) * den;
          const float cbl = (b0 * __uint_as_float(s[23]) + b1 * __uint_as_float(s[26]) +
                             b2 * __uint_as_float(s[29])) * den;
          const float alpha = __uint_as_float(s[30]);
          const int32_t pos = (int32_t)(bstart - rg.x + f + 1);
          if (mode == UMGS_MODE_DIRECT) {
            const float w = Tr * alpha;
            C0 += w * cr; C1 += w * cg; C2 += w * cbl;
            Tent = Tr;
            Tr = Tr * (1.0f - alpha);
            last = pos;
            if (Tr < kTStop) done = true;
            continue;
          }
          if (!in_entity) {
            Tin = Tr;
            Tent = Tr;
            t0 = t1 = t2 = t3 = 1.0f;
            in_entity = true;
          }
          const float O = 0.25f * (o[0] * t0 + o[1] * t1 + o[2] * t2 + o[3] * t3);
          const float w = Tin * O * alpha;
          C0 += w * cr; C1 += w * cg; C2 += w * cbl;
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
}

template <int TW, int TH>
hipError_t launch_tw(Ctx *c, float *image, float *T_final, int32_t *n_contrib, float *T_ent) {
  const size_t lds = (size_t)c->frag_batch * kSlotWords * sizeof(uint32_t);
  const uint32_t *vals = (const uint32_t *)(c->sorted_in ? c->v1.p : c->v0.p);
  ScopedTimer t(c, K_BLEND);
  hipLaunchKernelGGL((blend_kernel<TW, TH>), dim3((unsigned)c->n_tiles), dim3(TW * TH), lds,
                     c->stream, (const ViewParams *)c->d_views.p, c->V, c->N, c->T, c->mode,
                     c->frag_batch, c->bg[0], c->bg[1], c->bg[2], (const uint2 *)c->ranges.p,
                     vals, (const GaussRec *)c->grec.p, (const TriRec *)c->trec.p, image,
                     T_final, n_contrib, T_ent);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_blend(Ctx *c, float *image, float *T_final, int32_t *n_contrib,
                        float *T_entity_in) {
  if (c->n_tiles == 0) return hipSuccess;
  if (c->tile_w == 16 && c->tile_h == 16) return launch_tw<16, 16>(c, image, T_final, n_contrib, T_entity_in);
  if (c->tile_w == 8 && c->tile_h == 8) return launch_tw<8, 8>(c, image, T_final, n_contrib, T_entity_in);
  if (c->tile_w == 32 && c->tile_h == 8) return launch_tw<32, 8>(c, image, T_final, n_contrib, T_entity_in);
  return hipErrorInvalidValue;
}

}  // namespace umgs
