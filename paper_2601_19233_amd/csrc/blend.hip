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
#include "blend_common.h"

namespace umgs {

namespace {

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
  const bool direct = mode == UMGS_MODE_DIRECT;

  const uint2 rg = ranges[tile];
  const int64_t rbase = (int64_t)v * (N + T);

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
        const uint32_t rec = (uint32_t)((int64_t)v * N + local);
        stage_gauss(s, grec[rec], rec);
      } else {
        stage_tri(s, trec[(int64_t)v * T + (local - N)], P0x, P0y);
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
        const int32_t pos = (int32_t)(bstart - rg.x + f + 1);
        if ((tag & 1u) == 0u) {
          float alpha, G, dx, dy;
          if (!gauss_eval(s, pcx, pcy, alpha, G, dx, dy)) continue;
          const float test_T = Tr * (1.0f - alpha);
          if (test_T < kTStop) { done = true; continue; }
          const float w = Tr * alpha;
          C0 = fmaf(w, __uint_as_float(s[6]), C0);
          C1 = fmaf(w, __uint_as_float(s[7]), C1);
          C2 = fmaf(w, __uint_as_float(s[8]), C2);
          Tent = Tr;
          Tr = test_T;
          if (mode != UMGS_MODE_ONE_ENTITY) in_entity = false;
          last = pos;
        } else {
          double e[3];
          float o[4];
          if (tri_eval(s, rlx, rly, direct, e, o) == 0) continue;
          float cr, cg, cbl;
          tri_colour(s, e, cr, cg, cbl);
          const float alpha = __uint_as_float(s[30]);
          if (direct) {
            const float w = Tr * alpha;
            C0 = fmaf(w, cr, C0); C1 = fmaf(w, cg, C1); C2 = fmaf(w, cbl, C2);
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
