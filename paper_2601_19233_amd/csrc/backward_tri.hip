// Gradients of the triangles' appearance: per-vertex colours and opacity
// attributes, through the entity blend of Eq. 7-9 (coverage is a step
// function of the geometry and is held fixed).
//
// For an entity with entry transmittance T_in, triangles i = 1..n front to
// back, sub-sample coverage o_i^j, opacity a_i and colour c_i at the pixel,
// and colour B behind it (normalised by the transmittance after it), the
// pixel receives T_in mean_j S^j with
//   S^j = sum_i o_i^j t^j_{i-1} a_i c_i + t^j_n B,
//   t^j_i = prod_{k <= i} (1 - o_k^j a_k)            (front to back),
//   s^j_{i-1} = o_i^j a_i c_i + (1 - o_i^j a_i) s^j_i, s^j_n = B (back to front),
// so that, with g = dL/dC of the pixel,
//   dL/dc_i = T_in a_i mean_j (o_i^j t^j_{i-1}) g,
//   dL/da_i = T_in mean_j o_i^j t^j_{i-1} (c_i . g - s^j_i).
// Every gradient needs a product from the front of the entity and a sum
// from its back.  A plain division fails for opaque samples (a_i o_i^j = 1
// makes the product zero): the walk from the back (as in the Gaussian
// backward) finds each entity's span of list positions, the colour behind
// it and T_in; when the entity closes, the pixel walks the span again from
// the back, keeping s^j exactly.  Each triangle's t^j_{i-1} is then either
// the product over the span's triangles in front of it (O(n^2) triangle
// evaluations per entity of n triangles) or, when every nonzero factor is
// at least 1/16, read off two linear passes that count the exactly zero
// factors and divide only nonzero products.  Most entities hold one
// triangle, whose terms the first walk keeps (t = 1, s^j = B) and emits at
// the close directly.
// Direct mode (triangles blended like Gaussians) needs no entity:
// dL/dc = T a g, dL/da = T (c . g - B).
//
// One workgroup per tile, one pixel per thread.  The tile's triangle
// fragments get LDS accumulators (the first kTriTab of them by list
// position); a pixel adds its terms there and the workgroup adds each
// triangle's totals to global memory once.
#include "tri_grad.h"

#include <algorithm>

namespace umgs {

namespace {

constexpr int kTriTab = 512;    // triangle fragments of a tile with LDS accumulators
constexpr int kGUnroll = 8;     // Gaussians of a run evaluated together in the walk

// Highest set bit at or below slot f and at or above slot lo of the batch's
// triangle mask (lo - 1 if none).
__device__ __forceinline__ int prev_set_slot(const uint64_t *m, int f, int lo) {
  while (f >= lo) {
    const uint64_t w = m[f >> 6] & (~0ull >> (63 - (f & 63)));
    if (w) {
      const int b = (f & ~63) + 63 - (int)__builtin_clzll(w);
      return b >= lo ? b : lo - 1;
    }
    f = (f & ~63) - 1;
  }
  return lo - 1;
}

struct TriPix {
  float Tr, Tterm, dC0, dC1, dC2, Bd, ent;
  int last;
  float sd0, sd1, sd2, sd3;
  float p0, p1, p2, p3;
  PixEnt e;
};

// mask[tile] = 1 for every tile a triangle's tile rectangle reaches (a
// superset of the tiles whose lists hold a triangle; plain stores of the
// same value).
__global__ void tri_tile_mask_kernel(const ViewParams *__restrict__ views, int V, int N, int T,
                                     const uint2 *__restrict__ rects, uint32_t *__restrict__ mask) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)V * T) return;
  const int v = (int)(idx / T);
  const int64_t j = idx - (int64_t)v * T;
  const uint2 r = rects[(int64_t)v * (N + T) + N + j];
  const ViewParams &vp = views[v];
  const uint32_t tx0 = r.x & 0xFFFFu, ty0 = r.x >> 16, tx1 = r.y & 0xFFFFu, ty1 = r.y >> 16;
  for (uint32_t ty = ty0; ty < ty1; ++ty)
    for (uint32_t tx = tx0; tx < tx1; ++tx) mask[vp.tile_base + ty * (uint32_t)vp.ntx + tx] = 1u;
}

template <int TW, int TH>
__global__ __launch_bounds__(TW *TH) void tri_backward_kernel(
    const uint32_t *__restrict__ order, const uint32_t *__restrict__ key,
    const ViewParams *__restrict__ views, int V, int N, int T,
    int mode, int batch, float bg0, float bg1, float bg2, const uint2 *__restrict__ ranges,
    const uint32_t *__restrict__ v0, const uint32_t *__restrict__ v1,
    const FrameInfo *__restrict__ fi, const GaussRec *__restrict__ grec,
    const TriRec *__restrict__ trec, const TexView tex, const float *__restrict__ dLdimg,
    const float *__restrict__ Tfin, const int32_t *__restrict__ ncontrib,
    const float *__restrict__ Tent, float *__restrict__ d_rgb, float *__restrict__ d_alpha) {
  constexpr int NT = TW * TH;
  constexpr int NW = NT / 64;
  extern __shared__ uint32_t lds[];
  uint32_t *slots = lds;                                   // batch * kSlotWords
  uint32_t *tpos = lds + batch * kSlotWords;               // kTriTab
  uint32_t *ttab = tpos + kTriTab;                         // kTriTab
  float *acc = (float *)(ttab + kTriTab);                  // kTriTab * kTriAcc
  __shared__ int red[NW], red2[NW];
  __shared__ int s_ntri;
  __shared__ uint64_t tmask[NW];      // triangle slots of the staged batch (batch <= NT)
  const uint32_t *vals = fi->sorted_in ? v1 : v0;

  const uint32_t tile = order[blockIdx.x];
  if (key[tile] == 0u) return;       // no triangle reaches the tile (or nothing blended)
  const int v = find_view(views, V, tile);
  const ViewParams &vp = views[v];
  const uint32_t lt = tile - vp.tile_base;
  const int tx = (int)(lt % (uint32_t)vp.ntx), ty = (int)(lt / (uint32_t)vp.ntx);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int lx = tid % TW, ly = tid / TW;
  const int px = tx * TW + lx, py = ty * TH + ly;
  const float pcx = (float)px + 0.5f, pcy = (float)py + 0.5f;
  const int64_t P0x = (int64_t)(tx * TW) * kSubpx + kSubpx / 2;
  const int64_t P0y = (int64_t)(ty * TH) * kSubpx + kSubpx / 2;
  const double rlx = (double)(lx * kSubpx), rly = (double)(ly * kSubpx);
  const bool direct = mode == UMGS_MODE_DIRECT;
  const uint2 rg = ranges[tile];
  const int64_t rbase = (int64_t)v * (N + T);
  const int64_t HW = (int64_t)vp.W * vp.H;
  const int count = (int)(rg.y - rg.x);

  TriPix q;
  q.last = 0;
  q.Tr = 1.0f; q.Tterm = 1.0f; q.dC0 = 0.f; q.dC1 = 0.f; q.dC2 = 0.f;
  if (px < vp.W && py < vp.H) {
    const int64_t pix = (int64_t)py * vp.W + px;
    q.last = min(max(ncontrib[vp.pix_base + pix], 0), count);
    q.Tr = Tfin[vp.pix_base + pix];
    q.Tterm = Tent[vp.pix_base + pix];
    const float *d = dLdimg + 3 * vp.pix_base;
    q.dC0 = d[pix];
    q.dC1 = d[HW + pix];
    q.dC2 = d[2 * HW + pix];
  }
  q.Bd = fmaf(bg0, q.dC0, fmaf(bg1, q.dC1, bg2 * q.dC2));
  q.ent = __builtin_inff();
  q.sd0 = q.sd1 = q.sd2 = q.sd3 = 0.f;
  q.p0 = q.p1 = q.p2 = q.p3 = 1.f;
  ent_reset(q.e);

  int m = q.last;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
  if (lane == 0) red[wid] = m;
  if (tid == 0) s_ntri = 0;
  __syncthreads();
  int max_last = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) max_last = max(max_last, red[w]);
  __syncthreads();

  // the tile's triangle fragments among positions [0, max_last), in order
  for (int base = 0; base < max_last; base += NT) {
    const int pos = base + tid;
    const int64_t local = pos < max_last ? (int64_t)vals[rg.x + pos] - rbase : 0;
    const bool is_tri = pos < max_last && local >= N;
    const uint64_t bits = __ballot(is_tri);
    if (lane == 0) red[wid] = __popcll(bits);
    __syncthreads();
    int off = s_ntri;
    for (int w = 0; w < wid; ++w) off += red[w];
    off += __popcll(bits & ((1ull << lane) - 1ull));
    if (is_tri && off < kTriTab) {
      tpos[off] = (uint32_t)pos;
      ttab[off] = (uint32_t)(local - N);
    }
    __syncthreads();
    if (tid == 0) {
      int tot = 0;
      for (int w = 0; w < NW; ++w) tot += red[w];
      s_ntri += tot;
    }
    __syncthreads();
  }
  const int ntri = s_ntri;
  if (ntri == 0) return;                      // no triangle blended in this tile
  const int ntab = min(ntri, kTriTab);
  for (int i = tid; i < ntab * kTriAcc; i += NT) acc[i] = 0.0f;
  const TriRec *vrec = trec + (int64_t)v * T;

  // The pixel's frontmost covering triangle among the tabled ones (in
  // batches staged like the walk's); a pixel that blends no triangle walks
  // nothing, the others walk from their last blended fragment down to it.
  int first_cov = q.last;
  for (int c0 = 0; c0 < ntab; c0 += batch) {
    const int cn = min(batch, ntab - c0);
    __syncthreads();
    if (tid < cn) {
      const int64_t local = (int64_t)vals[rg.x + tpos[c0 + tid]] - rbase;
      const TriRec &tr = vrec[local - N];
      uint32_t *s = slots + tid * kSlotWords;
      stage_tri(s, tr, P0x, P0y);
      s[38] = tri_tile_box(tr, tx * TW, ty * TH, TW, TH);
    }
    __syncthreads();
    for (int f = 0; f < cn && first_cov == q.last; ++f) {
      const int pos = (int)tpos[c0 + f];
      if (pos >= q.last) break;
      const uint32_t *s = slots + f * kSlotWords;
      if (!in_tile_box(s[38], lx, ly)) continue;
      double e[3];
      float o[4];
      if (tri_eval(s, rlx, rly, direct, e, o) > 0) first_cov = pos;
    }
  }
  // triangles past the table are at later positions; one may still cover
  if (first_cov == q.last && ntri > ntab) first_cov = min(q.last, (int)tpos[ntab - 1] + 1);
  if (first_cov >= q.last) q.last = 0;
  int w_hi = q.last, w_lo = q.last > 0 ? first_cov : 0x7FFFFFFF;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    w_hi = max(w_hi, __shfl_xor(w_hi, o, 64));
    w_lo = min(w_lo, __shfl_xor(w_lo, o, 64));
  }
  __syncthreads();
  if (lane == 0) {
    red[wid] = w_hi;
    red2[wid] = w_lo;
  }
  __syncthreads();
  int t_hi = 0, t_lo = 0x7FFFFFFF;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    t_hi = max(t_hi, red[w]);
    t_lo = min(t_lo, red2[w]);
  }
  __syncthreads();
  TriCtx x;
  x.vals = vals + rg.x;
  x.rbase = rbase;
  x.N = N;
  x.trec = vrec;
  x.tex = tex;
  x.Px = P0x + (int64_t)(lx * kSubpx);
  x.Py = P0y + (int64_t)(ly * kSubpx);
  x.tpos = tpos;
  x.ttab = ttab;
  x.acc = acc;
  x.ntab = ntab;
  x.d_rgb = d_rgb;
  x.d_alpha = d_alpha;

  for (int bend = t_hi; bend > t_lo; bend -= batch) {
    const int bstart = max(t_lo, bend - batch);
    const int bn = bend - bstart;
    bool is_tri = false;
    if (tid < bn) {
      uint32_t *s = slots + tid * kSlotWords;
      const int64_t local = (int64_t)vals[rg.x + bstart + tid] - rbase;
      if (local < N) {
        const uint32_t rec = (uint32_t)((int64_t)v * N + local);
        stage_gauss(s, grec[rec], rec);
      } else {
        stage_tri(s, vrec[local - N], P0x, P0y);
        s[38] = tri_rank(tpos, ntab, bstart + tid);
        s[39] = (uint32_t)(local - N);
        is_tri = true;
      }
    }
    const uint64_t tbits = __ballot(is_tri);
    if (lane == 0) tmask[wid] = tbits;
    __syncthreads();
    // this wave's part of the batch, back to front: runs of Gaussians
    // between the triangles
    const int f_hi = min(bn, w_hi - bstart), f_lo = max(0, w_lo - bstart);
    int f = f_hi - 1;
    while (f >= f_lo) {
      const int ft = prev_set_slot(tmask, f, f_lo);
      if (ft < f) {
        // Gaussians (ft, f]: per-lane selects only (a fragment that is not
        // blended, or lies past the pixel's last, gets alpha 0, which leaves
        // T and B . g unchanged).  A blended Gaussian closes an open entity
        // in front of it with T as it stood at the start of the run (the
        // Gaussians before the first blended one change nothing), so the
        // close waits for the run's end.
        const float Tr0 = q.Tr;
        bool blended = false;
        for (; f - (kGUnroll - 1) > ft; f -= kGUnroll) {
          float al[kGUnroll], cd[kGUnroll];
#pragma unroll
          for (int k = 0; k < kGUnroll; ++k) {
            const uint32_t *s = slots + (f - k) * kSlotWords;
            float a;
            const bool ok = gauss_alpha(s, pcx, pcy, a) && bstart + f - k < q.last;
            blended = blended || ok;
            al[k] = ok ? a : 0.0f;
            cd[k] = fmaf(__uint_as_float(s[6]), q.dC0,
                         fmaf(__uint_as_float(s[7]), q.dC1, __uint_as_float(s[8]) * q.dC2));
          }
#pragma unroll
          for (int k = 0; k < kGUnroll; ++k) {
            const float Tb = (bstart + f - k == q.last - 1) ? q.Tterm
                                                            : q.Tr * __builtin_amdgcn_rcpf(1.0f - al[k]);
            q.Bd = fmaf(al[k], cd[k] - q.Bd, q.Bd);
            q.Tr = Tb;
          }
        }
        for (; f > ft; --f) {
          const uint32_t *s = slots + f * kSlotWords;
          float a;
          const bool ok = gauss_alpha(s, pcx, pcy, a) && bstart + f < q.last;
          blended = blended || ok;
          const float al = ok ? a : 0.0f;
          const float cd = fmaf(__uint_as_float(s[6]), q.dC0,
                                fmaf(__uint_as_float(s[7]), q.dC1, __uint_as_float(s[8]) * q.dC2));
          const float Tb = (bstart + f == q.last - 1) ? q.Tterm : q.Tr * __builtin_amdgcn_rcpf(1.0f - al);
          q.Bd = fmaf(al, cd - q.Bd, q.Bd);
          q.Tr = Tb;
        }
        if (blended && q.ent != __builtin_inff()) {
          ent_close(x, q.e, q.dC0, q.dC1, q.dC2, Tr0);
          q.ent = __builtin_inff();
        }
      }
      if (f < f_lo) break;
      // the triangle at slot f
      const uint32_t *s = slots + f * kSlotWords;
      const int pos = bstart + f;
      --f;
      if (!(pos < q.last)) continue;
      double e[3];
      float o[4];
      if (tri_eval(s, rlx, rly, direct, e, o) == 0) continue;
      float cr, cg, cb, alpha, w[3];
      float4 texel;
      tri_shade_w(SlotWords{s}, e, tex, cr, cg, cb, alpha, w, &texel);
      const float cd = fmaf(cr, q.dC0, fmaf(cg, q.dC1, cb * q.dC2));
      if (direct) {
        const float Tb = (pos == q.last - 1) ? q.Tterm : q.Tr / (1.0f - alpha);
        emit_tri(x, s[38], s[39], Tb * (cd - q.Bd), Tb * alpha, w, texel, q.dC0, q.dC1, q.dC2);
        q.Tr = Tb;
        q.Bd = fmaf(alpha, cd - q.Bd, q.Bd);
        continue;
      }
      const bool open = q.ent != __builtin_inff();
      if (!open) {
        // the walk enters an entity at its last triangle
        q.ent = (pos == q.last - 1) ? -1.0f : q.Tr;
        q.sd0 = q.sd1 = q.sd2 = q.sd3 = q.Bd;
        q.p0 = q.p1 = q.p2 = q.p3 = 1.0f;
      }
      ent_add(q.e, open, pos, s[38], s[39], q.Bd, cd, alpha,
              0.25f * ((o[0] + o[1]) + (o[2] + o[3])), w, texel);
      const float a0 = o[0] * alpha, a1 = o[1] * alpha, a2 = o[2] * alpha, a3 = o[3] * alpha;
      q.sd0 = fmaf(a0, cd - q.sd0, q.sd0);
      q.sd1 = fmaf(a1, cd - q.sd1, q.sd1);
      q.sd2 = fmaf(a2, cd - q.sd2, q.sd2);
      q.sd3 = fmaf(a3, cd - q.sd3, q.sd3);
      q.p0 *= 1.0f - a0; q.p1 *= 1.0f - a1; q.p2 *= 1.0f - a2; q.p3 *= 1.0f - a3;
      q.Bd = 0.25f * ((q.sd0 + q.sd1) + (q.sd2 + q.sd3));
      q.Tr = q.ent < 0.0f ? q.Tterm : q.ent / (0.25f * ((q.p0 + q.p1) + (q.p2 + q.p3)));
    }
    __syncthreads();
  }
  // past the tile's frontmost triangle: what is still open closes here
  if (q.ent != __builtin_inff()) ent_close(x, q.e, q.dC0, q.dC1, q.dC2, q.Tr);
  __syncthreads();

  for (int i = tid; i < ntab; i += NT) {
    const float *a = acc + kTriAcc * i;
    bool any = false;
#pragma unroll
    for (int k = 0; k < kTriAcc; ++k) any = any || a[k] != 0.0f;
    if (!any) continue;
    const int64_t t = tri_at(x, (int)tpos[i]);
    const uint32_t sw = vrec[t].swapped;
    unsafeAtomicAdd(d_alpha + t, a[0]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int vin = (sw && k) ? 3 - k : k;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) unsafeAtomicAdd(d_rgb + 9 * t + 3 * vin + ch, a[1 + 3 * k + ch]);
    }
  }
}

template <int TW, int TH>
hipError_t launch_tri_bwd_tw(Ctx *c, const float *dL, const float *Tf, const int32_t *nc,
                             const float *Te, float *d_rgb, float *d_alpha) {
  constexpr int NT = TW * TH;
  const int batch = std::min(c->frag_batch, NT);
  const size_t lds = ((size_t)batch * kSlotWords + 2 * kTriTab + (size_t)kTriTab * kTriAcc) * 4;
  const uint32_t nt = (uint32_t)c->n_tiles;
  uint32_t *key = (uint32_t *)c->bwd_order.p + 128;
  uint32_t *mask = key + 2 * (size_t)nt;
  hipError_t e = launch_fill_u32(c, mask, nt, 0u);
  if (e != hipSuccess) return e;
  const int64_t nvt = (int64_t)c->V * c->T;
  hipLaunchKernelGGL(tri_tile_mask_kernel, dim3((unsigned)ceil_div(nvt, 256)), dim3(256), 0,
                     c->stream, c->cur_views, c->V, c->N, c->T, (const uint2 *)c->rects.p, mask);
  const uint32_t *order = nullptr;
  if ((e = launch_walk_order(c, nc, &order, mask)) != hipSuccess) return e;
  hipLaunchKernelGGL((tri_backward_kernel<TW, TH>), dim3(nt), dim3(NT), lds,
                     c->stream, order, (const uint32_t *)key, c->cur_views, c->V, c->N, c->T, c->mode, batch, c->bg[0],
                     c->bg[1], c->bg[2], (const uint2 *)c->ranges.p, (const uint32_t *)c->v0.p,
                     (const uint32_t *)c->v1.p, (const FrameInfo *)c->finfo.p,
                     (const GaussRec *)c->grec.p, (const TriRec *)c->trec.p, frame_texture(c), dL,
                     Tf, nc, Te, d_rgb, d_alpha);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_backward_triangles(Ctx *c, const float *dL, const float *Tf, const int32_t *nc,
                                     const float *Te, float *d_rgb, float *d_alpha,
                                     bool accumulate) {
  hipError_t e = hipSuccess;
  if (!accumulate) {
    e = launch_fill_u32(c, (uint32_t *)d_rgb, 9 * (int64_t)c->T, 0u);
    if (e == hipSuccess) e = launch_fill_u32(c, (uint32_t *)d_alpha, c->T, 0u);
    if (e != hipSuccess) return e;
  }
  if (c->n_tiles == 0 || c->T == 0) return hipSuccess;
  ScopedTimer t(c, K_BLEND_BWD_TRI);
  if (c->tile_w == 16 && c->tile_h == 16) return launch_tri_bwd_tw<16, 16>(c, dL, Tf, nc, Te, d_rgb, d_alpha);
  if (c->tile_w == 8 && c->tile_h == 8) return launch_tri_bwd_tw<8, 8>(c, dL, Tf, nc, Te, d_rgb, d_alpha);
  return launch_tri_bwd_tw<32, 8>(c, dL, Tf, nc, Te, d_rgb, d_alpha);
}

}  // namespace umgs
