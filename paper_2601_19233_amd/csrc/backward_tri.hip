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
// from its back.  Recovering either by division fails for opaque samples
// (a_i o_i^j = 1 makes the product zero), so the kernel takes neither by
// division: the walk from the back (as in the Gaussian backward) finds each
// entity's span of list positions, the colour behind it and T_in; when the
// entity closes, the pixel walks the span again from the back, keeping s^j
// exactly, and takes each triangle's t^j_{i-1} as the product over the
// span's triangles in front of it.  That costs O(n^2) triangle evaluations
// per entity of n triangles; most entities hold one triangle, whose terms
// the first walk keeps (t = 1, s^j = B) and emits at the close directly.
// Direct mode (triangles blended like Gaussians) needs no entity:
// dL/dc = T a g, dL/da = T (c . g - B).
//
// One workgroup per tile, one pixel per thread.  The tile's triangle
// fragments get LDS accumulators (the first kTriTab of them by list
// position); a pixel adds its terms there and the workgroup adds each
// triangle's totals to global memory once.
#include "blend_common.h"

#include <algorithm>

namespace umgs {

namespace {

constexpr int kTriTab = 512;    // triangle fragments of a tile with LDS accumulators
constexpr int kTriAcc = 10;     // opacity, then 3 vertices x RGB

struct TriPix {
  float Tr, Tterm, dC0, dC1, dC2, Bd, ent;
  int last;
  float sd0, sd1, sd2, sd3;
  float p0, p1, p2, p3;
  int fpos, bpos;   // list positions of the open entity's front and back triangles
  float Bback;      // B . g behind the open entity
  int n_ent;        // its triangles so far
  // the gradient terms of its back triangle as if it were alone (t = 1,
  // s^j = B), without the factor T_in: what an entity of one triangle (most
  // of them) emits at its close, with no second walk
  uint32_t c_rank, c_t;
  float c_da, c_vis, c_w0, c_w1, c_w2;
  float4 c_texel;
};

struct TriCtx {
  const uint32_t *vals;       // the tile's list (global)
  int64_t rbase;              // view * (N + T)
  int N;
  const TriRec *trec;         // this view's records
  TexView tex;
  int64_t Px, Py;             // pixel centre, 1/256 px
  const uint32_t *tpos;       // LDS: ascending list positions of the tile's triangles
  float *acc;                 // LDS: their accumulators
  int ntab;                   // entries in tpos / acc
  float *d_rgb, *d_alpha;
};

// Rank of list position pos among the tile's triangle fragments if it has
// an LDS accumulator, else kNoRank.
constexpr uint32_t kNoRank = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t tri_rank(const uint32_t *tpos, int ntab, int pos) {
  int lo = 0, hi = ntab;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((int)tpos[mid] < pos) lo = mid + 1; else hi = mid;
  }
  return (lo < ntab && (int)tpos[lo] == pos) ? (uint32_t)lo : kNoRank;
}

// Adds one (pixel, triangle) term: dL/d(effective opacity) da and the
// colour gradient vis g (vis = T_in a mean_j o^j t^j), spread over the
// vertices with the interpolation weights w and the texel; rank is the
// triangle's accumulator (kNoRank: global memory).
__device__ __forceinline__ void emit(const TriCtx &x, uint32_t rank, int64_t t, float da, float vis,
                                     const float w[3], float4 texel, const TriPix &q) {
  const float da_attr = da * texel.w;
  const float gc[3] = {vis * texel.x * q.dC0, vis * texel.y * q.dC1, vis * texel.z * q.dC2};
  if (rank != kNoRank) {
    float *a = x.acc + kTriAcc * rank;
    atomicAdd(a, da_attr);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) atomicAdd(a + 1 + 3 * k + ch, w[k] * gc[ch]);
    return;
  }
  const uint32_t sw = x.trec[t].swapped;
  unsafeAtomicAdd(x.d_alpha + t, da_attr);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int vin = (sw && k) ? 3 - k : k;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) unsafeAtomicAdd(x.d_rgb + 9 * t + 3 * vin + ch, w[k] * gc[ch]);
  }
}

// Triangle index (within the view) of list position pos, or -1 for a Gaussian.
__device__ __forceinline__ int64_t tri_at(const TriCtx &x, int pos) {
  const int64_t local = (int64_t)x.vals[pos] - x.rbase;
  return local < x.N ? -1 : local - x.N;
}

// The gradients of the entity [q.fpos, q.bpos] of this pixel, entered with
// transmittance T_in.
__device__ void rewalk_entity(const TriCtx &x, const TriPix &q, float T_in) {
  float s0 = q.Bback, s1 = q.Bback, s2 = q.Bback, s3 = q.Bback;
  for (int pi = q.bpos; pi >= q.fpos; --pi) {
    const int64_t ti = tri_at(x, pi);
    if (ti < 0) continue;
    const TriRec &ri = x.trec[ti];
    double e[3];
    float o[4];
    if (tri_eval_rec(ri, x.Px, x.Py, false, e, o) == 0) continue;
    float cr, cg, cb, a, w[3];
    float4 texel;
    tri_shade_w(RecWords{&ri}, e, x.tex, cr, cg, cb, a, w, &texel);
    // t^j in front of triangle i within the entity
    float t0 = 1.0f, t1 = 1.0f, t2 = 1.0f, t3 = 1.0f;
    for (int pk = q.fpos; pk < pi; ++pk) {
      const int64_t tk = tri_at(x, pk);
      if (tk < 0) continue;
      const TriRec &rk = x.trec[tk];
      double ek[3];
      float ok[4];
      if (tri_eval_rec(rk, x.Px, x.Py, false, ek, ok) == 0) continue;
      float kr, kg, kb, ak;
      tri_shade_w(RecWords{&rk}, ek, x.tex, kr, kg, kb, ak);
      t0 *= 1.0f - ok[0] * ak; t1 *= 1.0f - ok[1] * ak;
      t2 *= 1.0f - ok[2] * ak; t3 *= 1.0f - ok[3] * ak;
    }
    const float cd = fmaf(cr, q.dC0, fmaf(cg, q.dC1, cb * q.dC2));
    const float v0 = o[0] * t0, v1 = o[1] * t1, v2 = o[2] * t2, v3 = o[3] * t3;
    const float da = T_in * 0.25f * ((v0 * (cd - s0) + v1 * (cd - s1)) + (v2 * (cd - s2) + v3 * (cd - s3)));
    const float vis = T_in * a * 0.25f * ((v0 + v1) + (v2 + v3));
    emit(x, tri_rank(x.tpos, x.ntab, pi), ti, da, vis, w, texel, q);
    s0 = fmaf(o[0] * a, cd - s0, s0);
    s1 = fmaf(o[1] * a, cd - s1, s1);
    s2 = fmaf(o[2] * a, cd - s2, s2);
    s3 = fmaf(o[3] * a, cd - s3, s3);
  }
}

__device__ __forceinline__ void close_entity(const TriCtx &x, const TriPix &q, float T_in) {
  if (q.n_ent == 1) {
    const float w[3] = {q.c_w0, q.c_w1, q.c_w2};
    emit(x, q.c_rank, q.c_t, T_in * q.c_da, T_in * q.c_vis, w, q.c_texel, q);
  } else {
    rewalk_entity(x, q, T_in);
  }
}

template <int TW, int TH>
__global__ __launch_bounds__(TW *TH) void tri_backward_kernel(
    const uint32_t *__restrict__ order, const ViewParams *__restrict__ views, int V, int N, int T,
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
  float *acc = (float *)(tpos + kTriTab);                  // kTriTab * kTriAcc
  __shared__ int red[NW], red2[NW];
  __shared__ int s_ntri;
  const uint32_t *vals = fi->sorted_in ? v1 : v0;

  const uint32_t tile = order[blockIdx.x];
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
  q.fpos = q.bpos = 0;
  q.Bback = 0.f;
  q.n_ent = 0;
  q.c_rank = kNoRank;
  q.c_t = 0;
  q.c_da = q.c_vis = q.c_w0 = q.c_w1 = q.c_w2 = 0.f;
  q.c_texel = make_float4(1.f, 1.f, 1.f, 1.f);

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
    const bool is_tri = pos < max_last && (int64_t)vals[rg.x + pos] - rbase >= N;
    const uint64_t bits = __ballot(is_tri);
    if (lane == 0) red[wid] = __popcll(bits);
    __syncthreads();
    int off = s_ntri;
    for (int w = 0; w < wid; ++w) off += red[w];
    off += __popcll(bits & ((1ull << lane) - 1ull));
    if (is_tri && off < kTriTab) tpos[off] = (uint32_t)pos;
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
      stage_tri(slots + tid * kSlotWords, vrec[local - N], P0x, P0y);
    }
    __syncthreads();
    for (int f = 0; f < cn && first_cov == q.last; ++f) {
      const int pos = (int)tpos[c0 + f];
      if (pos >= q.last) break;
      double e[3];
      float o[4];
      if (tri_eval(slots + f * kSlotWords, rlx, rly, direct, e, o) > 0) first_cov = pos;
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
  x.acc = acc;
  x.ntab = ntab;
  x.d_rgb = d_rgb;
  x.d_alpha = d_alpha;

  for (int bend = t_hi; bend > t_lo; bend -= batch) {
    const int bstart = max(t_lo, bend - batch);
    const int bn = bend - bstart;
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
      }
    }
    __syncthreads();
    // this wave's part of the batch
    const int f_hi = min(bn, w_hi - bstart), f_lo = max(0, w_lo - bstart);
    for (int f = f_hi - 1; f >= f_lo; --f) {
      const uint32_t *s = slots + f * kSlotWords;
      const int pos = bstart + f;
      if (!(pos < q.last)) continue;
      if ((s[31] & 1u) == 0u) {
        float alpha, a_un, dx, dy;
        if (!gauss_terms(s, pcx, pcy, alpha, a_un, dx, dy)) continue;
        // a blended Gaussian in front of an open entity closes it
        if (q.ent != __builtin_inff()) {
          close_entity(x, q, q.Tr);
          q.ent = __builtin_inff();
        }
        const float Tb = (pos == q.last - 1) ? q.Tterm : q.Tr * __builtin_amdgcn_rcpf(1.0f - alpha);
        const float cd = fmaf(__uint_as_float(s[6]), q.dC0,
                              fmaf(__uint_as_float(s[7]), q.dC1, __uint_as_float(s[8]) * q.dC2));
        q.Bd = fmaf(alpha, cd - q.Bd, q.Bd);
        q.Tr = Tb;
      } else {
        double e[3];
        float o[4];
        if (tri_eval(s, rlx, rly, direct, e, o) == 0) continue;
        float cr, cg, cb, alpha, w[3];
        float4 texel;
        tri_shade_w(SlotWords{s}, e, tex, cr, cg, cb, alpha, w, &texel);
        const float cd = fmaf(cr, q.dC0, fmaf(cg, q.dC1, cb * q.dC2));
        if (direct) {
          const float Tb = (pos == q.last - 1) ? q.Tterm : q.Tr / (1.0f - alpha);
          emit(x, s[38], s[39], Tb * (cd - q.Bd), Tb * alpha, w, texel, q);
          q.Tr = Tb;
          q.Bd = fmaf(alpha, cd - q.Bd, q.Bd);
          continue;
        }
        if (q.ent == __builtin_inff()) {
          // the walk enters an entity at its last triangle
          q.ent = (pos == q.last - 1) ? -1.0f : q.Tr;
          q.sd0 = q.sd1 = q.sd2 = q.sd3 = q.Bd;
          q.p0 = q.p1 = q.p2 = q.p3 = 1.0f;
          q.bpos = pos;
          q.Bback = q.Bd;
          q.n_ent = 0;
        }
        if (++q.n_ent == 1) {
          const float n = 0.25f * ((o[0] + o[1]) + (o[2] + o[3]));
          q.c_rank = s[38];
          q.c_t = s[39];
          q.c_da = n * (cd - q.Bd);
          q.c_vis = n * alpha;
          q.c_w0 = w[0];
          q.c_w1 = w[1];
          q.c_w2 = w[2];
          q.c_texel = texel;
        }
        q.fpos = pos;
        const float a0 = o[0] * alpha, a1 = o[1] * alpha, a2 = o[2] * alpha, a3 = o[3] * alpha;
        q.sd0 = fmaf(a0, cd - q.sd0, q.sd0);
        q.sd1 = fmaf(a1, cd - q.sd1, q.sd1);
        q.sd2 = fmaf(a2, cd - q.sd2, q.sd2);
        q.sd3 = fmaf(a3, cd - q.sd3, q.sd3);
        q.p0 *= 1.0f - a0; q.p1 *= 1.0f - a1; q.p2 *= 1.0f - a2; q.p3 *= 1.0f - a3;
        q.Bd = 0.25f * ((q.sd0 + q.sd1) + (q.sd2 + q.sd3));
        q.Tr = q.ent < 0.0f ? q.Tterm : q.ent / (0.25f * ((q.p0 + q.p1) + (q.p2 + q.p3)));
      }
    }
    __syncthreads();
  }
  // past the tile's frontmost triangle: what is still open closes here
  if (q.ent != __builtin_inff()) close_entity(x, q, q.Tr);
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
  const size_t lds = ((size_t)batch * kSlotWords + kTriTab + (size_t)kTriTab * kTriAcc) * 4;
  const uint32_t *order = nullptr;
  hipError_t e = launch_walk_order(c, nc, &order);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((tri_backward_kernel<TW, TH>), dim3((uint32_t)c->n_tiles), dim3(NT), lds,
                     c->stream, order, c->cur_views, c->V, c->N, c->T, c->mode, batch, c->bg[0],
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
