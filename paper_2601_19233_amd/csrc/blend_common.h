// Per-fragment evaluation shared by the forward and backward blend kernels.
// Both kernels must take identical discrete decisions (contributes or not,
// sub-sample coverage), so the arithmetic is written with explicit fmaf and
// lives in one place.
#pragma once

#include "internal.h"

namespace umgs {

constexpr int kSlotWords = 40;   // one staged fragment: 160 B of LDS

// Slot layout (32-bit words)
//   Gaussian: 0 mx, 1 my, 2 qa, 3 qb, 4 qc (times log2(e)), 5 lo = log2(o),
//             6 r, 7 g, 8 b, 9 1/o, 10 record index (view * N + i), 31 tag = 0
//   triangle: 0-5 E0[3] (FP64 edge functions at the tile's first pixel
//             centre), 6-11 dmax[3] (FP64, max |offset term| over samples),
//             12-14 dx[3], 15-17 dy[3] (int32), 18-20 1/z, 21-29 colour/z,
//             30 alpha, 31 tag = 1 | owned << 8, 32-37 (u, v)/z

// rotated-grid sample offsets from the pixel centre, 1/256 px
__device__ __forceinline__ int sample_ox(int j) { return j == 0 ? -32 : j == 1 ? 96 : j == 2 ? -96 : 32; }
__device__ __forceinline__ int sample_oy(int j) { return j == 0 ? -96 : j == 1 ? -32 : j == 2 ? 32 : 96; }

constexpr int kSlotInvO = 9;
constexpr int kSlotRec = 10;

__device__ __forceinline__ void stage_gauss(uint32_t *s, const GaussRec &g, uint32_t rec) {
  *(float4 *)(s + 0) = make_float4(g.mx, g.my, g.qa, g.qb);
  *(float4 *)(s + 4) = make_float4(g.qc, g.lo, g.r, g.g);
  s[8] = __float_as_uint(g.b);
  s[kSlotInvO] = __float_as_uint(g.inv_o);
  s[kSlotRec] = rec;
  s[31] = 0u;
}

// The pixels of a tile whose sub-samples can fall inside the triangle's
// bounding box (samples, and the direct mode's pixel centre, lie 32..224 /
// 256 px into their pixel), tile-relative [x0, x1) x [y0, y1) clamped to the
// tile, packed x0 | y0 << 8 | x1 << 16 | y1 << 24.  No pixel outside it has
// a covered sample.
__device__ __forceinline__ uint32_t tri_tile_box(const TriRec &tr, int px0, int py0, int TW, int TH) {
  const int minX = min(tr.X[0], min(tr.X[1], tr.X[2])), maxX = max(tr.X[0], max(tr.X[1], tr.X[2]));
  const int minY = min(tr.Y[0], min(tr.Y[1], tr.Y[2])), maxY = max(tr.Y[0], max(tr.Y[1], tr.Y[2]));
  const int x0 = min(max(((minX + 31) >> 8) - px0, 0), TW);
  const int x1 = min(max(((maxX - 32) >> 8) + 1 - px0, 0), TW);
  const int y0 = min(max(((minY + 31) >> 8) - py0, 0), TH);
  const int y1 = min(max(((maxY - 32) >> 8) + 1 - py0, 0), TH);
  return (uint32_t)x0 | ((uint32_t)y0 << 8) | ((uint32_t)x1 << 16) | ((uint32_t)y1 << 24);
}

__device__ __forceinline__ bool in_tile_box(uint32_t bx, int lx, int ly) {
  return lx >= (int)(bx & 0xFFu) && ly >= (int)((bx >> 8) & 0xFFu) && lx < (int)((bx >> 16) & 0xFFu) &&
         ly < (int)(bx >> 24);
}

__device__ __forceinline__ void stage_tri(uint32_t *s, const TriRec &tr, int64_t P0x, int64_t P0y) {
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
#pragma unroll
  for (int k = 0; k < 6; ++k) s[32 + k] = __float_as_uint(tr.uviz[k]);
}

// p = log2(o exp(power)) = (qa dx + qb dy) dx + (qc dy dy + lo) with the
// record's log2(e)-scaled coefficients and lo = log2(o) (5 operations);
// power <= 0 iff p <= lo.  Every kernel takes its decisions from this one
// expression.
__device__ __forceinline__ float gauss_logalpha(float qa, float qb, float qc, float lo, float dx,
                                                float dy) {
  return fmaf(fmaf(qa, dx, qb * dy), dx, fmaf(qc * dy, dy, lo));
}

// Gaussian: alpha = min(0.99, 2^p) at the pixel centre, without branches
// (lanes where power > 0 compute a value that is then discarded).  Returns
// whether the fragment contributes (power <= 0 and alpha >= 1/255).
__device__ __forceinline__ bool gauss_alpha(const uint32_t *s, float pcx, float pcy, float &alpha) {
  const float4 a = *(const float4 *)(s + 0);
  const float4 b = *(const float4 *)(s + 4);
  const float dx = a.x - pcx;
  const float dy = a.y - pcy;
  const float p = gauss_logalpha(a.z, a.w, b.x, b.y, dx, dy);
  alpha = fminf(kAlphaMax, __builtin_amdgcn_exp2f(p));
  return p <= b.y && alpha >= kAlphaMin;
}

// gauss_alpha that also returns a = o exp(power) before the clamp (o where
// power > 0) and the offsets the gradients need (all finite for any record;
// meaningful when it returns true).  Bit-identical alpha and decision.
__device__ __forceinline__ bool gauss_terms(const uint32_t *s, float pcx, float pcy, float &alpha,
                                            float &a_un, float &dx, float &dy) {
  const float4 a = *(const float4 *)(s + 0);
  const float4 b = *(const float4 *)(s + 4);
  dx = a.x - pcx;
  dy = a.y - pcy;
  const float p = gauss_logalpha(a.z, a.w, b.x, b.y, dx, dy);
  const bool inside = p <= b.y;
  a_un = __builtin_amdgcn_exp2f(inside ? p : b.y);
  alpha = a_un < kAlphaMax ? a_un : kAlphaMax;   // min(0.99, a), as a select
  return inside && alpha >= kAlphaMin;
}

// Sub-sample coverage from the exact edge values e[k] at the pixel centre,
// the edge steps dxk/dyk, the bound dmax[k] of the sample offset terms and
// the edge ownership bits.  Returns the number of covered samples (0: not a
// fragment of this pixel).  In direct mode only the pixel centre is tested
// and o[] is 1.
__device__ __forceinline__ int tri_cover(const double e[3], const double dxk[3], const double dyk[3],
                                         const double dmax[3], uint32_t owned, bool direct,
                                         float o[4]) {
  bool any = true, full = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double own = (double)((owned >> k) & 1u);
    any = any && (e[k] + dmax[k] + own > 0.0);
    full = full && (e[k] - dmax[k] > 0.0);
  }
  if (!any) return 0;
  if (direct) {
    bool c = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) c = c && (e[k] + (double)((owned >> k) & 1u) > 0.0);
    o[0] = o[1] = o[2] = o[3] = 1.0f;
    return c ? 4 : 0;
  }
  if (full) {
    o[0] = o[1] = o[2] = o[3] = 1.0f;
    return 4;
  }
  int n = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    bool c = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double ej = fma(dxk[k], (double)sample_oy(j), fma(-dyk[k], (double)sample_ox(j), e[k]));
      c = c && (ej + (double)((owned >> k) & 1u) > 0.0);
    }
    o[j] = c ? 1.0f : 0.0f;
    n += c;
  }
  return n;
}

// Triangle staged in an LDS slot: edge functions at the pixel (offset rlx,
// rly from the tile's first pixel centre, 1/256 px) and sub-sample coverage.
__device__ __forceinline__ int tri_eval(const uint32_t *s, double rlx, double rly, bool direct,
                                        double e[3], float o[4]) {
  const double *dv = (const double *)s;
  double dxk[3], dyk[3], dmax[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    dxk[k] = (double)(int32_t)s[12 + k];
    dyk[k] = (double)(int32_t)s[15 + k];
    e[k] = fma(dxk[k], rly, fma(-dyk[k], rlx, dv[k]));
    dmax[k] = dv[3 + k];
  }
  return tri_cover(e, dxk, dyk, dmax, s[31] >> 8, direct, o);
}

// The same from the triangle's record at the pixel centre (Px, Py) in
// 1/256 px: the edge functions are the same integers (exact in FP64 in both
// forms), so coverage and shading are bit-identical to tri_eval's.
__device__ __forceinline__ int tri_eval_rec(const TriRec &tr, int64_t Px, int64_t Py, bool direct,
                                            double e[3], float o[4]) {
  const int ea[3] = {1, 2, 0}, eb[3] = {2, 0, 1};
  double dxk[3], dyk[3], dmax[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int64_t dx = (int64_t)tr.X[eb[k]] - tr.X[ea[k]];
    const int64_t dy = (int64_t)tr.Y[eb[k]] - tr.Y[ea[k]];
    e[k] = (double)(dx * (Py - tr.Y[ea[k]]) - dy * (Px - tr.X[ea[k]]));
    dxk[k] = (double)dx;
    dyk[k] = (double)dy;
    dmax[k] = 96.0 * (double)((dx < 0 ? -dx : dx) + (dy < 0 ? -dy : dy));
  }
  return tri_cover(e, dxk, dyk, dmax, tr.owned, direct, o);
}

// a + f (b - a), the interpolation step of the bilinear texture fetch (a
// constant texture returns its value exactly)
__device__ __forceinline__ float4 lerp4(float4 a, float4 b, float f) {
  return make_float4(fmaf(f, b.x - a.x, a.x), fmaf(f, b.y - a.y, a.y), fmaf(f, b.z - a.z, a.z),
                     fmaf(f, b.w - a.w, a.w));
}

// Bilinear RGBA at texture coordinates (u, v): texel (i, j) is centred at
// ((i + 1/2)/w, (j + 1/2)/h); addresses clamp to the edge texels (also for
// non-finite coordinates, so no fetch leaves the texture).
__device__ __forceinline__ float4 tex_sample(const TexView &tv, float u, float v) {
  const float x = fmaf(u, (float)tv.w, -0.5f), y = fmaf(v, (float)tv.h, -0.5f);
  const float x0 = floorf(x), y0 = floorf(y);
  const float fx = x - x0, fy = y - y0;
  const float xc = fminf(fmaxf(x0, -1.0f), (float)tv.w), yc = fminf(fmaxf(y0, -1.0f), (float)tv.h);
  const int i0 = min(max((int)xc, 0), tv.w - 1), i1 = min(max((int)xc + 1, 0), tv.w - 1);
  const int j0 = min(max((int)yc, 0), tv.h - 1), j1 = min(max((int)yc + 1, 0), tv.h - 1);
  const float4 *r0 = tv.texels + (int64_t)j0 * tv.w, *r1 = tv.texels + (int64_t)j1 * tv.w;
  const float4 top = lerp4(r0[i0], r0[i1], fx), bot = lerp4(r1[i0], r1[i1], fx);
  return lerp4(top, bot, fy);
}

// A triangle's shading words, read from its LDS slot or from its record
// (slot word numbering: 18-20 1/z, 21-29 colour/z, 30 alpha, 32-37 (u, v)/z).
struct SlotWords {
  const uint32_t *s;
  __device__ __forceinline__ float operator()(int i) const { return __uint_as_float(s[i]); }
};
struct RecWords {
  const TriRec *r;
  __device__ __forceinline__ float operator()(int i) const {
    return i < 21 ? r->iz[i - 18] : i < 30 ? r->ciz[i - 21] : i == 30 ? r->alpha : r->uviz[i - 32];
  }
};

// Colour and opacity of a triangle at the pixel centre: the per-vertex
// colour and (with a texture) the texture coordinates interpolated
// perspective-correctly from the (clamped) barycentric edge functions; a
// textured triangle's colour is multiplied by the texel RGB and its opacity
// attribute by the texel alpha.  Optionally also returns the interpolation
// weights w[k] of the vertices (colour = sum_k w_k rgb_k, times the texel)
// and the texel (1 without a texture).
template <class Words>
__device__ __forceinline__ void tri_shade_w(const Words &at, const double e[3], const TexView &tv,
                                            float &cr, float &cg, float &cb, float &alpha,
                                            float *w = nullptr, float4 *texel = nullptr) {
  const float b0 = fmaxf((float)e[0], 0.0f), b1 = fmaxf((float)e[1], 0.0f),
              b2 = fmaxf((float)e[2], 0.0f);
  const float iz0 = at(18), iz1 = at(19), iz2 = at(20);
  const float den = 1.0f / (b0 * iz0 + b1 * iz1 + b2 * iz2);
  cr = (b0 * at(21) + b1 * at(24) + b2 * at(27)) * den;
  cg = (b0 * at(22) + b1 * at(25) + b2 * at(28)) * den;
  cb = (b0 * at(23) + b1 * at(26) + b2 * at(29)) * den;
  alpha = at(30);
  if (w) {
    w[0] = b0 * iz0 * den;
    w[1] = b1 * iz1 * den;
    w[2] = b2 * iz2 * den;
  }
  if (texel) *texel = make_float4(1.0f, 1.0f, 1.0f, 1.0f);
  if (tv.texels) {
    const float u = (b0 * at(32) + b1 * at(34) + b2 * at(36)) * den;
    const float v = (b0 * at(33) + b1 * at(35) + b2 * at(37)) * den;
    const float4 t = tex_sample(tv, u, v);
    cr *= t.x;
    cg *= t.y;
    cb *= t.z;
    alpha *= t.w;
    if (texel) *texel = t;
  }
}

__device__ __forceinline__ void tri_shade(const uint32_t *s, const double e[3], const TexView &tv,
                                          float &cr, float &cg, float &cb, float &alpha) {
  tri_shade_w(SlotWords{s}, e, tv, cr, cg, cb, alpha);
}

__device__ __forceinline__ int find_view(const ViewParams *views, int V, uint32_t tile) {
  int lo = 0, hi = V - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace umgs
