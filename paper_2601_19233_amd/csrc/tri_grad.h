// Pieces of the triangle gradients (per-vertex colour and opacity, through
// the sub-sample entity blend of Eq. 7-9): the entity bookkeeping of one
// pixel, the emission of a (pixel, triangle) term and the re-walk of an
// entity of several triangles.
//
// For an entity with entry transmittance T_in, triangles i = 1..n front to
// back, sub-sample coverage o_i^j, opacity a_i, colour c_i at the pixel and
// colour B behind it, with g = dL/dC of the pixel,
//   dL/dc_i = T_in a_i mean_j (o_i^j t^j_{i-1}) g,
//   dL/da_i = T_in mean_j o_i^j t^j_{i-1} (c_i . g - s^j_i),
//   t^j_i = prod_{k <= i} (1 - o_k^j a_k)   (front to back),
//   s^j_{i-1} = o_i^j a_i c_i + (1 - o_i^j a_i) s^j_i, s^j_n = B   (back to front).
// A tile's triangle fragments get LDS accumulators (kTriAcc floats) by a
// rank; terms of the rest go straight to global memory.
#pragma once

#include "blend_common.h"

namespace umgs {

constexpr int kTriAcc = 10;               // opacity, then 3 vertices x RGB
constexpr uint32_t kNoRank = 0xFFFFFFFFu;  // no LDS accumulator

struct TriCtx {
  const uint32_t *vals;       // the tile's list (global)
  int64_t rbase;              // view * (N + T)
  int N;
  const TriRec *trec;         // this view's records
  TexView tex;
  int64_t Px, Py;             // pixel centre, 1/256 px
  // ranks: the index in tpos (LDS, ascending list positions of the tile's
  // triangles) when tpos is set; else counted from the back of the walk
  // (the span's back triangle has rank rank_b and each triangle fragment
  // in front of it one more)
  const uint32_t *tpos;
  // with tpos: the triangle index (within the view) of each rank, in LDS,
  // so that a re-walk visits the span's triangles without the list
  const uint32_t *ttab;
  float *acc;                 // LDS accumulators
  int ntab;                   // accumulators
  float *d_rgb, *d_alpha;
};

// An entity's span of list positions, the rank of its back triangle and
// the colour behind it (as B . g).
struct EntSpan {
  int fpos, bpos;
  uint32_t rank_b;
  float Bback;
};

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
// vertices with the interpolation weights w and the texel; rank selects
// the accumulator (kNoRank or past the table: global memory, in the
// caller's vertex order).
__device__ __forceinline__ void emit_tri(const TriCtx &x, uint32_t rank, int64_t t, float da,
                                         float vis, const float w[3], float4 texel, float g0,
                                         float g1, float g2) {
  const float da_attr = da * texel.w;
  const float gc[3] = {vis * texel.x * g0, vis * texel.y * g1, vis * texel.z * g2};
  if (rank < (uint32_t)x.ntab) {
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

// Smallest nonzero factor and product floor for rewalk_linear: a factor of
// at least 1/16 carries a relative error of at most 15 ulp and no product
// underflows, so each quotient is good to about 32 n ulp for n triangles.
constexpr float kDivFactorMin = 1.0f / 16.0f;
constexpr float kDivProductMin = 1e-30f;

// The re-walk of an entity whose span is the tabled ranks [rf, rank_b] in
// two linear passes, when that is exact enough: the first counts, per
// sample, the factors 1 - o^j a that are exactly zero (opaque coverage) and
// multiplies the others; the second walks from the back keeping the same
// count and product over the suffix, so that the front product of triangle
// i is zero if a zero factor lies in front of it, else the entity's nonzero
// product over the suffix's.  Returns false (nothing emitted) when a
// nonzero factor is below kDivFactorMin or a product below kDivProductMin.
__device__ bool rewalk_linear(const TriCtx &x, const EntSpan &sp, int rf, float g0, float g1,
                              float g2, float T_in) {
  float P0 = 1.0f, P1 = 1.0f, P2 = 1.0f, P3 = 1.0f;
  int z0 = 0, z1 = 0, z2 = 0, z3 = 0;
  bool ok = true;
  for (int ri = (int)sp.rank_b; ri >= rf; --ri) {
    const TriRec &r = x.trec[x.ttab[ri]];
    double e[3];
    float o[4];
    if (tri_eval_rec(r, x.Px, x.Py, false, e, o) == 0) continue;
    float cr, cg, cb, a;
    tri_shade_w(RecWords{&r}, e, x.tex, cr, cg, cb, a);
    const float f[4] = {1.0f - o[0] * a, 1.0f - o[1] * a, 1.0f - o[2] * a, 1.0f - o[3] * a};
    ok = ok && (f[0] == 0.0f || f[0] >= kDivFactorMin) && (f[1] == 0.0f || f[1] >= kDivFactorMin) &&
         (f[2] == 0.0f || f[2] >= kDivFactorMin) && (f[3] == 0.0f || f[3] >= kDivFactorMin);
    if (f[0] == 0.0f) ++z0; else P0 *= f[0];
    if (f[1] == 0.0f) ++z1; else P1 *= f[1];
    if (f[2] == 0.0f) ++z2; else P2 *= f[2];
    if (f[3] == 0.0f) ++z3; else P3 *= f[3];
  }
  if (!ok || fminf(fminf(P0, P1), fminf(P2, P3)) < kDivProductMin) return false;
  float s0 = sp.Bback, s1 = sp.Bback, s2 = sp.Bback, s3 = sp.Bback;
  float S0 = 1.0f, S1 = 1.0f, S2 = 1.0f, S3 = 1.0f;
  for (int ri = (int)sp.rank_b; ri >= rf; --ri) {
    const int64_t ti = x.ttab[ri];
    const TriRec &r = x.trec[ti];
    double e[3];
    float o[4];
    if (tri_eval_rec(r, x.Px, x.Py, false, e, o) == 0) continue;
    float cr, cg, cb, a, w[3];
    float4 texel;
    tri_shade_w(RecWords{&r}, e, x.tex, cr, cg, cb, a, w, &texel);
    const float f0 = 1.0f - o[0] * a, f1 = 1.0f - o[1] * a, f2 = 1.0f - o[2] * a, f3 = 1.0f - o[3] * a;
    if (f0 == 0.0f) --z0; else S0 *= f0;
    if (f1 == 0.0f) --z1; else S1 *= f1;
    if (f2 == 0.0f) --z2; else S2 *= f2;
    if (f3 == 0.0f) --z3; else S3 *= f3;
    // z: zero factors in front of this triangle
    const float t0 = z0 > 0 ? 0.0f : P0 / S0, t1 = z1 > 0 ? 0.0f : P1 / S1;
    const float t2 = z2 > 0 ? 0.0f : P2 / S2, t3 = z3 > 0 ? 0.0f : P3 / S3;
    const float cd = fmaf(cr, g0, fmaf(cg, g1, cb * g2));
    const float v0 = o[0] * t0, v1 = o[1] * t1, v2 = o[2] * t2, v3 = o[3] * t3;
    const float da = T_in * 0.25f * ((v0 * (cd - s0) + v1 * (cd - s1)) + (v2 * (cd - s2) + v3 * (cd - s3)));
    const float vis = T_in * a * 0.25f * ((v0 + v1) + (v2 + v3));
    emit_tri(x, (uint32_t)ri, ti, da, vis, w, texel, g0, g1, g2);
    s0 = fmaf(o[0] * a, cd - s0, s0);
    s1 = fmaf(o[1] * a, cd - s1, s1);
    s2 = fmaf(o[2] * a, cd - s2, s2);
    s3 = fmaf(o[3] * a, cd - s3, s3);
  }
  return true;
}

// The gradients of an entity of two or more triangles, entered with
// transmittance T_in: its span walked again from the back, keeping s^j
// exactly; each triangle's t^j_{i-1} the product over the span's covering
// triangles in front of it (no division, so opaque samples are exact).
// Records come from global memory (bit-identical to the staged form).
__device__ void rewalk_entity(const TriCtx &x, const EntSpan &sp, float g0, float g1, float g2,
                              float T_in) {
  float s0 = sp.Bback, s1 = sp.Bback, s2 = sp.Bback, s3 = sp.Bback;
  if (x.ttab && sp.rank_b < (uint32_t)x.ntab) {
    // the span's triangles are the tabled ranks [rank of fpos, rank_b] (every
    // triangle in front of a tabled one is tabled): walks over them alone,
    // with no list reads and no Gaussians to skip
    const int rf = (int)tri_rank(x.tpos, x.ntab, sp.fpos);
    if ((int)sp.rank_b - rf >= 2 && rewalk_linear(x, sp, rf, g0, g1, g2, T_in)) return;
    for (int ri = (int)sp.rank_b; ri >= rf; --ri) {
      const int64_t ti = x.ttab[ri];
      const TriRec &r = x.trec[ti];
      double e[3];
      float o[4];
      if (tri_eval_rec(r, x.Px, x.Py, false, e, o) == 0) continue;
      float cr, cg, cb, a, w[3];
      float4 texel;
      tri_shade_w(RecWords{&r}, e, x.tex, cr, cg, cb, a, w, &texel);
      float t0 = 1.0f, t1 = 1.0f, t2 = 1.0f, t3 = 1.0f;
      for (int rk = rf; rk < ri; ++rk) {
        const TriRec &rr = x.trec[x.ttab[rk]];
        double ek[3];
        float ok[4];
        if (tri_eval_rec(rr, x.Px, x.Py, false, ek, ok) == 0) continue;
        float kr, kg, kb, ak;
        tri_shade_w(RecWords{&rr}, ek, x.tex, kr, kg, kb, ak);
        t0 *= 1.0f - ok[0] * ak; t1 *= 1.0f - ok[1] * ak;
        t2 *= 1.0f - ok[2] * ak; t3 *= 1.0f - ok[3] * ak;
      }
      const float cd = fmaf(cr, g0, fmaf(cg, g1, cb * g2));
      const float v0 = o[0] * t0, v1 = o[1] * t1, v2 = o[2] * t2, v3 = o[3] * t3;
      const float da = T_in * 0.25f * ((v0 * (cd - s0) + v1 * (cd - s1)) + (v2 * (cd - s2) + v3 * (cd - s3)));
      const float vis = T_in * a * 0.25f * ((v0 + v1) + (v2 + v3));
      emit_tri(x, (uint32_t)ri, ti, da, vis, w, texel, g0, g1, g2);
      s0 = fmaf(o[0] * a, cd - s0, s0);
      s1 = fmaf(o[1] * a, cd - s1, s1);
      s2 = fmaf(o[2] * a, cd - s2, s2);
      s3 = fmaf(o[3] * a, cd - s3, s3);
    }
    return;
  }
  uint32_t rank = sp.rank_b;
  for (int pi = sp.bpos; pi >= sp.fpos; --pi) {
    const int64_t ti = tri_at(x, pi);
    if (ti < 0) continue;
    const uint32_t ri_rank = x.tpos ? tri_rank(x.tpos, x.ntab, pi) : rank;
    ++rank;
    const TriRec &ri = x.trec[ti];
    double e[3];
    float o[4];
    if (tri_eval_rec(ri, x.Px, x.Py, false, e, o) == 0) continue;
    float cr, cg, cb, a, w[3];
    float4 texel;
    tri_shade_w(RecWords{&ri}, e, x.tex, cr, cg, cb, a, w, &texel);
    // t^j in front of triangle i within the entity
    float t0 = 1.0f, t1 = 1.0f, t2 = 1.0f, t3 = 1.0f;
    for (int pk = sp.fpos; pk < pi; ++pk) {
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
    const float cd = fmaf(cr, g0, fmaf(cg, g1, cb * g2));
    const float v0 = o[0] * t0, v1 = o[1] * t1, v2 = o[2] * t2, v3 = o[3] * t3;
    const float da = T_in * 0.25f * ((v0 * (cd - s0) + v1 * (cd - s1)) + (v2 * (cd - s2) + v3 * (cd - s3)));
    const float vis = T_in * a * 0.25f * ((v0 + v1) + (v2 + v3));
    emit_tri(x, ri_rank, ti, da, vis, w, texel, g0, g1, g2);
    s0 = fmaf(o[0] * a, cd - s0, s0);
    s1 = fmaf(o[1] * a, cd - s1, s1);
    s2 = fmaf(o[2] * a, cd - s2, s2);
    s3 = fmaf(o[3] * a, cd - s3, s3);
  }
}

// One pixel's bookkeeping of the entity it is in, and the terms of the
// entity's back triangle as if it were alone (t = 1, s^j = B), without the
// factor T_in: what an entity of one triangle (most of them) emits at its
// close with no second walk.
struct PixEnt {
  int fpos, bpos, n_ent;
  uint32_t rank_b, c_t;
  float Bback, c_da, c_vis, c_w0, c_w1, c_w2;
  float4 c_texel;
};

__device__ __forceinline__ void ent_reset(PixEnt &e) {
  e.fpos = e.bpos = e.n_ent = 0;
  e.rank_b = kNoRank;
  e.c_t = 0;
  e.Bback = e.c_da = e.c_vis = e.c_w0 = e.c_w1 = e.c_w2 = 0.f;
  e.c_texel = make_float4(1.f, 1.f, 1.f, 1.f);
}

// A covering triangle at list position pos joins the pixel's entity (open
// says whether one was open before it); Bd is B . g behind it, cd its
// colour . g, n_cov its covered share of the samples.
__device__ __forceinline__ void ent_add(PixEnt &e, bool open, int pos, uint32_t rank, uint32_t t,
                                        float Bd, float cd, float alpha, float n_cov,
                                        const float w[3], float4 texel) {
  if (!open) {
    e.bpos = pos;
    e.Bback = Bd;
    e.n_ent = 0;
    e.rank_b = rank;
  }
  if (++e.n_ent == 1) {
    e.c_t = t;
    e.c_da = n_cov * (cd - Bd);
    e.c_vis = n_cov * alpha;
    e.c_w0 = w[0];
    e.c_w1 = w[1];
    e.c_w2 = w[2];
    e.c_texel = texel;
  }
  e.fpos = pos;
}

__device__ __forceinline__ void ent_close(const TriCtx &x, const PixEnt &e, float g0, float g1,
                                          float g2, float T_in) {
  if (e.n_ent == 1) {
    const float w[3] = {e.c_w0, e.c_w1, e.c_w2};
    emit_tri(x, e.rank_b, e.c_t, T_in * e.c_da, T_in * e.c_vis, w, e.c_texel, g0, g1, g2);
  } else {
    const EntSpan sp = {e.fpos, e.bpos, e.rank_b, e.Bback};
    rewalk_entity(x, sp, g0, g1, g2, T_in);
  }
}

}  // namespace umgs
