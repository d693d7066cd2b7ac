// Tile rows of a projected Gaussian's support: the bin stage cuts every
// entry's supertile to the tiles whose pixel centres the support reaches.
//
// A Gaussian contributes to a pixel only where alpha = min(0.99, o exp(power))
// >= 1/255 (Eq. 1-2 with the 3DGS cut-off), i.e. where
//   Q(d) = A dx^2 + B dx dy + C dy^2 <= L = log2(o) + log2(255),
// with A, B, C the negated FP32 power coefficients of its record (stored times
// log2(e), next to log2(o)) -- the very numbers the blend evaluates.  The blend evaluates Q in FP32: each term
// carries a few roundings, so |Q_fp32 - Q| <= 1e-6 kappa Q with kappa the
// condition number of the form, and exp2 moves the threshold by well under
// 1e-3.  The support used here is the ellipse
//   Q <= tau = (L + 1e-3) (1 + 1e-4) / (1 - 1e-6 kappa),
// whose chords are evaluated in FP32 with the hardware square root and
// reciprocal (1 ulp; D = 4AC - B^2 in FP64, then rounded) and widened by
// 0.02 px plus 2e-3 of the ellipse's extent, which covers the FP32 error of
// the chord ends (at most a few 1e-4 of the extent, where the square root's
// argument cancels).  A tile is kept if one of its pixel
// centres lies inside; dropping the other tiles of the bounding rectangle
// changes no pixel.  Forms that are degenerate or too ill-conditioned for
// the bound keep the whole rectangle.
#pragma once

#include "internal.h"

namespace umgs {

struct Support {
  float mx, my, A, B, C, D, tau, ex, ey, m;   // ex, ey: half extents; m: chord slack
  float ys, i2A, fat;                         // B sqrt(tau / (C D)), 1 / (2A), 4 A tau
  bool exact;                                 // false: every tile of the rectangle is kept
};

__device__ __forceinline__ Support make_support(const GaussRec &g) {
#pragma clang fp contract(off)
  Support s;
  s.mx = g.mx;
  s.my = g.my;
  s.A = -g.qa;
  s.B = -g.qb;
  s.C = -g.qc;
  const double Dd = 4.0 * (double)s.A * (double)s.C - (double)s.B * (double)s.B;
  s.D = (float)Dd;
  const float L = g.lo + kLog2_255;
  const float h = __builtin_amdgcn_sqrtf((s.A - s.C) * (s.A - s.C) + s.B * s.B);
  const float lmax = 0.5f * ((s.A + s.C) + h);
  const float lmin = s.D * __builtin_amdgcn_rcpf(4.0f * lmax);   // eigenvalue product is D/4
  const float kappa = lmax * __builtin_amdgcn_rcpf(lmin);
  s.exact = s.A > 0.0f && s.C > 0.0f && s.D > 0.0f && lmin > 0.0f && kappa < 1e5f && L > 0.0f;
  s.tau = ((L + 1e-3f) * 1.0001f) * __builtin_amdgcn_rcpf(1.0f - 1e-6f * kappa);
  const float iD = __builtin_amdgcn_rcpf(s.D);
  s.ey = __builtin_amdgcn_sqrtf(4.0f * s.A * s.tau * iD);
  s.ex = __builtin_amdgcn_sqrtf(4.0f * s.C * s.tau * iD);
  s.m = 0.02f + 2e-3f * (s.ex + s.ey);
  // per-row constants: the rightmost point of the ellipse lies at dy = -ys,
  // the leftmost at +ys
  s.ys = s.B * __builtin_amdgcn_sqrtf(s.tau * __builtin_amdgcn_rcpf(s.C * s.D));
  s.i2A = __builtin_amdgcn_rcpf(2.0f * s.A);
  s.fat = 4.0f * s.A * s.tau;
  return s;
}

// Tile columns [a, b) of tile row ty that hold a pixel centre inside the
// support, within the pixel columns [plo, phi] of the bounding rectangle's
// tile columns [tx0, tx1).  Tiles are 2^lw x 2^lh pixels.
__device__ __forceinline__ void support_row(const Support &s, int ty, int lw, int lh, int H,
                                            int tx0, int tx1, float plo, float phi, int &a,
                                            int &b) {
#pragma clang fp contract(off)
  a = tx0;
  b = tx1;
  if (!s.exact) return;
  // pixel-centre rows of the tile row, relative to the mean
  const float y0 = ((float)(ty << lh) + 0.5f) - s.my - s.m;
  const float y1 = ((float)min((ty + 1) << lh, H) - 0.5f) - s.my + s.m;
  const float lo = fmaxf(y0, -s.ey), hi = fminf(y1, s.ey);
  if (lo > hi) {
    b = a;
    return;
  }
  // x at the ends of a chord: (-B dy +- sqrt(4 A tau - D dy^2)) / (2 A)
  const float dr = fminf(fmaxf(-s.ys, lo), hi), dl = fminf(fmaxf(s.ys, lo), hi);
  const float sr = __builtin_amdgcn_sqrtf(fmaxf(s.fat - s.D * dr * dr, 0.0f));
  const float sl = __builtin_amdgcn_sqrtf(fmaxf(s.fat - s.D * dl * dl, 0.0f));
  const float xmax = s.mx + (-s.B * dr + sr) * s.i2A + s.m;
  const float xmin = s.mx + (-s.B * dl - sl) * s.i2A - s.m;
  // pixel columns px with px + 0.5 in [xmin, xmax], inside the rectangle
  const float c0 = fminf(fmaxf(ceilf(xmin - 0.5f), plo), phi + 1.0f);
  const float c1 = fmaxf(fminf(floorf(xmax - 0.5f), phi), plo - 1.0f);
  if (c0 > c1) {
    b = a;
    return;
  }
  a = (int)c0 >> lw;
  b = ((int)c1 >> lw) + 1;
}

// Tiles of supertile (sx, sy) that the record reaches, as the 64 bits
// (ty - sy kST) kST + (tx - sx kST): the support rows, cut to the
// supertile's columns.
__device__ __forceinline__ uint64_t st_mask(const Support &s, int sx, int sy, int tx0, int ty0,
                                            int tx1, int ty1, int lw, int lh, int W, int H) {
  const int c0 = sx << kSTLog, y0 = sy << kSTLog;
  const int r0 = max(ty0, y0), r1 = min(ty1, y0 + kST);
  const float plo = (float)(tx0 << lw), phi = (float)(min(tx1 << lw, W) - 1);
  uint64_t m = 0;
  for (int ty = r0; ty < r1; ++ty) {
    int a, b;
    support_row(s, ty, lw, lh, H, tx0, tx1, plo, phi, a, b);
    const int l = max(a, c0), h = min(b, c0 + kST);
    if (l < h) m |= ((1ull << (h - l)) - 1ull) << ((l - c0) + ((ty - y0) << kSTLog));
  }
  return m;
}

}  // namespace umgs
