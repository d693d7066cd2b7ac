// Tile rows of a projected Gaussian's support, shared by the projection
// (which counts a record's tiles) and the bin stage (which emits them), so
// both derive the same tiles with the same arithmetic.
//
// A Gaussian contributes to a pixel only where alpha = min(0.99, o exp(power))
// >= 1/255 (Eq. 1-2 with the 3DGS cut-off), i.e. where
//   Q(d) = A dx^2 + B dx dy + C dy^2 <= L = ln(255 o),
// with A, B, C the negated FP32 power coefficients of its record -- the very
// numbers the blend evaluates.  The blend evaluates Q in FP32: each term
// carries a few roundings, so |Q_fp32 - Q| <= 1e-6 kappa Q with kappa the
// condition number of the form, and exp and the products move the threshold
// by well under 1e-3.  The support used here is therefore the ellipse
// Q <= tau = (L + 1e-3) / (1 - 1e-6 kappa), evaluated in FP64 with another
// 1e-3 px of slack; a tile is kept if one of its pixel centres lies inside.
// Dropping the other tiles of the bounding rectangle changes no pixel.
// Forms that are degenerate or too ill-conditioned for the bound keep the
// whole rectangle.
#pragma once

#include "internal.h"

namespace umgs {

struct Support {
  double mx, my, A, B, C, D, tau;
  bool exact;   // false: every tile of the rectangle is kept
};

__device__ __forceinline__ Support make_support(const GaussRec &g) {
#pragma clang fp contract(off)
  Support s;
  s.mx = (double)g.mx;
  s.my = (double)g.my;
  s.A = -(double)g.qa;
  s.B = -(double)g.qb;
  s.C = -(double)g.qc;
  s.D = 4.0 * s.A * s.C - s.B * s.B;
  const double L = log(255.0 * (double)g.opacity);
  const double h = sqrt((s.A - s.C) * (s.A - s.C) + s.B * s.B);
  const double lmax = 0.5 * ((s.A + s.C) + h);
  const double lmin = s.D / (4.0 * lmax);          // product of the eigenvalues is D/4
  const double kappa = lmax / lmin;
  s.exact = s.A > 0.0 && s.C > 0.0 && s.D > 0.0 && lmin > 0.0 && kappa < 1e5 && L > 0.0;
  s.tau = (L + 1e-3) / (1.0 - 1e-6 * kappa);
  return s;
}

// Tile columns [a, b) of tile row ty that hold a pixel centre inside the
// support, within the bounding rectangle's columns [tx0, tx1).
__device__ __forceinline__ void support_row(const Support &s, int ty, int tile_w, int tile_h,
                                            int W, int H, int tx0, int tx1, int &a, int &b) {
#pragma clang fp contract(off)
  a = tx0;
  b = tx1;
  if (!s.exact) return;
  const double m = 1e-3;
  // pixel-centre rows of the tile row, relative to the mean
  const double y0 = ((double)(ty * tile_h) + 0.5) - s.my - m;
  const double y1 = ((double)min(ty * tile_h + tile_h, H) - 0.5) - s.my + m;
  const double ey = sqrt(4.0 * s.A * s.tau / s.D);           // half height of the ellipse
  const double lo = fmax(y0, -ey), hi = fmin(y1, ey);
  if (lo > hi) {
    b = a;
    return;
  }
  // the rightmost point of the ellipse lies at dy = -ys, the leftmost at +ys;
  // x at the ends of a chord: (-B dy +- sqrt(4 A tau - D dy^2)) / (2 A)
  const double ys = s.B * sqrt(s.tau / (s.C * s.D));
  const double dr = fmin(fmax(-ys, lo), hi), dl = fmin(fmax(ys, lo), hi);
  const double sr = sqrt(fmax(4.0 * s.A * s.tau - s.D * dr * dr, 0.0));
  const double sl = sqrt(fmax(4.0 * s.A * s.tau - s.D * dl * dl, 0.0));
  const double xmax = s.mx + (-s.B * dr + sr) / (2.0 * s.A) + m;
  const double xmin = s.mx + (-s.B * dl - sl) / (2.0 * s.A) - m;
  // pixel columns px with px + 0.5 in [xmin, xmax], inside the rectangle
  const double plo = (double)(tx0 * tile_w), phi = (double)(min(tx1 * tile_w, W) - 1);
  const double c0 = fmin(fmax(ceil(xmin - 0.5), plo), phi + 1.0);
  const double c1 = fmax(fmin(floor(xmax - 0.5), phi), plo - 1.0);
  if (c0 > c1) {
    b = a;
    return;
  }
  a = (int)c0 / tile_w;
  b = (int)c1 / tile_w + 1;
}

}  // namespace umgs
