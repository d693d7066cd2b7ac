// Backward pass of the single-pass rasterizer.
//
// blend_backward_kernel: one wave per tile (tiles launched in decreasing
// order of their walk length), four pixels per lane, walking the tile's
// sorted list from the pixels' last blended fragment back to the front.
// Every unit (a Gaussian, or a whole triangle entity)
// acts on the pixel as C += T_before x contribution, T_after = T_before x m,
// so going backwards the pixel keeps
//   B  -- the colour behind the current unit, normalised by the
//         transmittance in front of it (starts at the background);
//   T  -- the transmittance in front of the current unit, recovered as
//         T / (1 - alpha) for a Gaussian and T / tau for an entity, except
//         for the last blended unit, whose front transmittance the forward
//         stored (it may be opaque).
// Gaussian k: dC/dc = T a, dC/da = T (c - B); then B = a c + (1 - a) B.
// Triangle entity (Eq. 7-9), per sub-sample j in reverse:
//   s^j = o^j a c + (1 - o^j a) s^j   (starting from B),
//   p^j = (1 - o^j a) p^j             (starting from 1),
// and when the entity closes B = mean_j s^j, tau = mean_j p^j.  Colours
// enter only through their dot product with the pixel's dL/dC, so B and the
// s^j are carried as such scalars.  Triangles are fixed occluders: they
// pass gradients through T but receive none.
// Per fragment the 9 gradient terms (mean 2D, the 3 power coefficients,
// opacity, colour) are summed over the lane's pixels, then over the wave
// (a transposing DPP reduction that leaves the totals in four lanes), and
// added once per tile with three float-atomic instructions.
//
// project_backward_kernel: one thread per Gaussian, looping over views:
// the chain rule back through the conic inverse, the EWA Jacobian (with the
// frustum clamp), the pinhole projection, the SH colour and its view
// direction, Sigma' = A Sigma A^T (when deformed) and Sigma = R S S R^T.
#include "blend_common.h"

#include <algorithm>

namespace umgs {

namespace {

// Backward state of one pixel while its list is walked from the back.
// Everything the gradients need of a colour is its dot product with the
// pixel's dL/dC (all of it is linear in colours), so the colour behind the
// current unit is carried as that scalar: Bd = B . dL/dC, and inside a
// triangle entity one such scalar per sub-sample.  ent is +inf outside an
// entity; inside one it holds the transmittance behind the entity (T_in
// tau), or -1 for the pixel's last blended unit, whose front transmittance
// the forward stored.  Each triangle of an entity leaves Bd and Tr as they
// are in front of the entity so far, so a Gaussian in front of it closes
// the entity by just clearing ent.
struct PixBwd {
  float Tr, Tterm, dC0, dC1, dC2, Bd, ent;
  int last;
  float sd0, sd1, sd2, sd3;
  float p0, p1, p2, p3;
};

// One Gaussian fragment (list position pos) of the walk: updates the
// pixel's state where it blended the fragment and leaves the pixel's 9
// gradient terms in g (exact zeros where it did not), in the reduced form
// that the wave sums: (dp dx, dp dy, dp dx^2, dp dx dy, dp dy^2, a dpow,
// w dC); add_sums9 turns the sums into the gradients of the mean and
// opacity with the fragment's constants, once per wave instead of per
// pixel.  Returns whether it blended it.  Every lane evaluates every term
// (no branches), so the wave sums that follow see defined values on all
// lanes.
// A staged Gaussian's constants, read from LDS once per fragment for all
// of a lane's pixels.
struct GFrag {
  float4 a;     // mean x, mean y, qa, qb
  float2 b;     // qc, log2(o)
  float c0, c1, c2;
};

__device__ __forceinline__ GFrag load_gfrag(const uint32_t *s) {
  GFrag f;
  f.a = *(const float4 *)(s + 0);
  f.b = *(const float2 *)(s + 4);
  f.c0 = __uint_as_float(s[6]);
  f.c1 = __uint_as_float(s[7]);
  f.c2 = __uint_as_float(s[8]);
  return f;
}

__device__ __forceinline__ bool gauss_bwd(const GFrag &fr, int pos, float pcx, float pcy,
                                          PixBwd &q, float *g) {
  // alpha and the decision exactly as gauss_terms takes them
  float dx = fr.a.x - pcx;
  float dy = fr.a.y - pcy;
  const float pw = gauss_logalpha(fr.a.z, fr.a.w, fr.b.x, fr.b.y, dx, dy);
  const bool inside = pw <= fr.b.y;
  const float a_un = __builtin_amdgcn_exp2f(inside ? pw : fr.b.y);
  // min(0.99, a) as a select on the compare the clamp's gradient also takes
  // (the same value as fminf for every a, NaN included)
  const float alpha = a_un < kAlphaMax ? a_un : kAlphaMax;
  const bool hit = inside && alpha >= kAlphaMin;
  const bool contrib = pos < q.last && hit;
  q.ent = contrib ? __builtin_inff() : q.ent;     // a blended Gaussian closes an entity
  // T in front of the fragment: one rcp (1 ulp) per step of the walk
  const float Tb = (pos == q.last - 1) ? q.Tterm : q.Tr * __builtin_amdgcn_rcpf(1.0f - alpha);
  const float cd = fmaf(fr.c0, q.dC0, fmaf(fr.c1, q.dC1, fr.c2 * q.dC2));
  const float diff = cd - q.Bd;             // (c - B) . dL/dC
  // where the pixel does not blend it every term is an exact zero (all
  // factors are finite) and the state is left as it is
  const float ac = contrib ? alpha : 0.0f;
  const float w = Tb * ac;
  q.Bd = fmaf(ac, diff, q.Bd);
  q.Tr = contrib ? Tb : q.Tr;
  // alpha below the 0.99 clamp depends on power and opacity
  const float dpow = (contrib && a_un < kAlphaMax) ? Tb * diff : 0.0f;
  const float dp = alpha * dpow;     // d alpha / d power = o exp(power) = alpha
  const float dpx = dp * dx, dpy = dp * dy;
  g[0] = dpx;
  g[1] = dpy;
  g[2] = dpx * dx;
  g[3] = dpx * dy;
  g[4] = dpy * dy;
  g[5] = a_un * dpow;                // times 1/o: d alpha / d o = exp(power)
  g[6] = w * q.dC0;
  g[7] = w * q.dC1;
  g[8] = w * q.dC2;
  return contrib;
}

// Wave sums of a fragment's 9 reduced terms, left spread over the lanes
// by their two lowest bits (every lane holds the totals of its group):
//   lane & 3 == 0: terms 0, 1, 2;  1: terms 5, 6, 7;  2: terms 3, 4;  3: term 8.
// The first two steps transpose as they add: partners L and L ^ 1 each keep
// one half of the terms, summed (5 values left), then L and L ^ 2 (3 left);
// lanes with the same two low bits then hold the same terms, summed with
// row rotations by 4 and 8 and across the rows with lane permutes.  That is
// 36 additions and selects per lane instead of 54 for nine full sums, and
// the totals end in four lanes, so three atomic instructions add them.
template <int CTRL>
__device__ __forceinline__ float dpp_src(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}

__device__ __forceinline__ void wave_sums9(const float (&v)[9], float (&t)[3], bool b0, bool b1) {
  float a[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const float hi = i < 4 ? v[5 + i] : 0.0f;
    const float keep = b0 ? hi : v[i];
    const float send = b0 ? v[i] : hi;
    a[i] = keep + dpp_src<0xB1>(send);           // quad_perm [1,0,3,2]: lane ^ 1
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float hi = i < 2 ? a[3 + i] : 0.0f;
    const float keep = b1 ? hi : a[i];
    const float send = b1 ? a[i] : hi;
    t[i] = keep + dpp_src<0x4E>(send);           // quad_perm [2,3,0,1]: lane ^ 2
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) t[i] += dpp_src<0x124>(t[i]);   // row_ror:4
#pragma unroll
  for (int i = 0; i < 3; ++i) t[i] += dpp_src<0x128>(t[i]);   // row_ror:8
#pragma unroll
  for (int i = 0; i < 3; ++i) t[i] += __shfl_xor(t[i], 16, 64);
#pragma unroll
  for (int i = 0; i < 3; ++i) t[i] += __shfl_xor(t[i], 32, 64);
}

// The wave totals of wave_sums9 added to the fragment's 2D gradients by
// lanes 0..3 (three atomic instructions), the mean and opacity terms first
// turned into gradients with the fragment's constants (the stored power
// coefficients carry log2(e)): d/dmean = ln2 (2 qa S_dx + qb S_dy,
// qb S_dx + 2 qc S_dy), d/do = S_a / o.
__device__ __forceinline__ void add_sums9(const uint32_t *s, const float (&t)[3], int lane,
                                          float *__restrict__ g2d) {
  if (lane < 4) {
    float *dst = g2d + 9 * (int64_t)s[kSlotRec];
    float x0 = t[0], x1 = t[1];
    int o0, o1, o2;
    if (lane == 0) {
      const float qa = __uint_as_float(s[2]), qb = __uint_as_float(s[3]),
                  qc = __uint_as_float(s[4]);
      x0 = kLn2 * (2.0f * qa * t[0] + qb * t[1]);
      x1 = kLn2 * (qb * t[0] + 2.0f * qc * t[1]);
    }
    if (lane == 1) x0 = t[0] * __uint_as_float(s[kSlotInvO]);
    o0 = lane == 0 ? 0 : lane == 1 ? 5 : lane == 2 ? 3 : 8;
    o1 = lane == 0 ? 1 : lane == 1 ? 6 : 4;
    o2 = lane == 0 ? 2 : 7;
    unsafeAtomicAdd(dst + o0, x0);
    if (lane < 3) unsafeAtomicAdd(dst + o1, x1);
    if (lane < 2) unsafeAtomicAdd(dst + o2, t[2]);
  }
}

// Triangle fragment of the walk for one pixel (a fixed occluder: it passes
// gradients through T and receives none).
__device__ __forceinline__ void tri_bwd(const uint32_t *s, int pos, double rlx, double rly,
                                        bool direct, const TexView &tex, PixBwd &q) {
  double e[3];
  float o[4];
  if (!(pos < q.last && tri_eval(s, rlx, rly, direct, e, o) > 0)) return;
  float cr, cg, cbl, alpha;
  tri_shade(s, e, tex, cr, cg, cbl, alpha);
  const float cd = fmaf(cr, q.dC0, fmaf(cg, q.dC1, cbl * q.dC2));
  if (direct) {
    q.Tr = (pos == q.last - 1) ? q.Tterm : q.Tr / (1.0f - alpha);
    q.Bd = fmaf(alpha, cd - q.Bd, q.Bd);
    return;
  }
  if (q.ent == __builtin_inff()) {
    // the walk enters an entity at its last triangle
    q.ent = (pos == q.last - 1) ? -1.0f : q.Tr;
    q.sd0 = q.sd1 = q.sd2 = q.sd3 = q.Bd;
    q.p0 = q.p1 = q.p2 = q.p3 = 1.0f;
  }
  const float a0 = o[0] * alpha, a1 = o[1] * alpha, a2 = o[2] * alpha, a3 = o[3] * alpha;
  q.sd0 = fmaf(a0, cd - q.sd0, q.sd0);
  q.sd1 = fmaf(a1, cd - q.sd1, q.sd1);
  q.sd2 = fmaf(a2, cd - q.sd2, q.sd2);
  q.sd3 = fmaf(a3, cd - q.sd3, q.sd3);
  q.p0 *= 1.0f - a0; q.p1 *= 1.0f - a1; q.p2 *= 1.0f - a2; q.p3 *= 1.0f - a3;
  // in front of the entity so far: colour behind B = mean_j s^j, T_in = T / tau
  q.Bd = 0.25f * ((q.sd0 + q.sd1) + (q.sd2 + q.sd3));
  q.Tr = q.ent < 0.0f ? q.Tterm : q.ent / (0.25f * ((q.p0 + q.p1) + (q.p2 + q.p3)));
}

// ---- heaviest-first tile order -------------------------------------------
// A tile's backward walks its list down from the largest last-blended
// position of its pixels, one wave per tile, so that position is the
// tile's critical path.  Tiles are launched in decreasing order of it
// (buckets of a quarter octave), so the longest walks start first and the
// short ones fill in behind them instead of leaving the long ones to run
// last.
constexpr int kBwdBuckets = 128;
// parts per 256-pixel tile (1: four pixels per lane; 2: two)
constexpr int kBwdSplit16 = 1;

__device__ __forceinline__ int walk_bucket(uint32_t k) {
  if (k < 4) return (int)k;
  const int e = 31 - __clz(k);                     // >= 2
  return min(kBwdBuckets - 1, 4 * (e - 1) + (int)((k >> (e - 2)) & 3u));
}

// key[tile] = the largest last-blended position of its pixels (clamped to
// its list, as the walk clamps it), or 0 where mask (if given) is 0; one
// wave per tile.
template <int TW, int TH>
__global__ __launch_bounds__(64) void walk_key_kernel(const ViewParams *__restrict__ views, int V,
                                                     const uint2 *__restrict__ ranges,
                                                     const int32_t *__restrict__ ncontrib,
                                                     const uint32_t *__restrict__ mask,
                                                     uint32_t *__restrict__ key) {
  const uint32_t tile = blockIdx.x;
  if (mask && mask[tile] == 0u) {
    if (threadIdx.x == 0) key[tile] = 0u;
    return;
  }
  const int v = find_view(views, V, tile);
  const ViewParams &vp = views[v];
  const uint32_t lt = tile - vp.tile_base;
  const int tx = (int)(lt % (uint32_t)vp.ntx), ty = (int)(lt / (uint32_t)vp.ntx);
  const uint2 rg = ranges[tile];
  const int count = (int)(rg.y - rg.x);
  int m = 0;
  for (int i = threadIdx.x; i < TW * TH; i += 64) {
    const int px = tx * TW + i % TW, py = ty * TH + i / TW;
    if (px < vp.W && py < vp.H)
      m = max(m, min(max(ncontrib[vp.pix_base + (int64_t)py * vp.W + px], 0), count));
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
  if (threadIdx.x == 0) key[tile] = (uint32_t)m;
}

__global__ void walk_count_kernel(const uint32_t *__restrict__ key, uint32_t n,
                                  uint32_t *__restrict__ cnt) {
  __shared__ uint32_t h[kBwdBuckets];
  if (threadIdx.x < kBwdBuckets) h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) atomicAdd(&h[walk_bucket(key[t])], 1u);
  __syncthreads();
  if (threadIdx.x < kBwdBuckets && h[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], h[threadIdx.x]);
}

// cursors in descending bucket order (heaviest first); one wave
__global__ void walk_scan_kernel(uint32_t *__restrict__ cnt) {
  if (threadIdx.x != 0) return;
  uint32_t run = 0;
  for (int b = kBwdBuckets - 1; b >= 0; --b) {
    const uint32_t c = cnt[b];
    cnt[b] = run;
    run += c;
  }
}

__global__ void walk_scatter_kernel(const uint32_t *__restrict__ key, uint32_t n,
                                    uint32_t *__restrict__ cursor, uint32_t *__restrict__ order) {
  __shared__ uint32_t h[kBwdBuckets], base[kBwdBuckets];
  if (threadIdx.x < kBwdBuckets) h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  int b = 0;
  uint32_t local = 0;
  if (t < n) {
    b = walk_bucket(key[t]);
    local = atomicAdd(&h[b], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kBwdBuckets && h[threadIdx.x])
    base[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], h[threadIdx.x]);
  __syncthreads();
  if (t < n) order[base[b] + local] = t;
}

// One workgroup of one wave per part of a tile (tiles taken heaviest
// first, each split into SPLIT parts of TH / SPLIT rows); each lane walks
// PPT pixels of its part (rows ly, ly + R, ... with R = TH / SPLIT / PPT),
// so one set of wave sums serves all of a part's pixels and no sums cross
// waves.
template <int TW, int TH, int SPLIT>
__global__ __launch_bounds__(64) void blend_backward_kernel(
    const uint32_t *__restrict__ order,
    const ViewParams *__restrict__ views, int V, int N, int T, int mode, int batch,
    float bg0, float bg1, float bg2, const uint2 *__restrict__ ranges,
    const uint32_t *__restrict__ v0, const uint32_t *__restrict__ v1,
    const FrameInfo *__restrict__ fi, const GaussRec *__restrict__ grec,
    const TriRec *__restrict__ trec, const TexView tex, const float *__restrict__ dLdimg,
    const float *__restrict__ Tfin, const int32_t *__restrict__ ncontrib,
    const float *__restrict__ Tent, float *__restrict__ g2d) {
  constexpr int ROWS = TH / SPLIT;                        // rows of a part
  constexpr int PPT = TW * ROWS / 64;                     // pixels per lane
  constexpr int RSTEP = ROWS / PPT;                       // row step of a lane's pixels
  static_assert(TW * ROWS == 64 * PPT && ROWS % PPT == 0, "one wave per part");
  extern __shared__ uint32_t slots[];                     // batch * kSlotWords
  const uint32_t *vals = fi->sorted_in ? v1 : v0;

  const uint32_t tile = order[blockIdx.x / SPLIT];
  const int part = (int)(blockIdx.x % SPLIT);
  const int v = find_view(views, V, tile);
  const ViewParams &vp = views[v];
  const uint32_t lt = tile - vp.tile_base;
  const int tx = (int)(lt % (uint32_t)vp.ntx), ty = (int)(lt / (uint32_t)vp.ntx);
  const int lane = threadIdx.x;
  const int lx = lane % TW, ly0 = part * ROWS + lane / TW;
  const int px = tx * TW + lx;
  const float pcx = (float)px + 0.5f;
  const int64_t P0x = (int64_t)(tx * TW) * kSubpx + kSubpx / 2;
  const int64_t P0y = (int64_t)(ty * TH) * kSubpx + kSubpx / 2;
  const double rlx = (double)(lx * kSubpx);
  const bool direct = mode == UMGS_MODE_DIRECT;
  const uint2 rg = ranges[tile];
  const int64_t rbase = (int64_t)v * (N + T);
  const int64_t HW = (int64_t)vp.W * vp.H;
  const int count = (int)(rg.y - rg.x);

  PixBwd q[PPT];
  int my_last = 0;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const int ly = ly0 + p * RSTEP;
    const int py = ty * TH + ly;
    q[p].last = 0;
    q[p].Tr = 1.0f; q[p].Tterm = 1.0f; q[p].dC0 = 0.f; q[p].dC1 = 0.f; q[p].dC2 = 0.f;
    if (px < vp.W && py < vp.H) {
      const int64_t pix = (int64_t)py * vp.W + px;
      // positions are 1-based within this tile's list; clamp so a per-pixel
      // array from another frame can never index past the tile's range
      q[p].last = min(max(ncontrib[vp.pix_base + pix], 0), count);
      q[p].Tr = Tfin[vp.pix_base + pix];
      q[p].Tterm = Tent[vp.pix_base + pix];
      const float *d = dLdimg + 3 * vp.pix_base;
      q[p].dC0 = d[pix];
      q[p].dC1 = d[HW + pix];
      q[p].dC2 = d[2 * HW + pix];
    }
    q[p].Bd = fmaf(bg0, q[p].dC0, fmaf(bg1, q[p].dC1, bg2 * q[p].dC2));
    q[p].ent = __builtin_inff();
    q[p].sd0 = q[p].sd1 = q[p].sd2 = q[p].sd3 = 0.f;
    q[p].p0 = q[p].p1 = q[p].p2 = q[p].p3 = 1.f;
    my_last = max(my_last, q[p].last);
  }
  int max_last = my_last;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) max_last = max(max_last, __shfl_xor(max_last, o, 64));

  for (int bend = max_last; bend > 0; bend -= batch) {
    const int bstart = max(0, bend - batch);
    const int bn = bend - bstart;
    // lane f stages fragment f (batch <= 64); bit f of tri_bits marks a triangle
    bool is_tri = false;
    if (lane < bn) {
      uint32_t *s = slots + lane * kSlotWords;
      const int64_t local = (int64_t)vals[rg.x + bstart + lane] - rbase;
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
    const uint64_t tri_bits = __ballot(is_tri);
    __syncthreads();
    for (int f = bn - 1; f >= 0; --f) {
      const uint32_t *s = slots + f * kSlotWords;
      const int pos = bstart + f;
      if (!__any(pos < my_last)) continue;
      if (((tri_bits >> f) & 1u) == 0u) {
        const GFrag fr = load_gfrag(s);
        float g[9];
        bool c = false;
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          const float pcy = (float)(ty * TH + ly0 + p * RSTEP) + 0.5f;
          float h[9];
          c |= gauss_bwd(fr, pos, pcx, pcy, q[p], h);
#pragma unroll
          for (int k = 0; k < 9; ++k) g[k] = p == 0 ? h[k] : g[k] + h[k];
        }
        if (!__any(c)) continue;     // no lane of the wave blends it
        float t[3];
        wave_sums9(g, t, (lane & 1) != 0, (lane & 2) != 0);
        add_sums9(s, t, lane, g2d);
      } else {
#pragma unroll
        for (int p = 0; p < PPT; ++p)
          // only pixels in the triangle's box can have a covered sample
          if (in_tile_box(s[38], lx, ly0 + p * RSTEP))
            tri_bwd(s, pos, rlx, (double)((ly0 + p * RSTEP) * kSubpx), direct, tex, q[p]);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------

__device__ __forceinline__ float view_row_c(const float *Rr, float t, float x, float y, float z) {
#pragma clang fp contract(off)
  return ((Rr[0] * x + Rr[1] * y) + Rr[2] * z) + t;
}

// Real SH basis values and gradients (w.r.t. the direction components) for
// degree DEG <= 3, same sign convention as the forward.
template <int DEG>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, float *Bv, float *Bx,
                                              float *By, float *Bz) {
  const float C0 = 0.28209479177387814f, C1 = 0.4886025119029199f;
  Bv[0] = C0; Bx[0] = By[0] = Bz[0] = 0.f;
  if constexpr (DEG < 1) return;
  Bv[1] = -C1 * y; Bx[1] = 0.f; By[1] = -C1; Bz[1] = 0.f;
  Bv[2] = C1 * z; Bx[2] = 0.f; By[2] = 0.f; Bz[2] = C1;
  Bv[3] = -C1 * x; Bx[3] = -C1; By[3] = 0.f; Bz[3] = 0.f;
  if constexpr (DEG < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  const float a0 = 1.0925484305920792f, a1 = -1.0925484305920792f, a2 = 0.31539156525252005f,
              a3 = -1.0925484305920792f, a4 = 0.5462742152960396f;
  Bv[4] = a0 * x * y; Bx[4] = a0 * y; By[4] = a0 * x; Bz[4] = 0.f;
  Bv[5] = a1 * y * z; Bx[5] = 0.f; By[5] = a1 * z; Bz[5] = a1 * y;
  Bv[6] = a2 * (2.f * zz - xx - yy); Bx[6] = -2.f * a2 * x; By[6] = -2.f * a2 * y; Bz[6] = 4.f * a2 * z;
  Bv[7] = a3 * x * z; Bx[7] = a3 * z; By[7] = 0.f; Bz[7] = a3 * x;
  Bv[8] = a4 * (xx - yy); Bx[8] = 2.f * a4 * x; By[8] = -2.f * a4 * y; Bz[8] = 0.f;
  if constexpr (DEG < 3) return;
  const float b0 = -0.5900435899266435f, b1 = 2.890611442640554f, b2 = -0.4570457994644658f,
              b3 = 0.3731763325901154f, b4 = -0.4570457994644658f, b5 = 1.445305721320277f,
              b6 = -0.5900435899266435f;
  Bv[9] = b0 * y * (3.f * xx - yy); Bx[9] = b0 * 6.f * x * y; By[9] = b0 * (3.f * xx - 3.f * yy); Bz[9] = 0.f;
  Bv[10] = b1 * x * y * z; Bx[10] = b1 * y * z; By[10] = b1 * x * z; Bz[10] = b1 * x * y;
  Bv[11] = b2 * y * (4.f * zz - xx - yy); Bx[11] = b2 * (-2.f * x * y);
  By[11] = b2 * (4.f * zz - xx - 3.f * yy); Bz[11] = b2 * 8.f * y * z;
  Bv[12] = b3 * z * (2.f * zz - 3.f * xx - 3.f * yy); Bx[12] = b3 * (-6.f * x * z);
  By[12] = b3 * (-6.f * y * z); Bz[12] = b3 * (6.f * zz - 3.f * xx - 3.f * yy);
  Bv[13] = b4 * x * (4.f * zz - xx - yy); Bx[13] = b4 * (4.f * zz - 3.f * xx - yy);
  By[13] = b4 * (-2.f * x * y); Bz[13] = b4 * 8.f * x * z;
  Bv[14] = b5 * z * (xx - yy); Bx[14] = b5 * 2.f * x * z; By[14] = b5 * (-2.f * y * z); Bz[14] = b5 * (xx - yy);
  Bv[15] = b6 * x * (xx - 3.f * yy); Bx[15] = b6 * (3.f * xx - 3.f * yy); By[15] = b6 * (-6.f * x * y); Bz[15] = 0.f;
}

// One instantiation per SH degree, so the coefficient loops are unrolled and
// the per-coefficient sums stay in registers.
template <int DEG>
__global__ __launch_bounds__(128) void project_backward_kernel(
                                        const ViewParams *__restrict__ views, int V, int N,
                                        const float *__restrict__ means,
                                        const float *__restrict__ scales,
                                        const float *__restrict__ quats,
                                        const float *__restrict__ xform,
                                        const float *__restrict__ sh,
                                        const float *__restrict__ g2d,
                                        float *__restrict__ d_means, float *__restrict__ d_scales,
                                        float *__restrict__ d_quats, float *__restrict__ d_opac,
                                        float *__restrict__ d_sh, float *__restrict__ d_xform,
                                        int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  constexpr int nc = (DEG + 1) * (DEG + 1);
  const float mx_w = means[3 * i], my_w = means[3 * i + 1], mz_w = means[3 * i + 2];
  // Sigma = M M^T, M = R(q) diag(s); deformed: Sigma' = A Sigma A^T
  float qw = quats[4 * i], qx = quats[4 * i + 1], qy = quats[4 * i + 2], qz = quats[4 * i + 3];
  const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  const float iq = 1.0f / qn;
  qw *= iq; qx *= iq; qy *= iq; qz *= iq;
  const float Rq[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                       2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                       2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
  const float sc[3] = {scales[3 * i], scales[3 * i + 1], scales[3 * i + 2]};
  float M[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * sc[c];
  float Sg[9];   // Sigma (full 3x3)
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) Sg[3 * r + c] = M[3 * r] * M[3 * c] + M[3 * r + 1] * M[3 * c + 1] + M[3 * r + 2] * M[3 * c + 2];
  float A[9];
  float Sp[9];   // Sigma' used by the projection
  if (xform) {
#pragma unroll
    for (int k = 0; k < 9; ++k) A[k] = xform[9 * (int64_t)i + k];
    float AS[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) AS[3 * r + c] = A[3 * r] * Sg[c] + A[3 * r + 1] * Sg[3 + c] + A[3 * r + 2] * Sg[6 + c];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) Sp[3 * r + c] = AS[3 * r] * A[3 * c] + AS[3 * r + 1] * A[3 * c + 1] + AS[3 * r + 2] * A[3 * c + 2];
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) Sp[k] = Sg[k];
  }

  float dmu[3] = {0.f, 0.f, 0.f};
  float dSp[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float dop = 0.f;
  float dshv[nc * 3];
#pragma unroll
  for (int k = 0; k < nc * 3; ++k) dshv[k] = 0.f;
  const float *shi = sh + (int64_t)i * nc * 3;

  for (int v = 0; v < V; ++v) {
    const float *g = g2d + 9 * ((int64_t)v * N + i);
    float gg[9];
    bool any = false;
#pragma unroll
    for (int k = 0; k < 9; ++k) { gg[k] = g[k]; any = any || gg[k] != 0.0f; }
    if (!any) continue;
    const ViewParams &vp = views[v];
    const float *W = vp.R;
    const float x = view_row_c(W, vp.t[0], mx_w, my_w, mz_w);
    const float y = view_row_c(W + 3, vp.t[1], mx_w, my_w, mz_w);
    const float z = view_row_c(W + 6, vp.t[2], mx_w, my_w, mz_w);
    const float iz = 1.0f / z, iz2 = iz * iz;
    const float limx = kFrustumClamp * vp.tanx, limy = kFrustumClamp * vp.tany;
    const float xz = x * iz, yz = y * iz;
    const bool clx = xz < -limx || xz > limx, cly = yz < -limy || yz > limy;
    const float txz = fminf(limx, fmaxf(-limx, xz)), tyz = fminf(limy, fmaxf(-limy, yz));
    const float J00 = vp.fx * iz, J02 = -vp.fx * txz * iz, J11 = vp.fy * iz, J12 = -vp.fy * tyz * iz;
    float Tm[6];   // T = J W (2x3)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Tm[k] = J00 * W[k] + J02 * W[6 + k];
      Tm[3 + k] = J11 * W[3 + k] + J12 * W[6 + k];
    }
    float TS[6];   // T Sigma'
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) TS[3 * r + c] = Tm[3 * r] * Sp[c] + Tm[3 * r + 1] * Sp[3 + c] + Tm[3 * r + 2] * Sp[6 + c];
    const float a = TS[0] * Tm[0] + TS[1] * Tm[1] + TS[2] * Tm[2] + kDilation;
    const float b = TS[0] * Tm[3] + TS[1] * Tm[4] + TS[2] * Tm[5];
    const float c = TS[3] * Tm[3] + TS[4] * Tm[4] + TS[5] * Tm[5] + kDilation;
    const float idet = 1.0f / (a * c - b * b);
    const float KA = c * idet, KB = -b * idet, KC = a * idet;   // conic
    // dL/dconic (the power coefficients are -A/2, -B, -C/2)
    const float gA = -0.5f * gg[2], gB = -gg[3], gC = -0.5f * gg[4];
    // S = -K G K with G = [[gA, gB/2], [gB/2, gC]]
    const float G01 = 0.5f * gB;
    const float KG00 = KA * gA + KB * G01, KG01 = KA * G01 + KB * gC;
    const float KG10 = KB * gA + KC * G01, KG11 = KB * G01 + KC * gC;
    const float S00 = -(KG00 * KA + KG01 * KB);
    const float S01 = -(KG00 * KB + KG01 * KC);
    const float S11 = -(KG10 * KB + KG11 * KC);
    // dL/dSigma' += T^T S T
    float ST[6];   // S T (2x3)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ST[k] = S00 * Tm[k] + S01 * Tm[3 + k];
      ST[3 + k] = S01 * Tm[k] + S11 * Tm[3 + k];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) dSp[3 * r + cc] += Tm[r] * ST[cc] + Tm[3 + r] * ST[3 + cc];
    // dL/dT = 2 S T Sigma'
    float dT[6];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
        dT[3 * r + cc] = 2.0f * (ST[3 * r] * Sp[cc] + ST[3 * r + 1] * Sp[3 + cc] + ST[3 * r + 2] * Sp[6 + cc]);
    // dL/dJ = dL/dT W^T (only the non-constant entries)
    const float dJ00 = dT[0] * W[0] + dT[1] * W[1] + dT[2] * W[2];
    const float dJ02 = dT[0] * W[6] + dT[1] * W[7] + dT[2] * W[8];
    const float dJ11 = dT[3] * W[3] + dT[4] * W[4] + dT[5] * W[5];
    const float dJ12 = dT[3] * W[6] + dT[4] * W[7] + dT[5] * W[8];
    float dpx = gg[0] * vp.fx * iz;
    float dpy = gg[1] * vp.fy * iz;
    float dpz = -gg[0] * vp.fx * x * iz2 - gg[1] * vp.fy * y * iz2;
    dpz += -dJ00 * vp.fx * iz2 - dJ11 * vp.fy * iz2;
    if (!clx) { dpx += -dJ02 * vp.fx * iz2; dpz += dJ02 * 2.0f * vp.fx * x * iz2 * iz; }
    else { dpz += dJ02 * vp.fx * txz * iz2; }
    if (!cly) { dpy += -dJ12 * vp.fy * iz2; dpz += dJ12 * 2.0f * vp.fy * y * iz2 * iz; }
    else { dpz += dJ12 * vp.fy * tyz * iz2; }
    dmu[0] += W[0] * dpx + W[3] * dpy + W[6] * dpz;
    dmu[1] += W[1] * dpx + W[4] * dpy + W[7] * dpz;
    dmu[2] += W[2] * dpx + W[5] * dpy + W[8] * dpz;
    dop += gg[5];
    // colour: rgb = max(0, sum_k B_k(d) sh_k + 0.5), d = (mu - camera centre) / |.|
    const float ccx = -(W[0] * vp.t[0] + W[3] * vp.t[1] + W[6] * vp.t[2]);
    const float ccy = -(W[1] * vp.t[0] + W[4] * vp.t[1] + W[7] * vp.t[2]);
    const float ccz = -(W[2] * vp.t[0] + W[5] * vp.t[1] + W[8] * vp.t[2]);
    float ddx = mx_w - ccx, ddy = my_w - ccy, ddz = mz_w - ccz;
    const float dl = sqrtf(ddx * ddx + ddy * ddy + ddz * ddz), idl = 1.0f / dl;
    ddx *= idl; ddy *= idl; ddz *= idl;
    float Bv[nc], Bx[nc], By[nc], Bz[nc];
    sh_basis_grad<DEG>(ddx, ddy, ddz, Bv, Bx, By, Bz);
    float gdx = 0.f, gdy = 0.f, gdz = 0.f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      float raw = 0.5f;
#pragma unroll
      for (int k = 0; k < nc; ++k) raw += Bv[k] * shi[3 * k + ch];
      if (!(raw > 0.0f)) continue;
      const float gc = gg[6 + ch];
#pragma unroll
      for (int k = 0; k < nc; ++k) {
        dshv[3 * k + ch] += Bv[k] * gc;
        const float sk = shi[3 * k + ch] * gc;
        gdx += Bx[k] * sk; gdy += By[k] * sk; gdz += Bz[k] * sk;
      }
    }
    const float dd = ddx * gdx + ddy * gdy + ddz * gdz;
    dmu[0] += (gdx - ddx * dd) * idl;
    dmu[1] += (gdy - ddy * dd) * idl;
    dmu[2] += (gdz - ddz * dd) * idl;
  }

  // write, or add to what an earlier call (another view group) wrote
  auto put = [accumulate](float *p, float v) { *p = accumulate ? *p + v : v; };
  // Sigma' -> Sigma
  float dS[9];
  if (xform && d_xform) {
    // Sigma' = A Sigma A^T: dL/dA = (dSp + dSp^T) A Sigma
    float AS[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) AS[3 * r + c] = A[3 * r] * Sg[c] + A[3 * r + 1] * Sg[3 + c] + A[3 * r + 2] * Sg[6 + c];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) acc += (dSp[3 * r + k] + dSp[3 * k + r]) * AS[3 * k + c];
        put(&d_xform[9 * (int64_t)i + 3 * r + c], acc);
      }
  }
  if (xform) {
    float AtG[9];   // A^T dSp
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) AtG[3 * r + c] = A[r] * dSp[c] + A[3 + r] * dSp[3 + c] + A[6 + r] * dSp[6 + c];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) dS[3 * r + c] = AtG[3 * r] * A[c] + AtG[3 * r + 1] * A[3 + c] + AtG[3 * r + 2] * A[6 + c];
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) dS[k] = dSp[k];
  }
  // Sigma = M M^T: dL/dM = (dS + dS^T) M
  float dM[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < 3; ++k) acc += (dS[3 * r + k] + dS[3 * k + r]) * M[3 * k + c];
      dM[3 * r + c] = acc;
    }
  float gR[9];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    put(&d_scales[3 * (int64_t)i + c], dM[c] * Rq[c] + dM[3 + c] * Rq[3 + c] + dM[6 + c] * Rq[6 + c]);
#pragma unroll
    for (int r = 0; r < 3; ++r) gR[3 * r + c] = dM[3 * r + c] * sc[c];
  }
  float gw = 2.f * (-qz * gR[1] + qy * gR[2] + qz * gR[3] - qx * gR[5] - qy * gR[6] + qx * gR[7]);
  float gx = 2.f * (qy * gR[1] + qz * gR[2] + qy * gR[3] - 2.f * qx * gR[4] - qw * gR[5] + qz * gR[6] + qw * gR[7] - 2.f * qx * gR[8]);
  float gy = 2.f * (-2.f * qy * gR[0] + qx * gR[1] + qw * gR[2] + qx * gR[3] + qz * gR[5] - qw * gR[6] + qz * gR[7] - 2.f * qy * gR[8]);
  float gz = 2.f * (-2.f * qz * gR[0] - qw * gR[1] + qx * gR[2] + qw * gR[3] - 2.f * qz * gR[4] + qy * gR[5] + qx * gR[6] + qy * gR[7]);
  // through the normalisation q_hat = q / |q|
  const float pr = qw * gw + qx * gx + qy * gy + qz * gz;
  put(&d_quats[4 * (int64_t)i], (gw - qw * pr) * iq);
  put(&d_quats[4 * (int64_t)i + 1], (gx - qx * pr) * iq);
  put(&d_quats[4 * (int64_t)i + 2], (gy - qy * pr) * iq);
  put(&d_quats[4 * (int64_t)i + 3], (gz - qz * pr) * iq);
  put(&d_means[3 * (int64_t)i], dmu[0]);
  put(&d_means[3 * (int64_t)i + 1], dmu[1]);
  put(&d_means[3 * (int64_t)i + 2], dmu[2]);
  put(&d_opac[i], dop);
#pragma unroll
  for (int k = 0; k < nc * 3; ++k) put(&d_sh[(int64_t)i * nc * 3 + k], dshv[k]);
}

}  // namespace

hipError_t launch_fill_u32(Ctx *c, uint32_t *p, int64_t n, uint32_t v);

namespace {

template <int TW, int TH>
hipError_t launch_walk_order_tw(Ctx *c, const int32_t *nc, const uint32_t **order_out,
                                const uint32_t *mask = nullptr) {
  const uint32_t nt = (uint32_t)c->n_tiles;
  uint32_t *cnt = (uint32_t *)c->bwd_order.p;
  uint32_t *key = cnt + kBwdBuckets;
  uint32_t *order = key + nt;
  *order_out = order;
  hipError_t e = launch_fill_u32(c, cnt, kBwdBuckets, 0u);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((walk_key_kernel<TW, TH>), dim3(nt), dim3(64), 0, c->stream, c->cur_views,
                     c->V, (const uint2 *)c->ranges.p, nc, mask, key);
  hipLaunchKernelGGL(walk_count_kernel, dim3(ceil_div(nt, 256)), dim3(256), 0, c->stream, key, nt,
                     cnt);
  hipLaunchKernelGGL(walk_scan_kernel, dim3(1), dim3(64), 0, c->stream, cnt);
  hipLaunchKernelGGL(walk_scatter_kernel, dim3(ceil_div(nt, 256)), dim3(256), 0, c->stream, key,
                     nt, cnt, order);
  return hipGetLastError();
}

template <int TW, int TH, int SPLIT>
hipError_t launch_bwd_tw(Ctx *c, const float *dL, const float *Tf, const int32_t *nc, const float *Te) {
  // the backward's own LDS batch of staged fragments, at most 64 (one per
  // lane; 10 KB per one-wave workgroup, so LDS does not limit the waves per CU)
  const int batch = std::min(c->frag_batch, 64);
  const size_t lds = (size_t)batch * kSlotWords * sizeof(uint32_t);
  const uint32_t nt = (uint32_t)c->n_tiles;
  ScopedTimer t(c, K_BLEND_BWD);
  const uint32_t *order = nullptr;
  hipError_t e = launch_walk_order_tw<TW, TH>(c, nc, &order);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((blend_backward_kernel<TW, TH, SPLIT>), dim3(nt * SPLIT),
                     dim3(64), lds, c->stream, order, c->cur_views, c->V, c->N, c->T, c->mode,
                     batch, c->bg[0], c->bg[1], c->bg[2], (const uint2 *)c->ranges.p,
                     (const uint32_t *)c->v0.p, (const uint32_t *)c->v1.p,
                     (const FrameInfo *)c->finfo.p, (const GaussRec *)c->grec.p,
                     (const TriRec *)c->trec.p, frame_texture(c), dL, Tf, nc, Te,
                     (float *)c->g2d.p);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fill_u32(Ctx *c, uint32_t *p, int64_t n, uint32_t v);

hipError_t launch_walk_order(Ctx *c, const int32_t *nc, const uint32_t **order,
                             const uint32_t *mask) {
  if (c->tile_w == 16 && c->tile_h == 16) return launch_walk_order_tw<16, 16>(c, nc, order, mask);
  if (c->tile_w == 8 && c->tile_h == 8) return launch_walk_order_tw<8, 8>(c, nc, order, mask);
  return launch_walk_order_tw<32, 8>(c, nc, order, mask);
}

hipError_t launch_backward(Ctx *c, const float *dL, const float *Tf, const int32_t *nc,
                           const float *Te, const float *means, const float *scales,
                           const float *quats, const float *xform, const float *sh,
                           float *d_means, float *d_scales, float *d_quats, float *d_opac,
                           float *d_sh, float *d_xform, bool accumulate) {
  hipError_t e = launch_fill_u32(c, (uint32_t *)c->g2d.p, 9 * (int64_t)c->V * c->N, 0u);
  if (e != hipSuccess) return e;
  if (c->n_tiles > 0) {
    if (c->tile_w == 16 && c->tile_h == 16) e = launch_bwd_tw<16, 16, kBwdSplit16>(c, dL, Tf, nc, Te);
    else if (c->tile_w == 8 && c->tile_h == 8) e = launch_bwd_tw<8, 8, 1>(c, dL, Tf, nc, Te);
    else e = launch_bwd_tw<32, 8, kBwdSplit16>(c, dL, Tf, nc, Te);
    if (e != hipSuccess) return e;
  }
  if (c->N == 0) return hipSuccess;
  ScopedTimer t(c, K_PROJECT_BWD);
  const dim3 grid(ceil_div(c->N, 128)), block(128);
  const float *g2d = (const float *)c->g2d.p;
  const int acc = accumulate ? 1 : 0;
  switch (c->sh_degree) {
    case 0:
      hipLaunchKernelGGL(project_backward_kernel<0>, grid, block, 0, c->stream, c->cur_views, c->V,
                         c->N, means, scales, quats, xform, sh, g2d, d_means, d_scales, d_quats,
                         d_opac, d_sh, d_xform, acc);
      break;
    case 1:
      hipLaunchKernelGGL(project_backward_kernel<1>, grid, block, 0, c->stream, c->cur_views, c->V,
                         c->N, means, scales, quats, xform, sh, g2d, d_means, d_scales, d_quats,
                         d_opac, d_sh, d_xform, acc);
      break;
    case 2:
      hipLaunchKernelGGL(project_backward_kernel<2>, grid, block, 0, c->stream, c->cur_views, c->V,
                         c->N, means, scales, quats, xform, sh, g2d, d_means, d_scales, d_quats,
                         d_opac, d_sh, d_xform, acc);
      break;
    default:
      hipLaunchKernelGGL(project_backward_kernel<3>, grid, block, 0, c->stream, c->cur_views, c->V,
                         c->N, means, scales, quats, xform, sh, g2d, d_means, d_scales, d_quats,
                         d_opac, d_sh, d_xform, acc);
      break;
  }
  return hipGetLastError();
}

}  // namespace umgs
