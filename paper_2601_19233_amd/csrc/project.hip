// Projection of Gaussians (EWA splatting) and fixed-point set-up of triangles.
//
// One thread per (primitive, view).  Each writes the primitive's depth key
// (FP32 bits of the view depth, or kCulled), its tile rectangle, its tile
// count (for the bin stage's scan) and the record the blend stage reads.
//
// The kernels also reduce the frame's range of depth keys, so that the sort
// keys can hold depth relative to the nearest primitive in fewer bits.
//
// Decision values -- view depth, pixel coordinates of triangle vertices and
// their 1/256-px snapping, the triangle depth key -- are evaluated with FP
// contraction disabled in a fixed operation order, so that they are
// reproducible bit for bit: x_view = ((R0 x + R1 y) + R2 z) + t,
// u = (fx x_view) / z_view + cx, X = rint(u * 256),
// key_tri = ((z0 + z1) + z2) * (1/3).
#include "support.h"

namespace umgs {

namespace {

__device__ __forceinline__ float view_row(const float *Rr, float t, float x, float y, float z) {
#pragma clang fp contract(off)
  float a = Rr[0] * x;
  float b = Rr[1] * y;
  float c = Rr[2] * z;
  return ((a + b) + c) + t;
}

__device__ __forceinline__ float pix_coord(float f, float c, float xv, float zv) {
#pragma clang fp contract(off)
  return (f * xv) / zv + c;
}

__device__ __forceinline__ float tri_key(float z0, float z1, float z2) {
#pragma clang fp contract(off)
  return ((z0 + z1) + z2) * (1.0f / 3.0f);
}

__device__ __forceinline__ uint2 pack_rect(int tx0, int ty0, int tx1, int ty1) {
  return make_uint2((uint32_t)tx0 | ((uint32_t)ty0 << 16), (uint32_t)tx1 | ((uint32_t)ty1 << 16));
}

// Real SH basis (3DGS sign convention), degree <= 3, evaluated at unit d.
__device__ __forceinline__ void sh_colour(const float *sh, int deg, float x, float y, float z,
                                          float &r, float &g, float &b) {
  const float C0 = 0.28209479177387814f;
  float acc[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[c] = C0 * sh[c];
  if (deg >= 1) {
    const float C1 = 0.4886025119029199f;
    float w1 = -C1 * y, w2 = C1 * z, w3 = -C1 * x;
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += w1 * sh[3 + c] + w2 * sh[6 + c] + w3 * sh[9 + c];
    if (deg >= 2) {
      float xx = x * x, yy = y * y, zz = z * z, xy = x * y, yz = y * z, xz = x * z;
      float w[5] = {1.0925484305920792f * xy, -1.0925484305920792f * yz,
                    0.31539156525252005f * (2.0f * zz - xx - yy), -1.0925484305920792f * xz,
                    0.5462742152960396f * (xx - yy)};
#pragma unroll
      for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] += w[k] * sh[(4 + k) * 3 + c];
      if (deg >= 3) {
        float v[7] = {-0.5900435899266435f * y * (3.0f * xx - yy),
                      2.890611442640554f * xy * z,
                      -0.4570457994644658f * y * (4.0f * zz - xx - yy),
                      0.3731763325901154f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy),
                      -0.4570457994644658f * x * (4.0f * zz - xx - yy),
                      1.445305721320277f * z * (xx - yy),
                      -0.5900435899266435f * x * (xx - 3.0f * yy)};
#pragma unroll
        for (int k = 0; k < 7; ++k)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[c] += v[k] * sh[(9 + k) * 3 + c];
      }
    }
  }
  r = fmaxf(acc[0] + 0.5f, 0.0f);
  g = fmaxf(acc[1] + 0.5f, 0.0f);
  b = fmaxf(acc[2] + 0.5f, 0.0f);
}

// Projects Gaussian i into view v; returns its depth key (kCulled if culled).
__device__ uint32_t project_gaussian(const ViewParams *__restrict__ views, int N, int T,
                                     int sh_deg, int tile_w, int tile_h,
                                     const float *__restrict__ means,
                                     const float *__restrict__ cov3d,
                                     const float *__restrict__ scales,
                                     const float *__restrict__ quats,
                                     const float *__restrict__ opacity,
                                     const float *__restrict__ sh,
                                     uint32_t *__restrict__ keys, uint2 *__restrict__ rects,
                                     uint64_t *__restrict__ counts,
                                     GaussRec *__restrict__ grec, int i, int v) {
  const ViewParams &vp = views[v];
  const int64_t rid = (int64_t)v * (N + T) + i;
  const float mx_w = means[3 * i], my_w = means[3 * i + 1], mz_w = means[3 * i + 2];
  const float zv = view_row(vp.R + 6, vp.t[2], mx_w, my_w, mz_w);
  const float o = opacity[i];
  // Culled if behind the near plane or unable to reach alpha 1/255 anywhere.
  if (!(zv > kNear) || !(o * 255.0f > 1.0f)) {
    keys[rid] = kCulled;
    counts[rid] = 0;
    rects[rid] = make_uint2(0, 0);
    return kCulled;
  }
  const float xv = view_row(vp.R, vp.t[0], mx_w, my_w, mz_w);
  const float yv = view_row(vp.R + 3, vp.t[1], mx_w, my_w, mz_w);

  // world covariance
  float S[6];
  if (cov3d) {
#pragma unroll
    for (int k = 0; k < 6; ++k) S[k] = cov3d[6 * i + k];
  } else {
    float qw = quats[4 * i], qx = quats[4 * i + 1], qy = quats[4 * i + 2], qz = quats[4 * i + 3];
    float inv = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= inv; qx *= inv; qy *= inv; qz *= inv;
    float Rq[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                   2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                   2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
    float s0 = scales[3 * i], s1 = scales[3 * i + 1], s2 = scales[3 * i + 2];
    float M[9];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      M[3 * r] = Rq[3 * r] * s0;
      M[3 * r + 1] = Rq[3 * r + 1] * s1;
      M[3 * r + 2] = Rq[3 * r + 2] * s2;
    }
    S[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    S[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    S[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
    S[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    S[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
    S[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
  }

  // EWA: Sigma_2D = (J W) Sigma (J W)^T + 0.3 I, J at the frustum-clamped point
  const float iz = 1.0f / zv;
  const float limx = kFrustumClamp * vp.tanx, limy = kFrustumClamp * vp.tany;
  const float txz = fminf(limx, fmaxf(-limx, xv * iz));
  const float tyz = fminf(limy, fmaxf(-limy, yv * iz));
  const float j00 = vp.fx * iz, j02 = -vp.fx * txz * iz;
  const float j11 = vp.fy * iz, j12 = -vp.fy * tyz * iz;
  const float *W = vp.R;
  float A0[3], A1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    A0[k] = j00 * W[k] + j02 * W[6 + k];
    A1[k] = j11 * W[3 + k] + j12 * W[6 + k];
  }
  float SA0[3], SA1[3];
  SA0[0] = S[0] * A0[0] + S[1] * A0[1] + S[2] * A0[2];
  SA0[1] = S[1] * A0[0] + S[3] * A0[1] + S[4] * A0[2];
  SA0[2] = S[2] * A0[0] + S[4] * A0[1] + S[5] * A0[2];
  SA1[0] = S[0] * A1[0] + S[1] * A1[1] + S[2] * A1[2];
  SA1[1] = S[1] * A1[0] + S[3] * A1[1] + S[4] * A1[2];
  SA1[2] = S[2] * A1[0] + S[4] * A1[1] + S[5] * A1[2];
  const float ca = A0[0] * SA0[0] + A0[1] * SA0[1] + A0[2] * SA0[2] + kDilation;
  const float cb = A0[0] * SA1[0] + A0[1] * SA1[1] + A0[2] * SA1[2];
  const float cc = A1[0] * SA1[0] + A1[1] * SA1[1] + A1[2] * SA1[2] + kDilation;
  const float det = ca * cc - cb * cb;
  if (!(det > 0.0f)) {
    keys[rid] = kCulled;
    counts[rid] = 0;
    rects[rid] = make_uint2(0, 0);
    return kCulled;
  }
  const float idet = 1.0f / det;
  const float mx = vp.fx * xv * iz + vp.cx;
  const float my = vp.fy * yv * iz + vp.cy;

  // Support {alpha >= 1/255} = {d^T conic d <= 2 ln(255 o)}: its bounding box
  // has half-extents sqrt(2 L Sigma_xx), sqrt(2 L Sigma_yy); 1 px guard.
  const float L = __logf(255.0f * o);
  const float hx = sqrtf(2.0f * L * ca) * 1.001f + 1.0f;
  const float hy = sqrtf(2.0f * L * cc) * 1.001f + 1.0f;
  int px0 = (int)floorf(fmaxf(mx - hx - 0.5f, -1.0f));
  int px1 = (int)floorf(fminf(mx + hx - 0.5f, (float)vp.W)) + 1;
  int py0 = (int)floorf(fmaxf(my - hy - 0.5f, -1.0f));
  int py1 = (int)floorf(fminf(my + hy - 0.5f, (float)vp.H)) + 1;
  px0 = max(px0, 0); py0 = max(py0, 0);
  px1 = min(px1, vp.W); py1 = min(py1, vp.H);
  // view-dependent colour from the camera centre -R^T t
  const float ccx = -(W[0] * vp.t[0] + W[3] * vp.t[1] + W[6] * vp.t[2]);
  const float ccy = -(W[1] * vp.t[0] + W[4] * vp.t[1] + W[7] * vp.t[2]);
  const float ccz = -(W[2] * vp.t[0] + W[5] * vp.t[1] + W[8] * vp.t[2]);
  float dx = mx_w - ccx, dy = my_w - ccy, dz = mz_w - ccz;
  const float dn = rsqrtf(dx * dx + dy * dy + dz * dz);
  dx *= dn; dy *= dn; dz *= dn;
  const int nc = (sh_deg + 1) * (sh_deg + 1);
  float r, g, b;
  sh_colour(sh + (int64_t)i * nc * 3, sh_deg, dx, dy, dz, r, g, b);

  GaussRec rec;
  rec.mx = mx;
  rec.my = my;
  const float sdet = idet * kLog2e;
  rec.qa = -0.5f * cc * sdet;   // log2(e) x (-conic_a / 2)
  rec.qb = cb * sdet;           // log2(e) x (-conic_b)
  rec.qc = -0.5f * ca * sdet;   // log2(e) x (-conic_c / 2)
  rec.opacity = o;
  rec.r = r;
  rec.g = g;
  rec.b = b;
  rec.lo = __builtin_amdgcn_logf(o);   // log2
  rec.inv_o = 1.0f / o;
  rec.pad = 0.0f;
  grec[(int64_t)v * N + i] = rec;

  // tiles and supertiles of the bounding rectangle (upper bounds: the masks
  // of the bin stage cut every row to the support)
  uint32_t cnt = 0, nst = 0;
  uint2 rect = make_uint2(0, 0);
  if (px0 < px1 && py0 < py1) {
    const int tx0 = px0 / tile_w, tx1 = (px1 - 1) / tile_w + 1;
    const int ty0 = py0 / tile_h, ty1 = (py1 - 1) / tile_h + 1;
    cnt = (uint32_t)((tx1 - tx0) * (ty1 - ty0));
    nst = (uint32_t)((((tx1 - 1) >> kSTLog) - (tx0 >> kSTLog) + 1) *
                     (((ty1 - 1) >> kSTLog) - (ty0 >> kSTLog) + 1));
    rect = pack_rect(tx0, ty0, tx1, ty1);
  }
  keys[rid] = __float_as_uint(zv);
  counts[rid] = (uint64_t)nst << 32 | cnt;
  rects[rid] = rect;
  return __float_as_uint(zv);
}

// Folds a workgroup's valid depth keys into the frame's [min, max]: one
// atomic pair per workgroup (256 threads), into its own slot pair of
// kMinMaxSlots.  Atomics on one address serialise at the memory side, so
// the frame's few thousand workgroups each get an address (with 64 slots,
// one pair per wave, they cost the projection 56 us at 1M Gaussians); the
// bin stage folds the slots.  Every thread of the workgroup calls it.
__device__ __forceinline__ void reduce_key_range(uint32_t key, uint32_t *minmax) {
  __shared__ uint32_t wlo[4], whi[4];
  const uint32_t lo = wave_min_u32(key);
  const uint32_t hi = wave_max_u32(key == kCulled ? 0u : key);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    wlo[w] = lo;
    whi[w] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t l = wlo[0], h = whi[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
      l = min(l, wlo[k]);
      h = max(h, whi[k]);
    }
    if (l != kCulled) {
      const uint32_t slot = (blockIdx.y * gridDim.x + blockIdx.x) & (kMinMaxSlots - 1);
      atomicMin(minmax + slot, l);
      atomicMax(minmax + kMinMaxSlots + slot, h);
    }
  }
}

__global__ __launch_bounds__(256) void project_gaussians_kernel(const ViewParams *__restrict__ views, int N, int T,
                                         int sh_deg, int tile_w, int tile_h,
                                         const float *__restrict__ means,
                                         const float *__restrict__ cov3d,
                                         const float *__restrict__ scales,
                                         const float *__restrict__ quats,
                                         const float *__restrict__ opacity,
                                         const float *__restrict__ sh,
                                         uint32_t *__restrict__ keys, uint2 *__restrict__ rects,
                                         uint64_t *__restrict__ counts,
                                         GaussRec *__restrict__ grec, uint32_t *__restrict__ minmax) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  uint32_t key = kCulled;
  if (i < N)
    key = project_gaussian(views, N, T, sh_deg, tile_w, tile_h, means, cov3d, scales, quats,
                           opacity, sh, keys, rects, counts, grec, i, v);
  reduce_key_range(key, minmax);
}

// Sets up triangle j for view v; returns its depth key (kCulled if culled).
__device__ uint32_t setup_triangle(const ViewParams *__restrict__ views, int N, int T,
                                   int tile_w, int tile_h, const float *__restrict__ xyz,
                                   const float *__restrict__ rgb, const float *__restrict__ alpha,
                                   const float *__restrict__ uv,
                                   uint32_t *__restrict__ keys, uint2 *__restrict__ rects,
                                   uint64_t *__restrict__ counts, TriRec *__restrict__ trec,
                                   int j, int v) {
  const ViewParams &vp = views[v];
  const int64_t rid = (int64_t)v * (N + T) + N + j;
  const float *P = xyz + 9 * (int64_t)j;
  float zv[3], uf[3], vf[3];
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float x = P[3 * k], y = P[3 * k + 1], z = P[3 * k + 2];
    const float xv = view_row(vp.R, vp.t[0], x, y, z);
    const float yv = view_row(vp.R + 3, vp.t[1], x, y, z);
    zv[k] = view_row(vp.R + 6, vp.t[2], x, y, z);
    ok = ok && (zv[k] > kNear);
    const float zs = zv[k] > kNear ? zv[k] : 1.0f;
    uf[k] = pix_coord(vp.fx, vp.cx, xv, zs);
    vf[k] = pix_coord(vp.fy, vp.cy, yv, zs);
  }
  int32_t X[3], Y[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float us = rintf(uf[k] * (float)kSubpx);
    const float vs = rintf(vf[k] * (float)kSubpx);
    ok = ok && (fabsf(us) <= (float)kCoordLimit) && (fabsf(vs) <= (float)kCoordLimit);
    X[k] = ok ? (int32_t)us : 0;
    Y[k] = ok ? (int32_t)vs : 0;
  }
  int64_t area2 = (int64_t)(X[1] - X[0]) * (Y[2] - Y[0]) - (int64_t)(Y[1] - Y[0]) * (X[2] - X[0]);
  ok = ok && (area2 != 0);
  if (!ok) {
    keys[rid] = kCulled;
    counts[rid] = 0;
    rects[rid] = make_uint2(0, 0);
    TriRec z = {};
    trec[(int64_t)v * T + j] = z;
    return kCulled;
  }
  const float key = tri_key(zv[0], zv[1], zv[2]);
  int perm[3] = {0, 1, 2};
  if (area2 < 0) { perm[1] = 2; perm[2] = 1; }
  TriRec rec;
  const float *C = rgb + 9 * (int64_t)j;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int s = perm[k];
    rec.X[k] = X[s];
    rec.Y[k] = Y[s];
    const float izk = 1.0f / zv[s];
    rec.iz[k] = izk;
    rec.ciz[3 * k] = C[3 * s] * izk;
    rec.ciz[3 * k + 1] = C[3 * s + 1] * izk;
    rec.ciz[3 * k + 2] = C[3 * s + 2] * izk;
    rec.uviz[2 * k] = uv ? uv[6 * (int64_t)j + 2 * s] * izk : 0.0f;
    rec.uviz[2 * k + 1] = uv ? uv[6 * (int64_t)j + 2 * s + 1] * izk : 0.0f;
  }
  rec.swapped = area2 < 0 ? 1u : 0u;
  rec.pad = 0.0f;
  rec.alpha = alpha[j];
  uint32_t owned = 0;
  const int ea[3] = {1, 2, 0}, eb[3] = {2, 0, 1};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int32_t ddx = rec.X[eb[k]] - rec.X[ea[k]];
    const int32_t ddy = rec.Y[eb[k]] - rec.Y[ea[k]];
    if (ddy > 0 || (ddy == 0 && ddx < 0)) owned |= 1u << k;
  }
  rec.owned = owned;
  trec[(int64_t)v * T + j] = rec;

  // Pixels whose samples (x offsets 32..224, y offsets 32..224 in 1/256 px)
  // can fall inside the snapped bounding box.
  const int minX = min(X[0], min(X[1], X[2])), maxX = max(X[0], max(X[1], X[2]));
  const int minY = min(Y[0], min(Y[1], Y[2])), maxY = max(Y[0], max(Y[1], Y[2]));
  int px0 = max((minX + 31) >> 8, 0), px1 = min(((maxX - 32) >> 8) + 1, vp.W);
  int py0 = max((minY + 31) >> 8, 0), py1 = min(((maxY - 32) >> 8) + 1, vp.H);
  uint32_t cnt = 0, nst = 0;
  uint2 rect = make_uint2(0, 0);
  if (px0 < px1 && py0 < py1) {
    const int tx0 = px0 / tile_w, tx1 = (px1 - 1) / tile_w + 1;
    const int ty0 = py0 / tile_h, ty1 = (py1 - 1) / tile_h + 1;
    cnt = (uint32_t)((tx1 - tx0) * (ty1 - ty0));
    nst = (uint32_t)((((tx1 - 1) >> kSTLog) - (tx0 >> kSTLog) + 1) *
                     (((ty1 - 1) >> kSTLog) - (ty0 >> kSTLog) + 1));
    rect = pack_rect(tx0, ty0, tx1, ty1);
  }
  keys[rid] = __float_as_uint(key);
  counts[rid] = (uint64_t)nst << 32 | cnt;
  rects[rid] = rect;
  return __float_as_uint(key);
}

__global__ __launch_bounds__(256) void setup_triangles_kernel(const ViewParams *__restrict__ views, int N, int T,
                                       int tile_w, int tile_h, const float *__restrict__ xyz,
                                       const float *__restrict__ rgb,
                                       const float *__restrict__ alpha,
                                       const float *__restrict__ uv,
                                       uint32_t *__restrict__ keys, uint2 *__restrict__ rects,
                                       uint64_t *__restrict__ counts,
                                       TriRec *__restrict__ trec, uint32_t *__restrict__ minmax) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  uint32_t key = kCulled;
  if (j < T)
    key = setup_triangle(views, N, T, tile_w, tile_h, xyz, rgb, alpha, uv, keys, rects, counts,
                         trec, j, v);
  reduce_key_range(key, minmax);
}

}  // namespace

hipError_t launch_project_gaussians(Ctx *c, const float *means, const float *cov3d,
                                    const float *scales, const float *quats,
                                    const float *opacity, const float *sh) {
  if (c->N == 0) return hipSuccess;
  dim3 grid(ceil_div(c->N, 256), c->V);
  ScopedTimer t(c, K_PROJECT);
  hipLaunchKernelGGL(project_gaussians_kernel, grid, dim3(256), 0, c->stream,
                     c->cur_views, c->N, c->T, c->sh_degree, c->tile_w,
                     c->tile_h, means, cov3d, scales, quats, opacity, sh,
                     (uint32_t *)c->keys.p, (uint2 *)c->rects.p, (uint64_t *)c->counts.p,
                     (GaussRec *)c->grec.p, (uint32_t *)c->minmax.p);
  return hipGetLastError();
}

hipError_t launch_setup_triangles(Ctx *c, const float *tri_xyz, const float *tri_rgb,
                                  const float *tri_alpha) {
  if (c->T == 0) return hipSuccess;
  dim3 grid(ceil_div(c->T, 256), c->V);
  ScopedTimer t(c, K_TRIANGLES);
  hipLaunchKernelGGL(setup_triangles_kernel, grid, dim3(256), 0, c->stream,
                     c->cur_views, c->N, c->T, c->tile_w, c->tile_h,
                     tri_xyz, tri_rgb, tri_alpha,
                     c->tex_w > 0 ? (const float *)c->tex_uv.p : nullptr, (uint32_t *)c->keys.p,
                     (uint2 *)c->rects.p, (uint64_t *)c->counts.p, (TriRec *)c->trec.p,
                     (uint32_t *)c->minmax.p);
  return hipGetLastError();
}

}  // namespace umgs
