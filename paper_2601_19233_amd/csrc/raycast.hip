// Binding association by ray casting (Section 3.3.1).
//
// For every Gaussian target point (its mean, or the eight corners of its
// bounding box mu + R diag(3 s) [-1,1]^3) a ray is cast from every camera
// centre towards the point; each proxy face the ray crosses (t > 0) is a
// candidate, and the target binds to the crossing nearest to it over all
// faces and cameras.
//
// The proxy is indexed by a linear BVH built on the device: Morton codes of
// the face centroids, a radix sort, and the hierarchy of Karras (HPG 2012,
// "Maximizing parallelism in the construction of BVHs, octrees and k-d
// trees") over the sorted codes, ties in code broken by sorted position.
// Each internal node stores the boxes of both children, so a traversal step
// reads one 64-byte node and tests two boxes.  One wavefront builds one node:
// its lanes reduce the children's boxes over their (contiguous) leaf ranges,
// so no bottom-up synchronisation is needed.
//
// The query is not a first-hit query: the target sits at t = 1 on the ray
// o + t (P - o), and a subtree is skipped when its slab interval misses
// [1 - b, 1 + b], b the best distance so far in units of |P - o|.  Children
// are visited nearest-interval first.  The crossing test is Moller-Trumbore
// (1997) in FP32.  Gaussians are cast in the Morton order of their means, so
// the lanes of a wavefront trace neighbouring rays through the same nodes.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace umgs {
namespace {

constexpr int kCastThreads = 64;  // one wavefront per workgroup (LDS stack per lane)
constexpr int kAuxCams = 16;      // float offset of the camera centres in bvh_aux
constexpr int kAuxFault = 8;      // uint32 offset of the fault flag in bvh_aux

__device__ inline float3 f3(float4 a) { return make_float3(a.x, a.y, a.z); }
__device__ inline float3 sub3(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ inline float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline float3 cross3(float3 a, float3 b) {
  return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

__device__ inline float wave_min(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
  return v;
}
__device__ inline float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// 10 bits per axis interleaved (x in the highest position of each triple).
__device__ inline uint32_t spread10(uint32_t v) {
  v = (v * 0x00010001u) & 0xFF0000FFu;
  v = (v * 0x00000101u) & 0x0F00F00Fu;
  v = (v * 0x00000011u) & 0xC30C30C3u;
  v = (v * 0x00000005u) & 0x49249249u;
  return v;
}

// Bounds of the face centroids (one workgroup) and the fault flag cleared.
__global__ __launch_bounds__(1024) void centroid_bounds_kernel(const float *__restrict__ V,
                                                               const int32_t *__restrict__ F,
                                                               int32_t nF, float *aux) {
  __shared__ float s_lo[3][16], s_hi[3][16];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int f = threadIdx.x; f < nF; f += blockDim.x) {
    const int a = F[3 * f], b = F[3 * f + 1], c = F[3 * f + 2];
    for (int k = 0; k < 3; ++k) {
      const float x = (V[3 * a + k] + V[3 * b + k] + V[3 * c + k]) * (1.0f / 3.0f);
      lo[k] = fminf(lo[k], x);
      hi[k] = fmaxf(hi[k], x);
    }
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int k = 0; k < 3; ++k) {
    lo[k] = wave_min(lo[k]);
    hi[k] = wave_max(hi[k]);
    if (lane == 0) {
      s_lo[k][w] = lo[k];
      s_hi[k][w] = hi[k];
    }
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int nw = blockDim.x >> 6;
    for (int k = 0; k < 3; ++k) {
      float l = lane < nw ? s_lo[k][lane] : INFINITY;
      float h = lane < nw ? s_hi[k][lane] : -INFINITY;
      l = wave_min(l);
      h = wave_max(h);
      if (lane == 0) {
        aux[k] = l;
        aux[3 + k] = h;
      }
    }
    if (lane == 0) ((uint32_t *)aux)[kAuxFault] = 0u;
  }
}

__global__ __launch_bounds__(256) void morton_kernel(const float *__restrict__ V,
                                                     const int32_t *__restrict__ F, int32_t nF,
                                                     const float *__restrict__ aux,
                                                     uint32_t *__restrict__ code,
                                                     uint32_t *__restrict__ id) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nF) return;
  const int a = F[3 * f], b = F[3 * f + 1], c = F[3 * f + 2];
  uint32_t m = 0;
  for (int k = 0; k < 3; ++k) {
    const float x = (V[3 * a + k] + V[3 * b + k] + V[3 * c + k]) * (1.0f / 3.0f);
    const float ext = aux[3 + k] - aux[k];
    const float r = ext > 0.0f ? (x - aux[k]) / ext : 0.0f;
    const uint32_t q = (uint32_t)fminf(fmaxf(r * 1024.0f, 0.0f), 1023.0f);
    m |= spread10(q) << (2 - k);
  }
  code[f] = m;
  id[f] = (uint32_t)f;
}

// Morton code of each Gaussian's mean in the proxy's centroid bounds
// (clamped): casting in this order keeps a wavefront's rays together.
__global__ __launch_bounds__(256) void mean_order_kernel(const float *__restrict__ means, int32_t N,
                                                         const float *__restrict__ aux,
                                                         uint32_t *__restrict__ code,
                                                         uint32_t *__restrict__ id) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  uint32_t m = 0;
  for (int k = 0; k < 3; ++k) {
    const float ext = aux[3 + k] - aux[k];
    const float r = ext > 0.0f ? (means[3 * (int64_t)g + k] - aux[k]) / ext : 0.0f;
    const uint32_t q = (uint32_t)fminf(fmaxf(r * 1024.0f, 0.0f), 1023.0f);
    m |= spread10(q) << (2 - k);
  }
  code[g] = m;
  id[g] = (uint32_t)g;
}

// Leaf triangles in sorted order, arranged for the crossing test: first the
// vertex the barycentrics leave implicit (V[f2], with the face id in .w),
// then V[f0] and V[f1], whose weights are the binding's (u, v).
__global__ __launch_bounds__(256) void leaf_kernel(const float *__restrict__ V,
                                                   const int32_t *__restrict__ F, int32_t nF,
                                                   const uint32_t *__restrict__ id,
                                                   float4 *__restrict__ tri) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nF) return;
  const int f = (int)id[i];
  const int v0 = F[3 * f], v1 = F[3 * f + 1], v2 = F[3 * f + 2];
  tri[3 * i] = make_float4(V[3 * v2], V[3 * v2 + 1], V[3 * v2 + 2], __int_as_float(f));
  tri[3 * i + 1] = make_float4(V[3 * v0], V[3 * v0 + 1], V[3 * v0 + 2], 0.0f);
  tri[3 * i + 2] = make_float4(V[3 * v1], V[3 * v1 + 1], V[3 * v1 + 2], 0.0f);
}

// Length of the common prefix of the keys (code << 32 | position) at sorted
// positions i and j; -1 outside [0, n).
__device__ inline int prefix_len(const uint32_t *code, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  const unsigned long long ki = ((unsigned long long)code[i] << 32) | (uint32_t)i;
  const unsigned long long kj = ((unsigned long long)code[j] << 32) | (uint32_t)j;
  return __clzll(ki ^ kj);
}

// Box of the leaves [first, last] (inclusive), reduced over the wavefront and
// widened so that the FP32 slab test never rejects a box that a crossing
// found by the triangle test lies in.
__device__ inline void range_box(const float4 *tri, int first, int last, int lane, float pad,
                                 float4 &lo, float4 &hi) {
  float l[3] = {INFINITY, INFINITY, INFINITY}, h[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int k = first + lane; k <= last; k += 64) {
    for (int v = 0; v < 3; ++v) {
      const float4 p = tri[3 * k + v];
      l[0] = fminf(l[0], p.x); h[0] = fmaxf(h[0], p.x);
      l[1] = fminf(l[1], p.y); h[1] = fmaxf(h[1], p.y);
      l[2] = fminf(l[2], p.z); h[2] = fmaxf(h[2], p.z);
    }
  }
  for (int k = 0; k < 3; ++k) {
    l[k] = wave_min(l[k]);
    h[k] = wave_max(h[k]);
    l[k] -= pad + 1e-6f * fabsf(l[k]);
    h[k] += pad + 1e-6f * fabsf(h[k]);
  }
  lo = make_float4(l[0], l[1], l[2], 0.0f);
  hi = make_float4(h[0], h[1], h[2], 0.0f);
}

// One wavefront per internal node i (n - 1 nodes; one node holding leaf 0
// twice when n = 1).  Children: >= 0 internal node, < 0 leaf ~c.
__global__ __launch_bounds__(256) void node_kernel(const uint32_t *__restrict__ code, int32_t n,
                                                   const float4 *__restrict__ tri,
                                                   const float *__restrict__ aux,
                                                   float4 *__restrict__ node) {
  const int i = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const int n_int = n > 1 ? n - 1 : 1;
  if (i >= n_int) return;
  const float pad =
      fmaxf(1e-5f * fmaxf(fmaxf(aux[3] - aux[0], aux[4] - aux[1]), aux[5] - aux[2]), 1e-6f);
  int first, last, split;
  if (n == 1) {
    first = 0;
    last = 0;
    split = 0;
  } else {
    const int d = prefix_len(code, n, i, i + 1) - prefix_len(code, n, i, i - 1) > 0 ? 1 : -1;
    const int dmin = prefix_len(code, n, i, i - d);
    int lmax = 2;
    while (prefix_len(code, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
      if (prefix_len(code, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = prefix_len(code, n, i, j);
    int s = 0, t = l;
    do {
      t = (t + 1) >> 1;
      if (prefix_len(code, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    split = i + s * d + (d < 0 ? -1 : 0);
    first = min(i, j);
    last = max(i, j);
  }
  float4 llo, lhi, rlo, rhi;
  int left, right;
  if (n == 1) {
    range_box(tri, 0, 0, lane, pad, llo, lhi);
    rlo = llo;
    rhi = lhi;
    left = right = ~0;
  } else {
    range_box(tri, first, split, lane, pad, llo, lhi);
    range_box(tri, split + 1, last, lane, pad, rlo, rhi);
    left = first == split ? ~split : split;
    right = last == split + 1 ? ~(split + 1) : split + 1;
  }
  if (lane == 0) {
    llo.w = __int_as_float(left);
    lhi.w = __int_as_float(right);
    node[4 * i] = llo;
    node[4 * i + 1] = lhi;
    node[4 * i + 2] = rlo;
    node[4 * i + 3] = rhi;
  }
}

// Slab interval of the ray o + t d inside [lo, hi]; returns its distance to
// t = 1 (negative when the interval is empty, lies behind the camera, or is
// farther from t = 1 than reach).  Each plane costs one FMA, x inv - o inv
// (oi = o inv).  Plane parameters carry a relative rounding error of a few
// units in the last place whatever the camera's distance, so the interval
// is widened by 2^-20 of its ends (the boxes' own widening is in scene
// units and would not cover a far camera).
__device__ inline float box_reach(float3 oi, float3 inv, float4 lo, float4 hi, float reach) {
  const float tx0 = fmaf(lo.x, inv.x, -oi.x), tx1 = fmaf(hi.x, inv.x, -oi.x);
  const float ty0 = fmaf(lo.y, inv.y, -oi.y), ty1 = fmaf(hi.y, inv.y, -oi.y);
  const float tz0 = fmaf(lo.z, inv.z, -oi.z), tz1 = fmaf(hi.z, inv.z, -oi.z);
  float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fminf(tz0, tz1));
  float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1));
  tn = fmaf(-0x1p-20f, fabsf(tn), tn);
  tf = fmaf(0x1p-20f, fabsf(tf), tf);
  if (!(tn <= tf) || !(tf > 0.0f)) return -1.0f;
  const float gap = fmaxf(fmaxf(tn - 1.0f, 1.0f - tf), 0.0f);
  return gap <= reach ? gap : -1.0f;
}

struct Best {
  float dist, b1, b2;
  int face, cam;
};

__device__ inline void test_leaf(const float4 *__restrict__ tri, int leaf, float3 o, float3 d,
                                 float dn, int cam, Best &best) {
  const float4 a4 = tri[3 * leaf];
  const float3 A = f3(a4);
  const float3 e1 = sub3(f3(tri[3 * leaf + 1]), A);
  const float3 e2 = sub3(f3(tri[3 * leaf + 2]), A);
  const float3 p = cross3(d, e2);
  const float det = dot3(e1, p);
  if (det == 0.0f) return;
  const float inv = 1.0f / det;
  const float3 s = sub3(o, A);
  const float b1 = dot3(s, p) * inv;
  if (!(b1 >= 0.0f) || b1 > 1.0f) return;
  const float3 q = cross3(s, e1);
  const float b2 = dot3(d, q) * inv;
  if (!(b2 >= 0.0f) || b1 + b2 > 1.0f) return;
  const float t = dot3(e2, q) * inv;
  if (!(t > 0.0f)) return;
  const float dist = fabsf(t - 1.0f) * dn;
  const int face = __float_as_int(a4.w);
  if (dist < best.dist || (dist == best.dist && cam == best.cam && face < best.face)) {
    best.dist = dist;
    best.b1 = b1;
    best.b2 = b2;
    best.face = face;
    best.cam = cam;
  }
}

__device__ inline float safe_inv(float x) {
  return fabsf(x) > 1e-30f ? 1.0f / x : copysignf(1e30f, x);
}

// One lane per target point (Gaussian g, corner k); cameras in order.  The
// traversal stack holds internal-node indices in LDS.  Each level of the
// hierarchy lengthens the common prefix of its keys (30-bit code, then the
// sorted position) by at least one of the bits that vary, so a path holds at
// most 30 + log2(n) internal nodes and the stack never needs more entries:
// 48 16-bit entries below 2^16 faces, 64 32-bit entries up to 2^31.
template <typename S, int kStack>
__global__ __launch_bounds__(kCastThreads) void cast_kernel(
    const float *__restrict__ means, const float *__restrict__ scales,
    const float *__restrict__ quats, const uint32_t *__restrict__ order, int32_t N, int32_t K,
    int32_t C,
    const float *__restrict__ aux, const float4 *__restrict__ node,
    const float4 *__restrict__ tri, int32_t n_int, int32_t *__restrict__ bind_face,
    float *__restrict__ bind_bary, float *__restrict__ dist_out, uint32_t *fault) {
  __shared__ S s_stack[kStack][kCastThreads];
  const int64_t idx = (int64_t)blockIdx.x * kCastThreads + threadIdx.x;
  if (idx >= (int64_t)N * K) return;
  const int64_t slot = idx / K;
  const int k = (int)(idx - slot * K);
  const int64_t g = order[slot];
  const int64_t out = g * K + k;
  float3 P = make_float3(means[3 * g], means[3 * g + 1], means[3 * g + 2]);
  if (K == 8) {
    float w = quats[4 * g], x = quats[4 * g + 1], y = quats[4 * g + 2], z = quats[4 * g + 3];
    const float rn = 1.0f / sqrtf(w * w + x * x + y * y + z * z);
    w *= rn; x *= rn; y *= rn; z *= rn;
    const float hx = (k & 1 ? 3.0f : -3.0f) * scales[3 * g];
    const float hy = (k & 2 ? 3.0f : -3.0f) * scales[3 * g + 1];
    const float hz = (k & 4 ? 3.0f : -3.0f) * scales[3 * g + 2];
    P.x += (1.0f - 2.0f * (y * y + z * z)) * hx + 2.0f * (x * y - w * z) * hy + 2.0f * (x * z + w * y) * hz;
    P.y += 2.0f * (x * y + w * z) * hx + (1.0f - 2.0f * (x * x + z * z)) * hy + 2.0f * (y * z - w * x) * hz;
    P.z += 2.0f * (x * z - w * y) * hx + 2.0f * (y * z + w * x) * hy + (1.0f - 2.0f * (x * x + y * y)) * hz;
  }
  const float *cams = aux + kAuxCams;
  Best best{INFINITY, 0.0f, 0.0f, -1, -1};
  bool overflow = false;
  const int lane = threadIdx.x;
  for (int c = 0; c < C && !overflow; ++c) {
    const float3 o = make_float3(cams[3 * c], cams[3 * c + 1], cams[3 * c + 2]);
    const float3 d = sub3(P, o);
    const float dn = sqrtf(dot3(d, d));
    if (!(dn > 0.0f)) continue;
    const float3 inv = make_float3(safe_inv(d.x), safe_inv(d.y), safe_inv(d.z));
    const float3 oi = make_float3(o.x * inv.x, o.y * inv.y, o.z * inv.z);
    int sp = 0;
    int cur = 0;
    // a traversal visits each internal node at most once; the cap bounds
    // the loop even for a malformed hierarchy
    for (int steps = 0;; ++steps) {
      if (steps > n_int) {
        overflow = true;
        break;
      }
      // reach in ray units, slightly widened so rounding never prunes a
      // subtree holding a crossing at exactly the best distance
      const float reach = isinf(best.dist) ? INFINITY : best.dist / dn * 1.0001f + 1e-7f;
      const float4 llo = node[4 * cur], lhi = node[4 * cur + 1];
      const float4 rlo = node[4 * cur + 2], rhi = node[4 * cur + 3];
      const int lc = __float_as_int(llo.w), rc = __float_as_int(lhi.w);
      const float gl = box_reach(oi, inv, llo, lhi, reach);
      const float gr = box_reach(oi, inv, rlo, rhi, reach);
      int next[2];
      int nn = 0;
      if (gl >= 0.0f) {
        if (lc < 0) test_leaf(tri, ~lc, o, d, dn, c, best);
        else next[nn++] = lc;
      }
      if (gr >= 0.0f) {
        if (rc < 0) test_leaf(tri, ~rc, o, d, dn, c, best);
        else next[nn++] = rc;
      }
      if (nn == 2) {
        const bool swap = gr < gl;   // nearer interval first
        const int near = swap ? next[1] : next[0], far = swap ? next[0] : next[1];
        if (sp == kStack) {
          overflow = true;
          break;
        }
        s_stack[sp++][lane] = (S)far;
        cur = near;
      } else if (nn == 1) {
        cur = next[0];
      } else {
        if (sp == 0) break;
        cur = (int)s_stack[--sp][lane];
      }
    }
  }
  if (overflow) *fault = 1u;
  bind_face[out] = best.face;
  bind_bary[2 * out] = best.face >= 0 ? best.b1 : 0.0f;
  bind_bary[2 * out + 1] = best.face >= 0 ? best.b2 : 0.0f;
  if (dist_out) dist_out[out] = best.dist;
}

}  // namespace

size_t bvh_aux_bytes(int32_t C) { return sizeof(float) * (kAuxCams + 3 * (size_t)C); }
uint32_t *bvh_fault_flag(Ctx *c) { return (uint32_t *)c->bvh_aux.p + kAuxFault; }
float *bvh_cam_slots(Ctx *c) { return (float *)c->bvh_aux.p + kAuxCams; }

hipError_t launch_bvh_build(Ctx *c) {
  const int32_t n = c->nF;
  const float *V = (const float *)c->V_rest.p;
  const int32_t *F = (const int32_t *)c->faces.p;
  float *aux = (float *)c->bvh_aux.p;
  uint32_t *code[2] = {(uint32_t *)c->bvh_code[0].p, (uint32_t *)c->bvh_code[1].p};
  uint32_t *id[2] = {(uint32_t *)c->bvh_id[0].p, (uint32_t *)c->bvh_id[1].p};
  hipLaunchKernelGGL(centroid_bounds_kernel, dim3(1), dim3(1024), 0, c->stream, V, F, n, aux);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(morton_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, c->stream, V, F, n,
                     (const float *)aux, code[0], id[0]);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_radix_sort_u32(c, code, id, (uint64_t)n, nullptr, nullptr, 30, -1, -1, -1)) !=
      hipSuccess)
    return e;
  const int res = radix_passes(30) & 1;
  hipLaunchKernelGGL(leaf_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, c->stream, V, F, n,
                     (const uint32_t *)id[res], (float4 *)c->bvh_tri.p);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int n_int = n > 1 ? n - 1 : 1;
  hipLaunchKernelGGL(node_kernel, dim3(ceil_div((uint64_t)n_int * 64, 256)), dim3(256), 0,
                     c->stream, (const uint32_t *)code[res], n, (const float4 *)c->bvh_tri.p,
                     (const float *)aux, (float4 *)c->bvh_node.p);
  return hipGetLastError();
}

hipError_t launch_raycast(Ctx *c, int32_t N, const float *means, const float *scales,
                          const float *quats, int32_t K, int32_t C, int32_t *bind_face,
                          float *bind_bary, float *dist) {
  const int64_t M = (int64_t)N * K;
  if (M == 0) return hipSuccess;
  uint32_t *code[2] = {(uint32_t *)c->cast_code[0].p, (uint32_t *)c->cast_code[1].p};
  uint32_t *id[2] = {(uint32_t *)c->cast_id[0].p, (uint32_t *)c->cast_id[1].p};
  hipLaunchKernelGGL(mean_order_kernel, dim3(ceil_div(N, 256)), dim3(256), 0, c->stream, means, N,
                     (const float *)c->bvh_aux.p, code[0], id[0]);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_radix_sort_u32(c, code, id, (uint64_t)N, nullptr, nullptr, 30, -1, -1, -1)) !=
      hipSuccess)
    return e;
  const uint32_t *order = id[radix_passes(30) & 1];
  const int32_t n_int = c->nF > 1 ? c->nF - 1 : 1;
  if (c->nF <= (1 << 16))
    hipLaunchKernelGGL((cast_kernel<uint16_t, 48>), dim3(ceil_div(M, kCastThreads)), dim3(kCastThreads),
                       0, c->stream, means, scales, quats, order, N, K, C,
                       (const float *)c->bvh_aux.p, (const float4 *)c->bvh_node.p,
                       (const float4 *)c->bvh_tri.p, n_int, bind_face, bind_bary, dist,
                       bvh_fault_flag(c));
  else
    hipLaunchKernelGGL((cast_kernel<uint32_t, 64>), dim3(ceil_div(M, kCastThreads)), dim3(kCastThreads),
                       0, c->stream, means, scales, quats, order, N, K, C,
                       (const float *)c->bvh_aux.p, (const float4 *)c->bvh_node.p,
                       (const float4 *)c->bvh_tri.p, n_int, bind_face, bind_bary, dist,
                       bvh_fault_flag(c));
  return hipGetLastError();
}

}  // namespace umgs
