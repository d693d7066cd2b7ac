// Deformation transfer from a proxy mesh to bound Gaussians.
//
// vertex_frames_kernel (one thread per proxy vertex, FP64):
//   Delta_v = V'_v - V_v (FP32 subtraction: it feeds the pinned mean);
//   D_v = (sum c e' e^T + w n' n^T)(sum c e e^T + w n n^T)^-1 over the rest
//   1-ring, c = (cot a + cot b)/2 accumulated face by face, n / n' the rest /
//   deformed area-weighted normals scaled by the mean 1-ring edge length of
//   their mesh, w the mean cotangent weight;
//   polar D = R S with R = [u1 u2 u1 x u2][v1 v2 v3]^T from the eigenvectors
//   of D^T D (a proper rotation; the nearest one to D);
//   r_v = log R (axis-angle, angle in [0, pi], robust near pi), written with
//   S as a 12-float row.
// face_rows_kernel: each face's three vertex rows side by side (144 B), so a
//   bound point reads one row that spans exactly two 128-B cache lines
//   (rows start at multiples of 16 B) instead of a face lookup followed by
//   three vertex rows in three places; row nF is all zeros (what an unbound
//   corner reads).
// transfer kernels (FP32): Eq. 12 at each of the K bound points, Eq. 13
//   averages: R' = exp(mean r_i), S' = mean S_i, A = R'S',
//   Sigma' = A Sigma A^T, mu' = mu + mean Delta_i (pinned order),
//   q' = quat(R') * q, one lane per Gaussian.  A corner whose face index
//   lies outside [0, nF) (the ray-cast binding writes -1 where no ray
//   crosses the proxy) is unbound: the means run over the bound corners
//   only, and a Gaussian without a bound corner keeps its rest pose.
#include "internal.h"

#include <mutex>

// Scratch of the allocation-free transfer (umgs_bind_transfer_noalloc): the
// per-vertex table (48 B per proxy vertex, unless the caller takes it) and
// the face rows (144 B per face, at a 256-byte boundary after it).  Every
// GPU the library runs on holds its own copy until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns for
// the current device.
static __device__ __align__(256) unsigned char scratch[umgs::kNoAllocScratchBytes];

namespace umgs {

namespace {
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_addr[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_addr[device] = p;
  return hipSuccess;
}

void *noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_addr[device];
}

size_t noalloc_transfer_bytes(int64_t nV, int64_t nF, bool vertex_table_in_scratch) {
  const size_t vt = vertex_table_in_scratch ? (size_t)(48 * nV + 255) / 256 * 256 : 0;
  return vt + (size_t)144 * ((size_t)nF + 1);   // face rows and the zero row
}

namespace {

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
__device__ __forceinline__ double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

// cot of the angle at p between p->q and p->r
__device__ __forceinline__ double cot_at(const double p[3], const double q[3], const double r[3]) {
  double u1[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
  double u2[3] = {r[0] - p[0], r[1] - p[1], r[2] - p[2]};
  double c[3];
  cross3(u1, u2, c);
  return dot3(u1, u2) / norm3(c);
}

__device__ void inv3(const double M[9], double I[9]) {
  const double c00 = M[4] * M[8] - M[5] * M[7];
  const double c01 = M[5] * M[6] - M[3] * M[8];
  const double c02 = M[3] * M[7] - M[4] * M[6];
  const double det = M[0] * c00 + M[1] * c01 + M[2] * c02;
  const double id = 1.0 / det;
  I[0] = c00 * id;
  I[1] = (M[2] * M[7] - M[1] * M[8]) * id;
  I[2] = (M[1] * M[5] - M[2] * M[4]) * id;
  I[3] = c01 * id;
  I[4] = (M[0] * M[8] - M[2] * M[6]) * id;
  I[5] = (M[2] * M[3] - M[0] * M[5]) * id;
  I[6] = c02 * id;
  I[7] = (M[1] * M[6] - M[0] * M[7]) * id;
  I[8] = (M[0] * M[4] - M[1] * M[3]) * id;
}

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix A (row-major).
// On return A's diagonal holds eigenvalues and V's columns the eigenvectors.
__device__ void jacobi3(double A[9], double V[9]) {
  for (int k = 0; k < 9; ++k) V[k] = (k % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 12; ++sweep) {
    const double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
    const double scale = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
    if (off <= 1e-30 * scale || off == 0.0) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0;
      const int q = pq == 0 ? 1 : 2;
      const double apq = A[3 * p + q];
      if (apq == 0.0) continue;
      const double app = A[3 * p + p], aqq = A[3 * q + q];
      const double theta = (aqq - app) / (2.0 * apq);
      const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      // A <- J^T A J with J the rotation in the (p,q) plane
      for (int k = 0; k < 3; ++k) {
        const double akp = A[3 * k + p], akq = A[3 * k + q];
        A[3 * k + p] = c * akp - s * akq;
        A[3 * k + q] = s * akp + c * akq;
      }
      for (int k = 0; k < 3; ++k) {
        const double apk = A[3 * p + k], aqk = A[3 * q + k];
        A[3 * p + k] = c * apk - s * aqk;
        A[3 * q + k] = s * apk + c * aqk;
      }
      for (int k = 0; k < 3; ++k) {
        const double vkp = V[3 * k + p], vkq = V[3 * k + q];
        V[3 * k + p] = c * vkp - s * vkq;
        V[3 * k + q] = s * vkp + c * vkq;
      }
    }
  }
}

// Principal rotation log r = theta a (theta in [0, pi]) of a rotation R
// (row-major).  w = (R21 - R12, R02 - R20, R10 - R01) = 2 sin(theta) a and
// cos(theta) = (tr R - 1)/2 give theta = atan2(|w|/2, cos theta), accurate
// at both ends.  Up to pi/2, r = theta / (2 sin theta) w; beyond, the axis is
// taken from the symmetric part (R + R^T)/2 - cos(theta) I = (1 - cos theta)
// a a^T (its column with the largest diagonal, normalised) and signed to
// agree with w, whose direction no longer carries it accurately.
__device__ void rot_log(const double R[9], double r[3]) {
  const double w[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};
  const double ct = 0.5 * (R[0] + R[4] + R[8] - 1.0);
  const double sn = 0.5 * norm3(w);
  const double th = atan2(sn, ct);
  if (ct >= 0.0) {
    const double f = th < 1e-4 ? 0.5 * (1.0 + th * th / 6.0) : th / (2.0 * sn);
    for (int i = 0; i < 3; ++i) r[i] = f * w[i];
    return;
  }
  double B[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) B[3 * i + j] = 0.5 * (R[3 * i + j] + R[3 * j + i]) - (i == j ? ct : 0.0);
  int k = 0;
  if (B[4] > B[3 * k + k]) k = 1;
  if (B[8] > B[3 * k + k]) k = 2;
  const double nrm = sqrt(B[3 * k + k] * (1.0 - ct));
  double a[3] = {B[k] / nrm, B[3 + k] / nrm, B[6 + k] / nrm};
  const double sg = (a[0] * w[0] + a[1] * w[1] + a[2] * w[2]) < 0.0 ? -1.0 : 1.0;
  for (int i = 0; i < 3; ++i) r[i] = sg * th * a[i];
}

// The per-vertex transform of vertex v and the intermediate values its
// derivative needs, in FP64.
struct VFrame {
  double Qi[9], D[9], R[9], S[9], r[3];
  double nrm[3], nrmd[3];   // rest and deformed 1-ring normal sums
  double sn, w, nf, lsd;    // rest normal scale, mean cot weight, faces, deformed edge length sum
};

__device__ void vertex_frame(int v, const float *__restrict__ Vr, const float *__restrict__ Vd,
                             const int32_t *__restrict__ faces, const int32_t *__restrict__ vf_ptr,
                             const int32_t *__restrict__ vf_idx, VFrame &F) {
  double P[9] = {0}, Q[9] = {0};
  double nrm[3] = {0, 0, 0}, nrmd[3] = {0, 0, 0};
  double wsum = 0.0, ls = 0.0, lsd = 0.0;
  const double pv[3] = {Vr[3 * v], Vr[3 * v + 1], Vr[3 * v + 2]};
  const double qv[3] = {Vd[3 * v], Vd[3 * v + 1], Vd[3 * v + 2]};
  const int f0 = vf_ptr[v], f1 = vf_ptr[v + 1];
  for (int k = f0; k < f1; ++k) {
    const int f = vf_idx[k];
    const int a0 = faces[3 * f], a1 = faces[3 * f + 1], a2 = faces[3 * f + 2];
    const int ia = (a0 == v) ? a1 : (a1 == v) ? a2 : a0;
    const int ib = (a0 == v) ? a2 : (a1 == v) ? a0 : a1;
    const double pa[3] = {Vr[3 * ia], Vr[3 * ia + 1], Vr[3 * ia + 2]};
    const double pb[3] = {Vr[3 * ib], Vr[3 * ib + 1], Vr[3 * ib + 2]};
    const double qa[3] = {Vd[3 * ia], Vd[3 * ia + 1], Vd[3 * ia + 2]};
    const double qb[3] = {Vd[3 * ib], Vd[3 * ib + 1], Vd[3 * ib + 2]};
    const double cb = cot_at(pb, pv, pa), ca = cot_at(pa, pv, pb);
    double ea[3], eb[3], fa[3], fb[3];
    for (int i = 0; i < 3; ++i) {
      ea[i] = pa[i] - pv[i]; eb[i] = pb[i] - pv[i];
      fa[i] = qa[i] - qv[i]; fb[i] = qb[i] - qv[i];
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        P[3 * i + j] += 0.5 * cb * fa[i] * ea[j] + 0.5 * ca * fb[i] * eb[j];
        Q[3 * i + j] += 0.5 * cb * ea[i] * ea[j] + 0.5 * ca * eb[i] * eb[j];
      }
    wsum += 0.5 * (ca + cb);
    double c[3];
    cross3(ea, eb, c);
    for (int i = 0; i < 3; ++i) nrm[i] += c[i];
    cross3(fa, fb, c);
    for (int i = 0; i < 3; ++i) nrmd[i] += c[i];
    ls += norm3(ea) + norm3(eb);
    lsd += norm3(fa) + norm3(fb);
  }
  const double nf = (double)(f1 - f0);
  const double sn = ls / (2.0 * nf) / norm3(nrm), snd = lsd / (2.0 * nf) / norm3(nrmd);
  const double w = wsum / nf;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      P[3 * i + j] += w * (nrmd[i] * snd) * (nrm[j] * sn);
      Q[3 * i + j] += w * (nrm[i] * sn) * (nrm[j] * sn);
    }
  inv3(Q, F.Qi);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      F.D[3 * i + j] = P[3 * i] * F.Qi[j] + P[3 * i + 1] * F.Qi[3 + j] + P[3 * i + 2] * F.Qi[6 + j];
  const double *D = F.D;

  // polar decomposition through the eigenvectors of D^T D
  double M[9], E[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      M[3 * i + j] = D[i] * D[j] + D[3 + i] * D[3 + j] + D[6 + i] * D[6 + j];
  jacobi3(M, E);
  int o0 = 0, o1 = 1, o2 = 2;   // order eigenvalues descending
  double l[3] = {M[0], M[4], M[8]};
  if (l[o0] < l[o1]) { int t = o0; o0 = o1; o1 = t; }
  if (l[o1] < l[o2]) { int t = o1; o1 = o2; o2 = t; }
  if (l[o0] < l[o1]) { int t = o0; o0 = o1; o1 = t; }
  double v1[3] = {E[o0], E[3 + o0], E[6 + o0]};
  double v2[3] = {E[o1], E[3 + o1], E[6 + o1]};
  double v3[3];
  cross3(v1, v2, v3);   // proper eigenvector frame
  double u1[3], u2[3], u3[3];
  for (int i = 0; i < 3; ++i) {
    u1[i] = D[3 * i] * v1[0] + D[3 * i + 1] * v1[1] + D[3 * i + 2] * v1[2];
    u2[i] = D[3 * i] * v2[0] + D[3 * i + 1] * v2[1] + D[3 * i + 2] * v2[2];
  }
  const double n1 = norm3(u1);
  for (int i = 0; i < 3; ++i) u1[i] /= n1;
  const double pr = dot3(u1, u2);
  for (int i = 0; i < 3; ++i) u2[i] -= pr * u1[i];
  const double n2 = norm3(u2);
  for (int i = 0; i < 3; ++i) u2[i] /= n2;
  cross3(u1, u2, u3);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) F.R[3 * i + j] = u1[i] * v1[j] + u2[i] * v2[j] + u3[i] * v3[j];
  const double *R = F.R;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      F.S[3 * i + j] = R[i] * D[j] + R[3 + i] * D[3 + j] + R[6 + i] * D[6 + j];
  rot_log(R, F.r);
  for (int i = 0; i < 3; ++i) {
    F.nrm[i] = nrm[i];
    F.nrmd[i] = nrmd[i];
  }
  F.sn = sn;
  F.w = w;
  F.nf = nf;
  F.lsd = lsd;
}

__global__ __launch_bounds__(128) void vertex_frames_kernel(int nV, const float *__restrict__ Vr,
                                     const float *__restrict__ Vd,
                                     const int32_t *__restrict__ faces,
                                     const int32_t *__restrict__ vf_ptr,
                                     const int32_t *__restrict__ vf_idx,
                                     float *__restrict__ vtab) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nV) return;
  VFrame F;
  vertex_frame(v, Vr, Vd, faces, vf_ptr, vf_idx, F);
  const double *S = F.S;
  float *out = vtab + 12 * (int64_t)v;
  out[0] = Vd[3 * v] - Vr[3 * v];
  out[1] = Vd[3 * v + 1] - Vr[3 * v + 1];
  out[2] = Vd[3 * v + 2] - Vr[3 * v + 2];
  out[3] = (float)F.r[0];
  out[4] = (float)F.r[1];
  out[5] = (float)F.r[2];
  out[6] = (float)S[0];
  out[7] = (float)(0.5 * (S[1] + S[3]));
  out[8] = (float)(0.5 * (S[2] + S[6]));
  out[9] = (float)S[4];
  out[10] = (float)(0.5 * (S[5] + S[7]));
  out[11] = (float)S[8];
}

// One thread per (face, float4 of the face row): row f = rows of vertices
// faces[3f], faces[3f+1], faces[3f+2], 3 float4 each; row nF zeros.
__global__ void face_rows_kernel(int nF, const int32_t *__restrict__ faces,
                                 const float4 *__restrict__ vtab, float4 *__restrict__ ftab) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 9 * ((int64_t)nF + 1)) return;
  if (t >= 9 * (int64_t)nF) {
    ftab[t] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  const int64_t f = t / 9;
  const int j = (int)(t - 9 * f);
  const int v = faces[3 * f + j / 3];
  ftab[t] = vtab[3 * (int64_t)v + j % 3];
}

typedef float f4v __attribute__((ext_vector_type(4)));   // arrays of it stay in registers

__device__ __forceinline__ float3 interp_delta(float u, float v, float w, const f4v &a,
                                               const f4v &b, const f4v &c) {
#pragma clang fp contract(off)
  float3 d;
  d.x = (u * a.x + v * b.x) + w * c.x;
  d.y = (u * a.y + v * b.y) + w * c.y;
  d.z = (u * a.z + v * b.z) + w * c.z;
  return d;
}

__device__ __forceinline__ float3 add3(float3 a, float3 b) {
#pragma clang fp contract(off)
  return make_float3(a.x + b.x, a.y + b.y, a.z + b.z);
}

__device__ __forceinline__ float pinned_w(float u, float v) {
#pragma clang fp contract(off)
  return (1.0f - u) - v;
}

__device__ __forceinline__ float pinned_mean(float m, float s, float invk) {
#pragma clang fp contract(off)
  return m + s * invk;
}

__device__ __forceinline__ float nt_load(const float *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void nt_store(float *p, float v) { __builtin_nontemporal_store(v, p); }

// Eq. 13 for Gaussian i from its corner sums: dsum = sum_k Delta_k (pinned
// order), rs = sum_k r_k, Ss = sum_k S_k (xx, xy, xz, yy, yz, zz).
__device__ __forceinline__ void finish_gaussian(int i, float3 dsum, const float rs[3],
                                                const float Ss[6], float invk, bool any_bound,
                                                const float *__restrict__ means,
                                                const float *__restrict__ quats,
                                                const float *__restrict__ scales,
                                                float *__restrict__ means_out,
                                                float *__restrict__ quats_out,
                                                float *__restrict__ cov3d_out,
                                                float *__restrict__ xform_out) {
  // inputs read once, and the outputs the projection does not read next
  // (A, q'), are streamed (non-temporal), so they do not push the face rows
  // out of L2
  // no bound corner: the rest pose (mu' = mu bit for bit, R' = S' = I)
  const float m0 = nt_load(means + 3 * i), m1 = nt_load(means + 3 * i + 1),
              m2 = nt_load(means + 3 * i + 2);
  means_out[3 * i] = any_bound ? pinned_mean(m0, dsum.x, invk) : m0;
  means_out[3 * i + 1] = any_bound ? pinned_mean(m1, dsum.y, invk) : m1;
  means_out[3 * i + 2] = any_bound ? pinned_mean(m2, dsum.z, invk) : m2;

  // R' = exp(mean r), S' = mean S, A = R'S'
  const float r0 = rs[0] * invk, r1 = rs[1] * invk, r2 = rs[2] * invk;
  const float th2 = r0 * r0 + r1 * r1 + r2 * r2;
  const float th = sqrtf(th2);
  float sa, hb, sh_over;   // sin(th)/th, (1-cos th)/th^2, sin(th/2)/th
  if (th < 1e-2f) {
    sa = 1.0f - th2 * (1.0f / 6.0f);
    hb = 0.5f - th2 * (1.0f / 24.0f);
    sh_over = 0.5f - th2 * (1.0f / 48.0f);
  } else {
    const float sn = sinf(th), h = sinf(0.5f * th);
    sa = sn / th;
    const float q = h / (0.5f * th);
    hb = 0.5f * q * q;
    sh_over = h / th;
  }
  // R' = I + sa K + hb K^2, K = [r]_x
  const float Rp[9] = {1.f - hb * (r1 * r1 + r2 * r2), -sa * r2 + hb * r0 * r1, sa * r1 + hb * r0 * r2,
                       sa * r2 + hb * r0 * r1, 1.f - hb * (r0 * r0 + r2 * r2), -sa * r0 + hb * r1 * r2,
                       -sa * r1 + hb * r0 * r2, sa * r0 + hb * r1 * r2, 1.f - hb * (r0 * r0 + r1 * r1)};
  const float sd = any_bound ? 0.f : 1.f;   // rs = Ss = 0 without a bound corner
  const float Sm[9] = {Ss[0] * invk + sd, Ss[1] * invk, Ss[2] * invk, Ss[1] * invk,
                       Ss[3] * invk + sd, Ss[4] * invk, Ss[2] * invk, Ss[4] * invk,
                       Ss[5] * invk + sd};
  float A[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      A[3 * r + c] = Rp[3 * r] * Sm[c] + Rp[3 * r + 1] * Sm[3 + c] + Rp[3 * r + 2] * Sm[6 + c];

  float qw = nt_load(quats + 4 * i), qx = nt_load(quats + 4 * i + 1), qy = nt_load(quats + 4 * i + 2),
        qz = nt_load(quats + 4 * i + 3);
  const float qn = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= qn; qx *= qn; qy *= qn; qz *= qn;
  const float Rq[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                       2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                       2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
  const float s0 = nt_load(scales + 3 * i), s1 = nt_load(scales + 3 * i + 1),
              s2 = nt_load(scales + 3 * i + 2);
  // B = A R(q) diag(s); Sigma' = B B^T
  float B[9];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    B[3 * r] = (A[3 * r] * Rq[0] + A[3 * r + 1] * Rq[3] + A[3 * r + 2] * Rq[6]) * s0;
    B[3 * r + 1] = (A[3 * r] * Rq[1] + A[3 * r + 1] * Rq[4] + A[3 * r + 2] * Rq[7]) * s1;
    B[3 * r + 2] = (A[3 * r] * Rq[2] + A[3 * r + 1] * Rq[5] + A[3 * r + 2] * Rq[8]) * s2;
  }
  float *cv = cov3d_out + 6 * (int64_t)i;
  cv[0] = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  cv[1] = B[0] * B[3] + B[1] * B[4] + B[2] * B[5];
  cv[2] = B[0] * B[6] + B[1] * B[7] + B[2] * B[8];
  cv[3] = B[3] * B[3] + B[4] * B[4] + B[5] * B[5];
  cv[4] = B[3] * B[6] + B[4] * B[7] + B[5] * B[8];
  cv[5] = B[6] * B[6] + B[7] * B[7] + B[8] * B[8];
  if (xform_out) {
#pragma unroll
    for (int k = 0; k < 9; ++k) nt_store(xform_out + 9 * (int64_t)i + k, A[k]);
  }
  if (quats_out) {
    const float pw = cosf(0.5f * th), px = sh_over * r0, py = sh_over * r1, pz = sh_over * r2;
    float *qo = quats_out + 4 * (int64_t)i;
    nt_store(qo + 0, pw * qw - px * qx - py * qy - pz * qz);
    nt_store(qo + 1, pw * qx + px * qw + py * qz - pz * qy);
    nt_store(qo + 2, pw * qy - px * qz + py * qw + pz * qx);
    nt_store(qo + 3, pw * qz + px * qy - py * qx + pz * qw);
  }
}

// Transfer kernel: one lane per Gaussian, its K bound points taken in K
// rounds.  In round k the wave first gathers the 64 face rows it needs
// (corner k of each of its Gaussians) into its own LDS block: the 576 float4
// are read in 9 instructions, lane L taking slot s = 64 m + L (row s / 9,
// part s % 9), so one instruction reads about seven whole rows, i.e. some 15
// cache lines, where one row per lane would touch 64.  Each lane then reads
// its row from LDS and adds Eq. 12's terms in corner order (the pinned order
// of the mean offset); the next round's rows are already loading meanwhile.
// A lane finally applies Eq. 13 to its own Gaussian.
constexpr int kTrRows = 64;   // Gaussians per wave (one wave per block)

__device__ __forceinline__ void gather_rows(const f4v *__restrict__ ftab, int nF, int face, int lane,
                                            f4v (&buf)[9]) {
#pragma unroll
  for (int m = 0; m < 9; ++m) {
    const int s = 64 * m + lane;
    const int row = s / 9;
    int f = __shfl(face, row, 64);
    f = (unsigned)f < (unsigned)nF ? f : nF;      // unbound: the zero row
    buf[m] = ftab[9 * (int64_t)f + (s - 9 * row)];
  }
}

// 1/k_b rounded to FP32 for k_b = 0..8 bound corners (0 unused)
__device__ __forceinline__ float inv_bound(int kb) {
  constexpr float t[9] = {0.f, 1.f, 1.f / 2, 1.f / 3, 1.f / 4, 1.f / 5, 1.f / 6, 1.f / 7, 1.f / 8};
  float r = t[0];
#pragma unroll
  for (int k = 1; k < 9; ++k) r = kb == k ? t[k] : r;
  return r;
}

// Backward finish of Gaussian i (BWD instantiation of the transfer kernel):
// from the corner sums rs, Ss and dL/dmu', dL/dA, the row
// g = (dL/dmu', dL/d rbar, sym dL/dS') / k_b its corners pass on (zero
// without a bound corner), through Eq. 13:
//   dL/dS' = R'^T dL/dA,  dL/dR' = dL/dA S'^T,
//   dL/d rbar = J_r(rbar)^T vee(R'^T dL/dR' - dL/dR'^T R')   (R' = exp(rbar)).
__device__ __forceinline__ void finish_backward(int i, const float rs[3], const float Ss[6],
                                                float invk, bool any_bound,
                                                const float *__restrict__ dmu,
                                                const float *__restrict__ dA,
                                                float *__restrict__ gG) {
  // rows of kGRow floats (64 B, aligned): the per-face pass gathers each
  // in one memory sector
  float4 *go4 = reinterpret_cast<float4 *>(gG + kGRow * (int64_t)i);
  if (!any_bound) {                    // rest pose: no dependence on the proxy
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    go4[0] = z;
    go4[1] = z;
    go4[2] = z;
    return;
  }
  const float r0 = rs[0] * invk, r1 = rs[1] * invk, r2 = rs[2] * invk;
  const float th2 = r0 * r0 + r1 * r1 + r2 * r2, th = sqrtf(th2);
  float sa, hb, cb;   // sin(th)/th, (1 - cos th)/th^2, (th - sin th)/th^3
  if (th < 1e-2f) {
    sa = 1.0f - th2 * (1.0f / 6.0f);
    hb = 0.5f - th2 * (1.0f / 24.0f);
    cb = 1.0f / 6.0f - th2 * (1.0f / 120.0f);
  } else {
    const float sn = sinf(th), h = sinf(0.5f * th);
    sa = sn / th;
    const float q = h / (0.5f * th);
    hb = 0.5f * q * q;
    cb = (1.0f - sa) / th2;
  }
  const float Rp[9] = {1.f - hb * (r1 * r1 + r2 * r2), -sa * r2 + hb * r0 * r1, sa * r1 + hb * r0 * r2,
                       sa * r2 + hb * r0 * r1, 1.f - hb * (r0 * r0 + r2 * r2), -sa * r0 + hb * r1 * r2,
                       -sa * r1 + hb * r0 * r2, sa * r0 + hb * r1 * r2, 1.f - hb * (r0 * r0 + r1 * r1)};
  const float Sm[9] = {Ss[0] * invk, Ss[1] * invk, Ss[2] * invk, Ss[1] * invk, Ss[3] * invk,
                       Ss[4] * invk, Ss[2] * invk, Ss[4] * invk, Ss[5] * invk};
  float GA[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) GA[k] = dA ? nt_load(dA + 9 * (int64_t)i + k) : 0.0f;
  float GS[9], GR[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      GS[3 * a + b] = Rp[a] * GA[b] + Rp[3 + a] * GA[3 + b] + Rp[6 + a] * GA[6 + b];           // R'^T GA
      GR[3 * a + b] = GA[3 * a] * Sm[b] + GA[3 * a + 1] * Sm[3 + b] + GA[3 * a + 2] * Sm[6 + b];  // GA S'^T
    }
  float X[9];   // R'^T GR
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) X[3 * a + b] = Rp[a] * GR[b] + Rp[3 + a] * GR[3 + b] + Rp[6 + a] * GR[6 + b];
  const float y[3] = {X[7] - X[5], X[2] - X[6], X[3] - X[1]};
  // J_r(r)^T y = y + hb r x y + cb r x (r x y)
  const float rxy[3] = {r1 * y[2] - r2 * y[1], r2 * y[0] - r0 * y[2], r0 * y[1] - r1 * y[0]};
  const float rxrxy[3] = {r1 * rxy[2] - r2 * rxy[1], r2 * rxy[0] - r0 * rxy[2], r0 * rxy[1] - r1 * rxy[0]};
  float go[12];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    go[q] = (dmu ? nt_load(dmu + 3 * (int64_t)i + q) : 0.0f) * invk;
    go[3 + q] = (y[q] + hb * rxy[q] + cb * rxrxy[q]) * invk;
  }
  go[6] = GS[0] * invk;
  go[7] = 0.5f * (GS[1] + GS[3]) * invk;
  go[8] = 0.5f * (GS[2] + GS[6]) * invk;
  go[9] = GS[4] * invk;
  go[10] = 0.5f * (GS[5] + GS[7]) * invk;
  go[11] = GS[8] * invk;
  go4[0] = make_float4(go[0], go[1], go[2], go[3]);
  go4[1] = make_float4(go[4], go[5], go[6], go[7]);
  go4[2] = make_float4(go[8], go[9], go[10], go[11]);
}

// Arguments of the backward instantiation (unused by the forward one).
struct TransferBwdArgs {
  const float *dmu, *dA;     // dL/dmu' (N,3), dL/dA (N,9); NULL: zero
  float *gG;                 // (N, kGRow) rows: g's 12 terms, padded to 64 B
  uint32_t *keys, *vals;     // per corner: its face (nF: unbound) and its index
};

template <int K, bool BWD = false>
__global__ __launch_bounds__(kTrRows) __attribute__((amdgpu_waves_per_eu(4))) void transfer_kernel(
    int N, int nF, const float4 *__restrict__ ftab, const int32_t *__restrict__ bind_face,
    const float *__restrict__ bind_bary, const float *__restrict__ means,
    const float *__restrict__ quats, const float *__restrict__ scales,
    float *__restrict__ means_out, float *__restrict__ quats_out, float *__restrict__ cov3d_out,
    float *__restrict__ xform_out, TransferBwdArgs bw = {}) {
  __shared__ f4v rows[kTrRows * 9];
  __shared__ int n_bound[kTrRows];
  const f4v *__restrict__ ftab4 = reinterpret_cast<const f4v *>(ftab);
  const int lane = threadIdx.x;
  const int i = blockIdx.x * kTrRows + lane;
  const bool valid = i < N;
  // this lane's K bindings (face 0 stands in past the end: its row is read
  // and the result dropped)
  int face[K];
  float bu[K], bv[K];
  if constexpr (K == 8) {
    // read once: streamed past the caches the face rows live in
    typedef int i4v __attribute__((ext_vector_type(4)));
    i4v f0 = {0, 0, 0, 0}, f1 = f0;
    f4v b0 = {0.f, 0.f, 0.f, 0.f}, b1 = b0, b2 = b0, b3 = b0;
    if (valid) {
      const i4v *fp = reinterpret_cast<const i4v *>(bind_face) + 2 * (int64_t)i;
      const f4v *bp = reinterpret_cast<const f4v *>(bind_bary) + 4 * (int64_t)i;
      f0 = __builtin_nontemporal_load(fp);
      f1 = __builtin_nontemporal_load(fp + 1);
      b0 = __builtin_nontemporal_load(bp);
      b1 = __builtin_nontemporal_load(bp + 1);
      b2 = __builtin_nontemporal_load(bp + 2);
      b3 = __builtin_nontemporal_load(bp + 3);
    }
    face[0] = f0.x; face[1] = f0.y; face[2] = f0.z; face[3] = f0.w;
    face[4] = f1.x; face[5] = f1.y; face[6] = f1.z; face[7] = f1.w;
    bu[0] = b0.x; bv[0] = b0.y; bu[1] = b0.z; bv[1] = b0.w;
    bu[2] = b1.x; bv[2] = b1.y; bu[3] = b1.z; bv[3] = b1.w;
    bu[4] = b2.x; bv[4] = b2.y; bu[5] = b2.z; bv[5] = b2.w;
    bu[6] = b3.x; bv[6] = b3.y; bu[7] = b3.z; bv[7] = b3.w;
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      face[k] = valid ? bind_face[K * (int64_t)i + k] : 0;
      bu[k] = valid ? bind_bary[2 * (K * (int64_t)i + k)] : 0.f;
      bv[k] = valid ? bind_bary[2 * (K * (int64_t)i + k) + 1] : 0.f;
    }
  }
  // an unbound corner (face outside [0, nF)) gathers the all-zero row nF:
  // with finite barycentrics its terms are exact zeros, which leave every
  // sum, the pinned mean offset included, as it is.  The count of bound
  // corners waits in LDS for Eq. 13 (registers are short in the rounds).
  {
    int kb = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) kb += (unsigned)face[k] < (unsigned)nF ? 1 : 0;
    n_bound[lane] = kb;
  }
  if constexpr (BWD) {
    if (valid) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int64_t c = K * (int64_t)i + k;
        bw.keys[c] = (unsigned)face[k] < (unsigned)nF ? (uint32_t)face[k] : (uint32_t)nF;
        bw.vals[c] = (uint32_t)c;
      }
    }
  }
  float3 ds = make_float3(0.f, 0.f, 0.f);
  float rs[3] = {0.f, 0.f, 0.f}, Ss[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  f4v buf[9];
  gather_rows(ftab4, nF, face[0], lane, buf);
  // one round per bound point; the bindings shift down one place per round,
  // so every index below is static
  auto round = [&](bool prefetch) {
#pragma unroll
    for (int m = 0; m < 9; ++m) rows[64 * m + lane] = buf[m];
    __syncthreads();
    if (prefetch) gather_rows(ftab4, nF, face[K > 1 ? 1 : 0], lane, buf);
    const f4v *row = rows + 9 * lane;
    const f4v a0 = row[0], a1 = row[1], a2 = row[2];
    const f4v b0 = row[3], b1 = row[4], b2 = row[5];
    const f4v c0 = row[6], c1 = row[7], c2 = row[8];
    const float u = bu[0], v = bv[0], w = pinned_w(u, v);
    const float3 di = interp_delta(u, v, w, a0, b0, c0);
    // pinned order: the bound corners' offsets added in corner order (0 + x
    // and x + 0 are exact, so the zero start and unbound corners change nothing)
    ds = add3(ds, di);
    rs[0] += u * a0.w + v * b0.w + w * c0.w;
    rs[1] += u * a1.x + v * b1.x + w * c1.x;
    rs[2] += u * a1.y + v * b1.y + w * c1.y;
    Ss[0] += u * a1.z + v * b1.z + w * c1.z;
    Ss[1] += u * a1.w + v * b1.w + w * c1.w;
    Ss[2] += u * a2.x + v * b2.x + w * c2.x;
    Ss[3] += u * a2.y + v * b2.y + w * c2.y;
    Ss[4] += u * a2.z + v * b2.z + w * c2.z;
    Ss[5] += u * a2.w + v * b2.w + w * c2.w;
#pragma unroll
    for (int j = 0; j + 1 < K; ++j) {
      face[j] = face[j + 1];
      bu[j] = bu[j + 1];
      bv[j] = bv[j + 1];
    }
    __syncthreads();
  };
  if constexpr (K > 1) {
#pragma unroll 1
    for (int k = 0; k + 1 < K; ++k) round(true);
  }
  round(false);
  const int kb = n_bound[lane];
  if constexpr (BWD) {
    if (valid) finish_backward(i, rs, Ss, inv_bound(kb), kb > 0, bw.dmu, bw.dA, bw.gG);
  } else {
    if (valid)
      finish_gaussian(i, ds, rs, Ss, inv_bound(kb), kb > 0, means, quats, scales, means_out,
                      quats_out, cov3d_out, xform_out);
  }
}


// ---- backward: the gradient with respect to the deformed proxy ------------
//
// The transfer kernel's backward instantiation (one lane per Gaussian, the
// same gather rounds) forms each Gaussian's row g = (dL/dmu', dL/d rbar,
// sym dL/dS') / k_b (finish_backward) and one sort key per corner (its
// face; nF when unbound); Eq. 12 hands the corner's face vertex j the share
// b_j g.  The corners are sorted by face (the frame's radix sort) and
// transfer_bwd_faces_kernel sums the shares of each run of one face within
// a wave, adding 36 floats per run to a per-face table.
// vertex_bwd_kernel (one thread per vertex, FP64): with r = log R,
// D = R S (polar), D = P Q^-1, the vertex's (dL/dDelta, dL/dr, G = dL/dS)
// become
//   h = J_r(r)^-T dL/dr,   m = (tr(S) I - S)^-1 (h + vee(S G - G S)),
//   dL/dD = R ([m]_x + G),  dL/dP = dL/dD Q^-T,
// (the differential of the polar factor: R^T dR = [w]_x with
// (tr(S) I - S) w = vee(R^T dD - dD^T R), dS = R^T dD - [w]_x S), then
// P's 1-ring edge terms and its normal pair pass dL/dP to the deformed
// edges f = V'_a - V'_v (through the cross products and edge lengths of the
// deformed normal), i.e. to V' of the vertex and its neighbours.

// Per-face sums of the sorted corners: one lane per corner computes its
// face's three vertex shares (u g, v g, w g) (36 floats) into LDS; the
// wave's runs of equal faces (ballot of the lanes where the face changes)
// are then summed column by column by lanes 0..35 and added to the face's
// row of the table with one float atomic per column and run.
__global__ __launch_bounds__(64) void transfer_bwd_faces_kernel(
    int64_t M, int K, int nF, const uint32_t *__restrict__ skeys, const uint32_t *__restrict__ svals,
    const float *__restrict__ gG, const float *__restrict__ bind_bary, float *__restrict__ ff) {
  __shared__ float part[64 * 37];      // row stride 37: the column sums hit distinct banks
  const int lane = threadIdx.x;
  const int64_t j = (int64_t)blockIdx.x * 64 + lane;
  uint32_t f = (uint32_t)nF;
  if (j < M) f = skeys[j];
  const bool live = f < (uint32_t)nF;
  float *row = part + 37 * lane;
  if (live) {
    const uint32_t c = svals[j];
    const float u = bind_bary[2 * (int64_t)c], v = bind_bary[2 * (int64_t)c + 1];
    const float w = (1.0f - u) - v;
    const float4 *g4 = reinterpret_cast<const float4 *>(gG + kGRow * (int64_t)(c / (uint32_t)K));
    const float4 ga = g4[0], gb = g4[1], gc = g4[2];
    const float g[12] = {ga.x, ga.y, ga.z, ga.w, gb.x, gb.y, gb.z, gb.w, gc.x, gc.y, gc.z, gc.w};
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      const float gq = g[q];
      row[q] = u * gq;
      row[12 + q] = v * gq;
      row[24 + q] = w * gq;
    }
  }
  const uint32_t prev = __shfl_up(f, 1, 64);
  const uint64_t heads = __ballot(live && (lane == 0 || prev != f));
  const uint64_t lives = __ballot(live);
  __syncthreads();
  uint64_t h = heads;
  while (h) {
    const int a = __builtin_ctzll(h);
    h &= h - 1;
    // the run ends at the next head or at the last live lane
    const int b = h ? __builtin_ctzll(h) : 64 - __builtin_clzll(lives);
    const uint32_t fa = __shfl(f, a, 64);
    if (lane < 36) {
      float sum = 0.0f;
      for (int l = a; l < b; ++l) sum += part[37 * l + lane];
      if (sum != 0.0f) unsafeAtomicAdd(ff + 36 * (int64_t)fa + lane, sum);
    }
  }
}

__global__ __launch_bounds__(128) void vertex_bwd_kernel(
    int nV, const float *__restrict__ Vr, const float *__restrict__ Vd,
    const int32_t *__restrict__ faces, const int32_t *__restrict__ vf_ptr,
    const int32_t *__restrict__ vf_idx, const float *__restrict__ ff, float *__restrict__ dV) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nV) return;
  // the vertex's (dL/dDelta, dL/dr, dL/dS): its slot of each incident face's sums
  double g[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = vf_ptr[v]; k < vf_ptr[v + 1]; ++k) {
    const int f = vf_idx[k];
    const int j = faces[3 * f] == v ? 0 : faces[3 * f + 1] == v ? 1 : 2;
    const float *src = ff + 36 * (int64_t)f + 12 * j;
    for (int c = 0; c < 12; ++c) g[c] += src[c];
  }
  bool any = false;
  for (int c = 0; c < 12; ++c) any = any || g[c] != 0.0;
  if (!any) return;
  VFrame F;
  vertex_frame(v, Vr, Vd, faces, vf_ptr, vf_idx, F);
  const double *R = F.R, *S = F.S, *r = F.r;
  // h = J_r(r)^-T g_r = g_r - r x g_r / 2 + beta r x (r x g_r)
  const double th2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2], th = sqrt(th2);
  const double beta = th < 1e-4 ? 1.0 / 12.0 + th2 / 720.0
                                : (1.0 - 0.5 * th * cos(0.5 * th) / sin(0.5 * th)) / th2;
  const double gr[3] = {g[3], g[4], g[5]};
  double rxg[3], rxrxg[3];
  cross3(r, gr, rxg);
  cross3(r, rxg, rxrxg);
  double k3[3];
  for (int c = 0; c < 3; ++c) k3[c] = gr[c] - 0.5 * rxg[c] + beta * rxrxg[c];
  const double G[9] = {g[6], g[7], g[8], g[7], g[9], g[10], g[8], g[10], g[11]};
  double SG[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      SG[3 * a + b] = S[3 * a] * G[b] + S[3 * a + 1] * G[3 + b] + S[3 * a + 2] * G[6 + b];
  // vee(S G - G S) = vee(SG - SG^T) (S, G symmetric)
  k3[0] += SG[7] - SG[5];
  k3[1] += SG[2] - SG[6];
  k3[2] += SG[3] - SG[1];
  const double trS = S[0] + S[4] + S[8];
  double Y[9], Yi[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Y[3 * a + b] = (a == b ? trS : 0.0) - 0.5 * (S[3 * a + b] + S[3 * b + a]);
  inv3(Y, Yi);
  double m[3];
  for (int a = 0; a < 3; ++a) m[a] = Yi[3 * a] * k3[0] + Yi[3 * a + 1] * k3[1] + Yi[3 * a + 2] * k3[2];
  const double Mx[9] = {G[0], G[1] - m[2], G[2] + m[1], G[3] + m[2], G[4], G[5] - m[0],
                        G[6] - m[1], G[7] + m[0], G[8]};   // [m]_x + G
  double GD[9], GP[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      GD[3 * a + b] = R[3 * a] * Mx[b] + R[3 * a + 1] * Mx[3 + b] + R[3 * a + 2] * Mx[6 + b];
  for (int a = 0; a < 3; ++a)      // dL/dP = dL/dD Q^-T
    for (int b = 0; b < 3; ++b)
      GP[3 * a + b] = GD[3 * a] * F.Qi[3 * b] + GD[3 * a + 1] * F.Qi[3 * b + 1] + GD[3 * a + 2] * F.Qi[3 * b + 2];
  // the normal pair w n' n^T, n = nrm sn, n' = u l' / |u| (u = nrmd, l' the mean deformed edge length)
  double nrest[3], dnp[3];
  for (int c = 0; c < 3; ++c) nrest[c] = F.nrm[c] * F.sn;
  for (int a = 0; a < 3; ++a)
    dnp[a] = F.w * (GP[3 * a] * nrest[0] + GP[3 * a + 1] * nrest[1] + GP[3 * a + 2] * nrest[2]);
  const double nu = norm3(F.nrmd), lp = F.lsd / (2.0 * F.nf);
  double uh[3];
  for (int c = 0; c < 3; ++c) uh[c] = F.nrmd[c] / nu;
  const double dl = dot3(uh, dnp);
  double du[3];
  for (int c = 0; c < 3; ++c) du[c] = lp / nu * (dnp[c] - uh[c] * dl);
  const double dlsd = dl / (2.0 * F.nf);

  double acc[3] = {g[0], g[1], g[2]};   // Delta_v = V'_v - V_v
  const double pv[3] = {Vr[3 * v], Vr[3 * v + 1], Vr[3 * v + 2]};
  const double qv[3] = {Vd[3 * v], Vd[3 * v + 1], Vd[3 * v + 2]};
  for (int k = vf_ptr[v]; k < vf_ptr[v + 1]; ++k) {
    const int f = vf_idx[k];
    const int a0 = faces[3 * f], a1 = faces[3 * f + 1], a2 = faces[3 * f + 2];
    const int ia = (a0 == v) ? a1 : (a1 == v) ? a2 : a0;
    const int ib = (a0 == v) ? a2 : (a1 == v) ? a0 : a1;
    const double pa[3] = {Vr[3 * ia], Vr[3 * ia + 1], Vr[3 * ia + 2]};
    const double pb[3] = {Vr[3 * ib], Vr[3 * ib + 1], Vr[3 * ib + 2]};
    const double cb = cot_at(pb, pv, pa), ca = cot_at(pa, pv, pb);
    double ea[3], eb[3], fa[3], fb[3];
    for (int c = 0; c < 3; ++c) {
      ea[c] = pa[c] - pv[c]; eb[c] = pb[c] - pv[c];
      fa[c] = Vd[3 * ia + c] - qv[c]; fb[c] = Vd[3 * ib + c] - qv[c];
    }
    double t1[3], t2[3];
    cross3(fb, du, t1);   // from u = sum fa x fb
    cross3(du, fa, t2);
    const double la = norm3(fa), lb = norm3(fb);
    double gfa[3], gfb[3];
    for (int a = 0; a < 3; ++a) {
      gfa[a] = 0.5 * cb * (GP[3 * a] * ea[0] + GP[3 * a + 1] * ea[1] + GP[3 * a + 2] * ea[2]) + t1[a] +
               dlsd * fa[a] / la;
      gfb[a] = 0.5 * ca * (GP[3 * a] * eb[0] + GP[3 * a + 1] * eb[1] + GP[3 * a + 2] * eb[2]) + t2[a] +
               dlsd * fb[a] / lb;
    }
    for (int c = 0; c < 3; ++c) {
      unsafeAtomicAdd(dV + 3 * (int64_t)ia + c, (float)gfa[c]);
      unsafeAtomicAdd(dV + 3 * (int64_t)ib + c, (float)gfb[c]);
      acc[c] -= gfa[c] + gfb[c];
    }
  }
  for (int c = 0; c < 3; ++c) unsafeAtomicAdd(dV + 3 * (int64_t)v + c, (float)acc[c]);
}

}  // namespace

// The transfer's launches with the per-vertex table at vtab and the face rows
// at ftab; timed launches report to the context's profiler.
static hipError_t transfer_launches(Ctx *c, const float *V_def, int32_t N,
                                    const int32_t *bind_face, const float *bind_bary,
                                    const float *means, const float *quats, const float *scales,
                                    float *means_out, float *quats_out, float *cov3d_out,
                                    float *xform_out, float *vtab, float4 *ftab, bool timed) {
  hipError_t e;
  {
    ScopedTimer t(c, timed ? K_VERTEX_FRAMES : -1);
    hipLaunchKernelGGL(vertex_frames_kernel, dim3(ceil_div(c->nV, 128)), dim3(128), 0, c->stream,
                       c->nV, (const float *)c->V_rest.p, V_def, (const int32_t *)c->faces.p,
                       (const int32_t *)c->vf_ptr.p, (const int32_t *)c->vf_idx.p, vtab);
    e = hipGetLastError();
    if (e == hipSuccess && N > 0) {
      hipLaunchKernelGGL(face_rows_kernel, dim3((unsigned)ceil_div(9 * ((int64_t)c->nF + 1), 256)),
                         dim3(256), 0, c->stream, c->nF, (const int32_t *)c->faces.p,
                         (const float4 *)vtab, ftab);
      e = hipGetLastError();
    }
  }
  if (e != hipSuccess || N == 0) return e;
  ScopedTimer tt(c, timed ? K_TRANSFER : -1);
  const dim3 grid(ceil_div(N, kTrRows)), block(kTrRows);
  if (c->opt.k_bind == 8)
    hipLaunchKernelGGL(transfer_kernel<8>, grid, block, 0, c->stream, N, c->nF, (const float4 *)ftab,
                       bind_face, bind_bary, means, quats, scales, means_out, quats_out, cov3d_out,
                       xform_out);
  else
    hipLaunchKernelGGL(transfer_kernel<1>, grid, block, 0, c->stream, N, c->nF, (const float4 *)ftab,
                       bind_face, bind_bary, means, quats, scales, means_out, quats_out, cov3d_out,
                       xform_out);
  return hipGetLastError();
}

hipError_t launch_transfer_backward(Ctx *c, const float *V_def, int32_t N,
                                    const int32_t *bind_face, const float *bind_bary,
                                    const float *dL_dmeans, const float *dL_dxform,
                                    float *dL_dV_def, bool accumulate) {
  float *vtab = (float *)c->vtab.p;
  float *ff = (float *)c->tb_face.p;
  const int K = c->opt.k_bind;
  const int64_t M = (int64_t)N * K;
  hipError_t e = hipSuccess;
  if (!accumulate) e = launch_fill_u32(c, (uint32_t *)dL_dV_def, 3 * (int64_t)c->nV, 0u);
  if (e == hipSuccess) e = launch_fill_u32(c, (uint32_t *)ff, 36 * (int64_t)c->nF, 0u);
  if (e != hipSuccess) return e;
  ScopedTimer t(c, K_TRANSFER_BWD);
  hipLaunchKernelGGL(vertex_frames_kernel, dim3(ceil_div(c->nV, 128)), dim3(128), 0, c->stream,
                     c->nV, (const float *)c->V_rest.p, V_def, (const int32_t *)c->faces.p,
                     (const int32_t *)c->vf_ptr.p, (const int32_t *)c->vf_idx.p, vtab);
  hipLaunchKernelGGL(face_rows_kernel, dim3((unsigned)ceil_div(9 * ((int64_t)c->nF + 1), 256)),
                     dim3(256), 0, c->stream, c->nF, (const int32_t *)c->faces.p,
                     (const float4 *)vtab, (float4 *)c->ftab.p);
  if (N > 0) {
    uint32_t *keys[2] = {(uint32_t *)c->tb_key[0].p, (uint32_t *)c->tb_key[1].p};
    uint32_t *vals[2] = {(uint32_t *)c->tb_val[0].p, (uint32_t *)c->tb_val[1].p};
    float *gG = (float *)c->tb_g.p;
    const dim3 grid(ceil_div(N, kTrRows)), block(kTrRows);
    const TransferBwdArgs ba = {dL_dmeans, dL_dxform, gG, keys[0], vals[0]};
    if (K == 8)
      hipLaunchKernelGGL((transfer_kernel<8, true>), grid, block, 0, c->stream, N, c->nF,
                         (const float4 *)c->ftab.p, bind_face, bind_bary, nullptr, nullptr, nullptr,
                         nullptr, nullptr, nullptr, nullptr, ba);
    else
      hipLaunchKernelGGL((transfer_kernel<1, true>), grid, block, 0, c->stream, N, c->nF,
                         (const float4 *)c->ftab.p, bind_face, bind_bary, nullptr, nullptr, nullptr,
                         nullptr, nullptr, nullptr, nullptr, ba);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int bits = 1;
    while ((1ll << bits) <= (int64_t)c->nF) ++bits;   // keys 0..nF
    if ((e = launch_radix_sort_u32(c, keys, vals, (uint64_t)M, nullptr, nullptr, bits, -1, -1, -1)) !=
        hipSuccess)
      return e;
    const int res = radix_passes(bits) & 1;
    hipLaunchKernelGGL(transfer_bwd_faces_kernel, dim3((unsigned)ceil_div(M, 64)),
                       dim3(64), 0, c->stream, M, K, c->nF, (const uint32_t *)keys[res],
                       (const uint32_t *)vals[res], (const float *)gG, bind_bary, ff);
  }
  hipLaunchKernelGGL(vertex_bwd_kernel, dim3(ceil_div(c->nV, 128)), dim3(128), 0, c->stream, c->nV,
                     (const float *)c->V_rest.p, V_def, (const int32_t *)c->faces.p,
                     (const int32_t *)c->vf_ptr.p, (const int32_t *)c->vf_idx.p, (const float *)ff,
                     dL_dV_def);
  return hipGetLastError();
}

hipError_t launch_transfer(Ctx *c, const float *V_def, int32_t N, const int32_t *bind_face,
                           const float *bind_bary, const float *means, const float *quats,
                           const float *scales, float *means_out, float *quats_out,
                           float *cov3d_out, float *xform_out, float *vertex_out) {
  float *vtab = vertex_out ? vertex_out : (float *)c->vtab.p;
  return transfer_launches(c, V_def, N, bind_face, bind_bary, means, quats, scales, means_out,
                           quats_out, cov3d_out, xform_out, vtab, (float4 *)c->ftab.p, true);
}

hipError_t launch_transfer_noalloc(Ctx *c, void *scratch_base, const float *V_def, int32_t N,
                                   const int32_t *bind_face, const float *bind_bary,
                                   const float *means, const float *quats, const float *scales,
                                   float *means_out, float *quats_out, float *cov3d_out,
                                   float *xform_out, float *vertex_out) {
  unsigned char *base = (unsigned char *)scratch_base;
  float *vtab = vertex_out ? vertex_out : (float *)base;
  const size_t ftab_off = vertex_out ? 0 : noalloc_transfer_bytes(c->nV, 0, true);
  return transfer_launches(c, V_def, N, bind_face, bind_bary, means, quats, scales, means_out,
                           quats_out, cov3d_out, xform_out, vtab, (float4 *)(base + ftab_off),
                           false);
}

}  // namespace umgs
