// Host side of the C ABI: contexts, argument validation, work buffers and
// the entry points declared in unimgs.h.
#include <stdarg.h>
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>

#include "internal.h"

namespace umgs {

umgs_status fail(Ctx *c, umgs_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return s;
}

umgs_status hip_check(Ctx *c, hipError_t e, const char *what) {
  if (e == hipSuccess) return UMGS_OK;
  return fail(c, UMGS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

umgs_status ensure(Ctx *c, DevBuf &b, size_t bytes, const char *what) {
  if (bytes <= b.cap) return UMGS_OK;
  if (c->capturing)
    return fail(c, UMGS_ERR_CAPACITY, "%s: %zu bytes needed while capturing (reserve or render "
                "an eager frame of this size first)", what, bytes);
  if (b.p) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_check(c, e, "stream sync before reallocation");
    (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
  }
  size_t cap = bytes + bytes / 8 + 256;
  hipError_t e = hipMalloc(&b.p, cap);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(c, UMGS_ERR_CAPACITY, "allocation of %zu bytes for %s failed: %s", cap, what,
                hipGetErrorString(e));
  }
  b.cap = cap;
  return UMGS_OK;
}

static void free_buf(DevBuf &b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}

static bool valid_options(const umgs_options *o, std::string &why) {
  const bool tile_ok = (o->tile_w == 16 && o->tile_h == 16) || (o->tile_w == 8 && o->tile_h == 8) ||
                       (o->tile_w == 32 && o->tile_h == 8);
  if (!tile_ok) { why = "tile shape must be 8x8, 16x16 or 32x8"; return false; }
  const int b = o->frag_batch;
  if (!(b == 32 || b == 64 || b == 128 || b == 256)) { why = "frag_batch must be 32, 64, 128 or 256"; return false; }
  if (o->sh_degree < 0 || o->sh_degree > 3) { why = "sh_degree must be 0..3"; return false; }
  if (!(o->k_bind == 1 || o->k_bind == 8)) { why = "k_bind must be 1 or 8"; return false; }
  if (o->mode < UMGS_MODE_UNIMGS || o->mode > UMGS_MODE_LITERAL_T) { why = "unknown mode"; return false; }
  if (o->schedule != UMGS_SCHEDULE_TILE_GRID && o->schedule != UMGS_SCHEDULE_PERSISTENT) { why = "unknown schedule"; return false; }
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(o->bg[k])) { why = "background must be finite"; return false; }
  return true;
}

static hipEvent_t get_event(Ctx *c) {
  if (!c->prof.pool.empty()) {
    hipEvent_t e = c->prof.pool.back();
    c->prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ScopedTimer::ScopedTimer(Ctx *ctx, int kid) : c(ctx), id(kid) {
  if (!c->prof.on || kid < 0) return;
  a = get_event(c);
  b = get_event(c);
  if (a && b) (void)hipEventRecord(a, c->stream);
}

ScopedTimer::~ScopedTimer() {
  if (!c->prof.on || !a || !b) return;
  (void)hipEventRecord(b, c->stream);
  c->prof.pending.push_back({id, a, b});
}

static umgs_status drain_profile(Ctx *c) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_check(c, e, "profiler sync");
  for (auto &p : c->prof.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->prof.ms[p.id] += ms;
      c->prof.n[p.id] += 1;
    }
    c->prof.pool.push_back(p.a);
    c->prof.pool.push_back(p.b);
  }
  c->prof.pending.clear();
  return UMGS_OK;
}

}  // namespace umgs

using namespace umgs;

extern "C" {

void umgs_default_options(umgs_options *opt) {
  if (!opt) return;
  opt->tile_w = 16;
  opt->tile_h = 16;
  opt->frag_batch = 128;
  opt->sh_degree = 0;
  opt->k_bind = 8;
  opt->mode = UMGS_MODE_UNIMGS;
  opt->schedule = UMGS_SCHEDULE_TILE_GRID;
  opt->bg[0] = opt->bg[1] = opt->bg[2] = 0.0f;
}

umgs_status umgs_create(umgs_ctx **out, const umgs_options *opt, void *hip_stream) {
  if (!out || !opt) return UMGS_ERR_INVALID_ARG;
  *out = nullptr;
  std::string why;
  if (!valid_options(opt, why)) return UMGS_ERR_INVALID_ARG;
  umgs_ctx *h = new (std::nothrow) umgs_ctx();
  if (!h) return UMGS_ERR_CAPACITY;
  Ctx *c = &h->c;
  c->opt = *opt;
  c->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete h;
    return UMGS_ERR_HIP;
  }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess)
    c->num_cu = ncu;
  // the allocation-free entry point's scratch on this device (looked up once
  // per device, with it current)
  if (noalloc_scratch_init(c->device) != hipSuccess) {
    delete h;
    return UMGS_ERR_HIP;
  }
  *out = h;
  return UMGS_OK;
}

void umgs_destroy(umgs_ctx *ctx) {
  if (!ctx) return;
  Ctx *c = &ctx->c;
  if (c->capturing) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(c->stream, &g);
    if (g) (void)hipGraphDestroy(g);
  }
  (void)hipStreamSynchronize(c->stream);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  DevBuf *bufs[] = {&c->V_rest, &c->faces, &c->vf_ptr, &c->vf_idx, &c->vtab, &c->ftab, &c->bvh_code[0], &c->bvh_code[1],
                    &c->bvh_id[0], &c->bvh_id[1], &c->bvh_tri, &c->bvh_node, &c->bvh_aux,
                    &c->cast_code[0], &c->cast_code[1], &c->cast_id[0], &c->cast_id[1], &c->d_views,
                    &c->keys, &c->rects, &c->counts, &c->dk[0], &c->dk[1], &c->dv[0],
                    &c->dv[1], &c->offs, &c->grec, &c->trec, &c->scan_tmp,
                    &c->sk[0], &c->sk[1], &c->sv[0], &c->sv[1], &c->masks[0], &c->masks[1], &c->st_rng,
                    &c->chunk_base, &c->cnt2, &c->chunk_tab, &c->tstart, &c->totals,
                    &c->v0, &c->v1, &c->hist, &c->ranges, &c->g2d,
                    &c->minmax, &c->lb, &c->finfo, &c->tile_order, &c->bwd_order, &c->pair_count,
                    &c->view_sums, &c->tex, &c->tex_uv, &c->tb_g, &c->tb_key[0], &c->tb_key[1],
                    &c->tb_val[0], &c->tb_val[1], &c->tb_face};
  for (DevBuf *b : bufs) free_buf(*b);
  for (auto &p : c->prof.pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : c->prof.pool) (void)hipEventDestroy(e);
  if (c->host_pinned.p) (void)hipHostFree(c->host_pinned.p);
  if (c->ev_totals) (void)hipEventDestroy(c->ev_totals);
  delete ctx;
}

const char *umgs_last_error(const umgs_ctx *ctx) { return ctx ? ctx->c.err.c_str() : ""; }

umgs_status umgs_set_options(umgs_ctx *ctx, const umgs_options *opt) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (!opt) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_set_options: NULL options");
  std::string why;
  if (!valid_options(opt, why)) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_set_options: %s", why.c_str());
  c->opt = *opt;
  return UMGS_OK;
}

umgs_status umgs_set_proxy(umgs_ctx *ctx, int32_t nV, const float *V_rest, int32_t nF,
                           const int32_t *faces) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (!V_rest || !faces) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_set_proxy: NULL array");
  if (nV < 3 || nF < 1) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_set_proxy: nV=%d nF=%d", nV, nF);
  std::vector<int32_t> ptr(nV + 1, 0);
  for (int64_t k = 0; k < 3LL * nF; ++k) {
    const int32_t v = faces[k];
    if (v < 0 || v >= nV)
      return fail(c, UMGS_ERR_INVALID_ARG, "umgs_set_proxy: face %lld references vertex %d",
                  (long long)(k / 3), v);
    ptr[v + 1]++;
  }
  for (int f = 0; f < nF; ++f)
    if (faces[3 * f] == faces[3 * f + 1] || faces[3 * f] == faces[3 * f + 2] ||
        faces[3 * f + 1] == faces[3 * f + 2])
      return fail(c, UMGS_ERR_INVALID_ARG, "umgs_set_proxy: face %d is degenerate", f);
  for (int v = 0; v < nV; ++v) {
    if (ptr[v + 1] == 0) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_set_proxy: vertex %d has no face", v);
    ptr[v + 1] += ptr[v];
  }
  std::vector<int32_t> idx(ptr[nV]);
  std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
  for (int f = 0; f < nF; ++f)
    for (int k = 0; k < 3; ++k) idx[fill[faces[3 * f + k]]++] = f;
  umgs_status s;
  if ((s = ensure(c, c->V_rest, sizeof(float) * 3 * nV, "proxy vertices")) ||
      (s = ensure(c, c->faces, sizeof(int32_t) * 3 * nF, "proxy faces")) ||
      (s = ensure(c, c->vf_ptr, sizeof(int32_t) * (nV + 1), "vertex-face offsets")) ||
      (s = ensure(c, c->vf_idx, sizeof(int32_t) * idx.size(), "vertex-face lists")) ||
      (s = ensure(c, c->vtab, sizeof(float) * 12 * nV, "vertex transforms")) ||
      (s = ensure(c, c->ftab, sizeof(float) * 36 * ((size_t)nF + 1), "face transforms")))
    return s;
  hipError_t e;
  if ((e = hipMemcpy(c->V_rest.p, V_rest, sizeof(float) * 3 * nV, hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(c->faces.p, faces, sizeof(int32_t) * 3 * nF, hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(c->vf_ptr.p, ptr.data(), sizeof(int32_t) * (nV + 1), hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(c->vf_idx.p, idx.data(), sizeof(int32_t) * idx.size(), hipMemcpyHostToDevice)))
    return hip_check(c, e, "umgs_set_proxy upload");
  c->nV = nV;
  c->nF = nF;
  return UMGS_OK;
}

umgs_status umgs_bind_raycast(umgs_ctx *ctx, int32_t N, const float *means, const float *scales,
                              const float *quats, int32_t K, int32_t C, const float *cam_centers,
                              int32_t *bind_face, float *bind_bary, float *dist) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (c->nV == 0) return fail(c, UMGS_ERR_STATE, "umgs_bind_raycast: no proxy (call umgs_set_proxy)");
  if (c->capturing) return fail(c, UMGS_ERR_STATE, "umgs_bind_raycast: not allowed during graph capture");
  if (N < 0 || (K != 1 && K != 8) || C < 1 || C > (1 << 20))
    return fail(c, UMGS_ERR_INVALID_ARG, "umgs_bind_raycast: N=%d K=%d C=%d", N, K, C);
  if (!cam_centers) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_bind_raycast: NULL cam_centers");
  if (N > 0 && (!means || !bind_face || !bind_bary || (K == 8 && (!scales || !quats))))
    return fail(c, UMGS_ERR_INVALID_ARG, "umgs_bind_raycast: NULL array");
  if ((int64_t)N * K >= (1LL << 31))
    return fail(c, UMGS_ERR_CAPACITY, "umgs_bind_raycast: N*K = %lld targets", (long long)N * K);
  for (int64_t i = 0; i < 3LL * C; ++i)
    if (!std::isfinite(cam_centers[i]))
      return fail(c, UMGS_ERR_INVALID_ARG, "umgs_bind_raycast: camera %lld centre is not finite",
                  (long long)(i / 3));
  const int64_t nF = c->nF;
  const int64_t hb = (int64_t)radix_hist_bytes((uint64_t)std::max<int64_t>(nF, N));
  umgs_status s;
  if ((s = ensure(c, c->bvh_code[0], sizeof(uint32_t) * nF, "BVH codes")) ||
      (s = ensure(c, c->bvh_code[1], sizeof(uint32_t) * nF, "BVH codes")) ||
      (s = ensure(c, c->bvh_id[0], sizeof(uint32_t) * nF, "BVH ids")) ||
      (s = ensure(c, c->bvh_id[1], sizeof(uint32_t) * nF, "BVH ids")) ||
      (s = ensure(c, c->bvh_tri, 3 * sizeof(float4) * nF, "BVH leaves")) ||
      (s = ensure(c, c->bvh_node, 4 * sizeof(float4) * std::max<int64_t>(nF - 1, 1), "BVH nodes")) ||
      (s = ensure(c, c->bvh_aux, bvh_aux_bytes(C), "BVH bounds and cameras")) ||
      (s = ensure(c, c->cast_code[0], sizeof(uint32_t) * std::max<int64_t>(N, 1), "cast order")) ||
      (s = ensure(c, c->cast_code[1], sizeof(uint32_t) * std::max<int64_t>(N, 1), "cast order")) ||
      (s = ensure(c, c->cast_id[0], sizeof(uint32_t) * std::max<int64_t>(N, 1), "cast order")) ||
      (s = ensure(c, c->cast_id[1], sizeof(uint32_t) * std::max<int64_t>(N, 1), "cast order")) ||
      (s = ensure(c, c->hist, (size_t)hb, "radix histograms")) ||
      (s = ensure(c, c->scan_tmp,
                  scan_tmp_bytes(std::max<int64_t>({nF + 1, (int64_t)N + 1, 1 << 20, hb / 4})),
                  "scan scratch")))
    return s;
  hipError_t e = hipMemcpyAsync(bvh_cam_slots(c), cam_centers, sizeof(float) * 3 * (size_t)C,
                                hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return hip_check(c, e, "umgs_bind_raycast camera upload");
  if ((e = launch_bvh_build(c)) != hipSuccess) return hip_check(c, e, "BVH build");
  if ((e = launch_raycast(c, N, means, scales, quats, K, C, bind_face, bind_bary, dist)) != hipSuccess)
    return hip_check(c, e, "ray cast");
  uint32_t fault = 0;
  if ((e = hipMemcpyAsync(&fault, bvh_fault_flag(c), sizeof(fault), hipMemcpyDeviceToHost,
                          c->stream)) != hipSuccess ||
      (e = hipStreamSynchronize(c->stream)) != hipSuccess)
    return hip_check(c, e, "umgs_bind_raycast");
  if (fault)
    return fail(c, UMGS_ERR_CAPACITY, "umgs_bind_raycast: BVH traversal exceeded its stack or step bound");
  return UMGS_OK;
}

umgs_status umgs_bind_transfer(umgs_ctx *ctx, const float *V_def, int32_t N,
                               const int32_t *bind_face, const float *bind_bary,
                               const float *means, const float *quats, const float *scales,
                               float *means_out, float *quats_out, float *cov3d_out,
                               float *xform_out, float *vertex_out) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (c->nV == 0) return fail(c, UMGS_ERR_STATE, "umgs_bind_transfer: no proxy (call umgs_set_proxy)");
  if (N < 0) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_bind_transfer: N=%d", N);
  if (!V_def) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_bind_transfer: NULL V_def");
  if (N > 0 && (!bind_face || !bind_bary || !means || !quats || !scales || !means_out ||
                !cov3d_out))
    return fail(c, UMGS_ERR_INVALID_ARG, "umgs_bind_transfer: NULL Gaussian array");
  if (((uintptr_t)vertex_out & 15) != 0)
    return fail(c, UMGS_ERR_INVALID_ARG, "umgs_bind_transfer: vertex_out is not 16-byte aligned");
  if (c->opt.k_bind == 8 && N > 0 && ((((uintptr_t)bind_face) | ((uintptr_t)bind_bary)) & 15) != 0)
    return fail(c, UMGS_ERR_INVALID_ARG,
                "umgs_bind_transfer: bind_face and bind_bary must be 16-byte aligned");
  return hip_check(c, launch_transfer(c, V_def, N, bind_face, bind_bary, means, quats, scales,
                                      means_out, quats_out, cov3d_out, xform_out, vertex_out),
                   "transfer launch");
}

umgs_status umgs_bind_transfer_noalloc(umgs_ctx *ctx, const float *V_def, int32_t N,
                                       const int32_t *bind_face, const float *bind_bary,
                                       const float *means, const float *quats,
                                       const float *scales, float *means_out, float *quats_out,
                                       float *cov3d_out, float *xform_out, float *vertex_out) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (c->nV == 0)
    return fail(c, UMGS_ERR_STATE, "umgs_bind_transfer_noalloc: no proxy (call umgs_set_proxy)");
  if (N < 0) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_bind_transfer_noalloc: N=%d", N);
  if (!V_def) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_bind_transfer_noalloc: NULL V_def");
  if (N > 0 && (!bind_face || !bind_bary || !means || !quats || !scales || !means_out ||
                !cov3d_out))
    return fail(c, UMGS_ERR_INVALID_ARG, "umgs_bind_transfer_noalloc: NULL Gaussian array");
  if (((uintptr_t)vertex_out & 15) != 0)
    return fail(c, UMGS_ERR_INVALID_ARG,
                "umgs_bind_transfer_noalloc: vertex_out is not 16-byte aligned");
  if (c->opt.k_bind == 8 && N > 0 && ((((uintptr_t)bind_face) | ((uintptr_t)bind_bary)) & 15) != 0)
    return fail(c, UMGS_ERR_INVALID_ARG,
                "umgs_bind_transfer_noalloc: bind_face and bind_bary must be 16-byte aligned");
  const size_t need = noalloc_transfer_bytes(c->nV, c->nF, vertex_out == nullptr);
  if (need > kNoAllocScratchBytes)
    return fail(c, UMGS_ERR_CAPACITY,
                "umgs_bind_transfer_noalloc: a proxy of %d vertices and %d faces needs %zu bytes "
                "of scratch, more than the %zu the library holds per GPU",
                c->nV, c->nF, need, kNoAllocScratchBytes);
  void *base = noalloc_scratch(c->device);
  if (!base)
    return fail(c, UMGS_ERR_STATE, "umgs_bind_transfer_noalloc: no scratch on device %d", c->device);
  return hip_check(c, launch_transfer_noalloc(c, base, V_def, N, bind_face, bind_bary, means, quats,
                                              scales, means_out, quats_out, cov3d_out, xform_out,
                                              vertex_out),
                   "transfer launch");
}

umgs_status umgs_set_texture(umgs_ctx *ctx, int32_t tex_w, int32_t tex_h, const float *tex_rgba,
                             int32_t T, const float *tri_uv) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (c->capturing) return fail(c, UMGS_ERR_STATE, "umgs_set_texture: not allowed during graph capture");
  if (!tex_rgba) {
    c->tex_w = c->tex_h = c->tex_T = 0;
    return UMGS_OK;
  }
  if (tex_w < 1 || tex_h < 1 || tex_w > 16384 || tex_h > 16384 || T < 0 || (T > 0 && !tri_uv))
    return fail(c, UMGS_ERR_INVALID_ARG, "umgs_set_texture: %dx%d texture, T=%d, tri_uv=%p", tex_w,
                tex_h, T, (const void *)tri_uv);
  const size_t tb = sizeof(float) * 4 * (size_t)tex_w * (size_t)tex_h;
  const size_t ub = sizeof(float) * 6 * (size_t)std::max(T, 1);
  umgs_status s;
  if ((s = ensure(c, c->tex, tb, "texture")) || (s = ensure(c, c->tex_uv, ub, "texture coordinates")))
    return s;
  hipError_t e = hipMemcpyAsync(c->tex.p, tex_rgba, tb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && T > 0)
    e = hipMemcpyAsync(c->tex_uv.p, tri_uv, sizeof(float) * 6 * (size_t)T, hipMemcpyDeviceToDevice,
                       c->stream);
  if (e != hipSuccess) return hip_check(c, e, "umgs_set_texture copy");
  c->tex_w = tex_w;
  c->tex_h = tex_h;
  c->tex_T = T;
  return UMGS_OK;
}

static umgs_status build_views(Ctx *c, int32_t V, const umgs_camera *cams,
                               std::vector<ViewParams> &vps, int64_t &tiles, int64_t &pix,
                               int64_t *st_total = nullptr) {
  const umgs_options &o = c->opt;
  vps.assign(V, ViewParams());
  tiles = 0;
  pix = 0;
  int64_t sts = 0;
  for (int v = 0; v < V; ++v) {
    const umgs_camera &cm = cams[v];
    if (cm.width < 1 || cm.height < 1 || cm.width > 16384 || cm.height > 16384)
      return fail(c, UMGS_ERR_INVALID_ARG, "view %d size %dx%d", v, cm.width, cm.height);
    if (!(cm.fx > 0) || !(cm.fy > 0) || !std::isfinite(cm.cx) || !std::isfinite(cm.cy))
      return fail(c, UMGS_ERR_INVALID_ARG, "view %d intrinsics", v);
    ViewParams &p = vps[v];
    memcpy(p.R, cm.R, sizeof p.R);
    memcpy(p.t, cm.t, sizeof p.t);
    p.fx = cm.fx; p.fy = cm.fy; p.cx = cm.cx; p.cy = cm.cy;
    p.tanx = (float)cm.width / (2.0f * cm.fx);
    p.tany = (float)cm.height / (2.0f * cm.fy);
    p.W = cm.width; p.H = cm.height;
    p.ntx = (cm.width + o.tile_w - 1) / o.tile_w;
    p.nty = (cm.height + o.tile_h - 1) / o.tile_h;
    p.tile_base = (uint32_t)tiles;
    p.st_base = (uint32_t)sts;
    p.pix_base = pix;
    if (c->view_offsets) {
      // caller-placed views: increasing, non-overlapping pixel ranges
      const int64_t off = c->view_offsets[v];
      if (off < pix)
        return fail(c, UMGS_ERR_INVALID_ARG, "view %d offset %lld overlaps the previous view", v,
                    (long long)off);
      p.pix_base = off;
      pix = off;
    }
    tiles += (int64_t)p.ntx * p.nty;
    sts += (int64_t)((p.ntx + kST - 1) / kST) * ((p.nty + kST - 1) / kST);
    pix += (int64_t)cm.width * cm.height;
  }
  if (st_total) *st_total = sts;
  if (c->view_offsets && pix > c->view_offsets[V])
    return fail(c, UMGS_ERR_INVALID_ARG, "last view ends at %lld, past view_offsets[V] = %lld",
                (long long)pix, (long long)c->view_offsets[V]);
  if (tiles >= (1LL << 31)) return fail(c, UMGS_ERR_CAPACITY, "%lld tiles", (long long)tiles);
  return UMGS_OK;
}

umgs_status umgs_project(umgs_ctx *ctx, int32_t V, const umgs_camera *cams, int32_t N,
                         const float *means, const float *cov3d, const float *scales,
                         const float *quats, const float *opacity, const float *sh,
                         int32_t T, const float *tri_xyz, const float *tri_rgb,
                         const float *tri_alpha) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (V < 1 || !cams) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_project: V=%d cams=%p", V, (const void *)cams);
  if (N < 0 || T < 0) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_project: N=%d T=%d", N, T);
  if (N > 0 && (!means || !opacity || !sh || (!cov3d && (!scales || !quats))))
    return fail(c, UMGS_ERR_INVALID_ARG, "umgs_project: NULL Gaussian array");
  if (T > 0 && (!tri_xyz || !tri_rgb || !tri_alpha))
    return fail(c, UMGS_ERR_INVALID_ARG, "umgs_project: NULL triangle array");
  if ((int64_t)V * ((int64_t)N + T) >= (1LL << 31))
    return fail(c, UMGS_ERR_CAPACITY, "umgs_project: V*(N+T) = %lld records", (long long)V * (N + T));
  if (c->tex_w > 0 && T != c->tex_T)
    return fail(c, UMGS_ERR_INVALID_ARG,
                "umgs_project: the texture coordinates cover %d triangles, the frame has %d",
                c->tex_T, T);
  const umgs_options &o = c->opt;
  std::vector<ViewParams> vps;
  int64_t tiles = 0, pix = 0, sts = 0;
  umgs_status s = build_views(c, V, cams, vps, tiles, pix, &sts);
  if (s != UMGS_OK) return s;
  // Device view tables are stored once per distinct camera set, so a captured
  // graph can replay frames (or view groups) whose tables were uploaded by
  // eager calls.
  int set = -1;
  for (size_t k = 0; k < c->view_sets.size() && set < 0; ++k) {
    const std::vector<ViewParams> &t = c->view_sets[k];
    if ((int)t.size() == V && memcmp(t.data(), vps.data(), sizeof(ViewParams) * V) == 0) set = (int)k;
  }
  if (set < 0 && c->capturing)
    return fail(c, UMGS_ERR_STATE, "umgs_project: while capturing, the cameras must be those of "
                                   "an eager frame (update them with umgs_update_views)");
  if (V > kViewSlots) return fail(c, UMGS_ERR_CAPACITY, "umgs_project: %d views", V);
  const int64_t nrec = (int64_t)V * (N + T);
  if ((s = ensure(c, c->d_views, sizeof(ViewParams) * kViewSlots, "view tables")) ||
      (s = ensure(c, c->keys, sizeof(uint32_t) * std::max<int64_t>(nrec, 1), "depth keys")) ||
      (s = ensure(c, c->rects, sizeof(uint2) * std::max<int64_t>(nrec, 1), "tile rects")) ||
      (s = ensure(c, c->counts, sizeof(uint64_t) * std::max<int64_t>(nrec, 1), "tile counts")) ||
      (s = ensure(c, c->dk[0], sizeof(uint32_t) * std::max<int64_t>(nrec, 1), "depth order")) ||
      (s = ensure(c, c->dk[1], sizeof(uint32_t) * std::max<int64_t>(nrec, 1), "depth order")) ||
      (s = ensure(c, c->dv[0], sizeof(uint32_t) * std::max<int64_t>(nrec, 1), "depth order")) ||
      (s = ensure(c, c->dv[1], sizeof(uint32_t) * std::max<int64_t>(nrec, 1), "depth order")) ||
      (s = ensure(c, c->offs, sizeof(uint64_t) * (nrec + 1), "record offsets")) ||
      (s = ensure(c, c->hist, radix_hist_bytes(std::max<int64_t>(nrec, 1)), "radix histograms")) ||
      (s = ensure(c, c->view_sums, sizeof(uint64_t) * V, "view sums")) ||
      (s = ensure(c, c->grec, sizeof(GaussRec) * std::max<int64_t>((int64_t)V * N, 1), "Gaussian records")) ||
      (s = ensure(c, c->trec, sizeof(TriRec) * std::max<int64_t>((int64_t)V * T, 1), "triangle records")) ||
      (s = ensure(c, c->scan_tmp,
                  scan_tmp_bytes(std::max<int64_t>({nrec + 1, 1 << 20,
                                                    (int64_t)radix_hist_bytes(std::max<int64_t>(nrec, 1)) / 4})),
                  "scan scratch")) ||
      (s = ensure(c, c->ranges, sizeof(uint2) * tiles, "tile ranges")) ||
      (s = ensure(c, c->tstart, sizeof(uint32_t) * (tiles + 1), "tile starts")) ||
      (s = ensure(c, c->st_rng, sizeof(uint2) * sts, "supertile ranges")) ||
      (s = ensure(c, c->chunk_base, sizeof(uint32_t) * (sts + 1), "supertile chunks")) ||
      (s = ensure(c, c->totals, 2 * sizeof(uint64_t), "frame totals")) ||
      (s = ensure(c, c->minmax, 2 * kMinMaxSlots * sizeof(uint32_t), "depth range")) ||
      (s = ensure(c, c->lb, sizeof(LbState), "scan state")) ||
      (s = ensure(c, c->finfo, sizeof(FrameInfo), "frame info")) ||
      (s = ensure(c, c->tile_order, sizeof(uint32_t) * (64 + tiles), "tile order")) ||
      (s = ensure(c, c->bwd_order, sizeof(uint32_t) * (128 + 3 * tiles), "backward tile order")))
    return s;
  const bool fresh_info = c->finfo.cap && c->views.empty();
  const bool fresh_lb = !c->lb_zeroed;
  bool upload = false;
  if (set < 0) {
    if (c->view_used + V > kViewSlots) {   // store full: start over (eager only)
      c->view_sets.clear();
      c->view_set_off.clear();
      c->view_used = 0;
    }
    set = (int)c->view_sets.size();
    c->view_sets.push_back(vps);
    c->view_set_off.push_back(c->view_used);
    c->view_used += V;
    upload = true;
  }
  ViewParams *dv = (ViewParams *)c->d_views.p + c->view_set_off[set];
  c->cur_views = dv;
  c->views = vps;
  c->V = V; c->N = N; c->T = T;
  c->tile_w = o.tile_w; c->tile_h = o.tile_h; c->frag_batch = o.frag_batch;
  c->mode = o.mode; c->sh_degree = o.sh_degree;
  c->bg[0] = o.bg[0]; c->bg[1] = o.bg[1]; c->bg[2] = o.bg[2];
  c->n_records = nrec;
  c->n_tiles = tiles;
  c->n_pixels = pix;
  c->n_st = sts;
  c->n_st_max = std::max(c->n_st_max, sts);
  int bits = 1;
  while (bits < 31 && (1LL << bits) < sts) ++bits;
  c->st_bits = bits;
  c->st_key16 = sts <= 65536;
  c->stage = 0;
  hipError_t e = hipSuccess;
  if (fresh_info) e = launch_fill_u32(c, (uint32_t *)c->finfo.p, sizeof(FrameInfo) / 4, 0u);
  if (e == hipSuccess && fresh_lb) {
    e = launch_fill_u32(c, (uint32_t *)c->lb.p, sizeof(LbState) / 4, 0u);
    c->lb_zeroed = e == hipSuccess;
  }
  if (e == hipSuccess && upload)
    e = hipMemcpyAsync(dv, vps.data(), sizeof(ViewParams) * V, hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return hip_check(c, e, "view upload");
  // the range slots start reset; after that the bin stage resets them as it
  // folds them (a projection without a bin in between widens the next
  // frame's range, which still holds every key)
  if (!c->minmax_ready) {
    e = launch_minmax_reset(c);
    if (e != hipSuccess) return hip_check(c, e, "depth range reset");
    c->minmax_ready = true;
  }
  if ((e = launch_project_gaussians(c, means, cov3d, scales, quats, opacity, sh)) != hipSuccess)
    return hip_check(c, e, "project_gaussians launch");
  if ((e = launch_setup_triangles(c, tri_xyz, tri_rgb, tri_alpha)) != hipSuccess)
    return hip_check(c, e, "setup_triangles launch");
  c->stage = 1;
  return UMGS_OK;
}

// Buffers of the tile lists (n duplicates) and of the first binning level
// (st supertile entries) for the current frame's supertiles.
static umgs_status ensure_lists(Ctx *c, uint64_t n, uint64_t st) {
  umgs_status s;
  n = std::max<uint64_t>(n, 1);
  st = std::max<uint64_t>(st, 1);
  const int64_t n_st = std::max(c->n_st, c->n_st_max);
  if ((s = ensure(c, c->v0, 4 * n, "tile lists")) ||
      (s = ensure(c, c->sk[0], 4 * st, "supertile entries")) ||
      (s = ensure(c, c->sk[1], 4 * st, "supertile entries")) ||
      (s = ensure(c, c->sv[0], 4 * st, "supertile entries")) ||
      (s = ensure(c, c->sv[1], 4 * st, "supertile entries")) ||
      (s = ensure(c, c->masks[0], 8 * st, "supertile masks")) ||
      (s = ensure(c, c->masks[1], 8 * st, "supertile masks")) ||
      (s = ensure(c, c->cnt2, 64 * sizeof(uint32_t) * max_chunks(st, n_st), "chunk counts")) ||
      (s = ensure(c, c->chunk_tab, chunk_rec_bytes() * max_chunks(st, n_st), "chunk table")) ||
      (s = ensure(c, c->hist, radix_hist_bytes(std::max<uint64_t>(st, c->n_records)), "radix histograms")) ||
      (s = ensure(c, c->scan_tmp,
                  scan_tmp_bytes(std::max<int64_t>({(int64_t)radix_hist_bytes(st) / 4, c->n_records + 1,
                                                    c->n_tiles + 1, n_st + 1})),
                  "scan scratch")))
    return s;
  c->list_key = n;
  c->list_st = st;
  c->list_nst = n_st;
  return UMGS_OK;
}

umgs_status umgs_bin(umgs_ctx *ctx) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (c->stage < 1) return fail(c, UMGS_ERR_STATE, "umgs_bin: no projected frame");
  if (!c->fixed_cap && c->capturing)
    return fail(c, UMGS_ERR_STATE, "umgs_bin: capturing without a reservation");
  hipError_t e = launch_depth_order(c);
  if (e != hipSuccess) return hip_check(c, e, "depth order launch");
  if (c->fixed_cap) {
    // sizes stay on the device; every first-level grid covers the capacity
    if (ensure_lists(c, c->key_cap, c->st_cap) != UMGS_OK) return UMGS_ERR_CAPACITY;
    c->st_launch = c->st_cap;
  } else {
    if (!c->host_pinned.p) {
      if ((e = hipHostMalloc(&c->host_pinned.p, 256, hipHostMallocDefault)) != hipSuccess)
        return hip_check(c, e, "pinned scratch");
      c->host_pinned.cap = 256;
    }
    if (!c->ev_totals &&
        (e = hipEventCreateWithFlags(&c->ev_totals, hipEventDisableTiming)) != hipSuccess)
      return hip_check(c, e, "readback event");
    uint64_t *h = (uint64_t *)c->host_pinned.p;
    if ((e = hipMemcpyAsync(h, c->totals.p, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost,
                            c->stream)) != hipSuccess ||
        (e = hipEventRecord(c->ev_totals, c->stream)) != hipSuccess)
      return hip_check(c, e, "duplicate count readback");
    // While the counts travel, the first level goes ahead into the buffers
    // of earlier frames (grids over their capacity, counts read on the
    // device, as in a reserved frame); the host then waits for the counts
    // only, not for that work.  A frame that does not fit is binned again
    // once the buffers have grown.
    const bool spec = c->list_key > 0 && c->list_st > 0 &&
                      std::max(c->n_st, c->n_st_max) <= c->list_nst;
    if (spec) {
      c->key_cap = c->list_key;
      c->st_cap = c->list_st;
      c->st_launch = c->list_st;
      if ((e = launch_st_bin(c)) != hipSuccess) return hip_check(c, e, "supertile binning launch");
    }
    if ((e = hipEventSynchronize(c->ev_totals)) != hipSuccess)
      return hip_check(c, e, "duplicate count readback");
    const uint64_t nd = h[0], n1 = h[1];
    if (nd >= 0xFFFF0000ull)
      return fail(c, UMGS_ERR_CAPACITY, "umgs_bin: %llu duplicates exceed 2^32", (unsigned long long)nd);
    if (n1 >= 0xFFFF0000ull)
      return fail(c, UMGS_ERR_CAPACITY, "umgs_bin: %llu supertile entries exceed 2^32",
                  (unsigned long long)n1);
    c->n_dup = nd;
    if (nd) c->st_ratio = (double)n1 / (double)nd;
    if (spec && nd <= c->list_key && n1 <= c->list_st) {
      c->stage = 2;
      return UMGS_OK;
    }
    // the work that went ahead (if any) must end before buffers move
    if (spec && (e = hipStreamSynchronize(c->stream)) != hipSuccess)
      return hip_check(c, e, "supertile binning");
    umgs_status s = ensure_lists(c, nd, n1);
    if (s != UMGS_OK) return s;
    c->key_cap = std::max<uint64_t>(nd, 1);
    c->st_cap = std::max<uint64_t>(n1, 1);
    c->st_launch = n1;
    if (spec) {
      // what it left: the sticky overflow flag it raised, the supertile
      // ranges it wrote
      if ((e = launch_fill_u32(c, (uint32_t *)c->finfo.p + offsetof(FrameInfo, overflow) / 4, 1, 0u)) !=
              hipSuccess ||
          (e = launch_fill_u32(c, (uint32_t *)c->st_rng.p, 2 * c->n_st, 0u)) != hipSuccess)
        return hip_check(c, e, "supertile binning reset");
    }
  }
  if ((e = launch_st_bin(c)) != hipSuccess) return hip_check(c, e, "supertile binning launch");
  c->stage = 2;
  return UMGS_OK;
}

umgs_status umgs_sort(umgs_ctx *ctx) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (c->stage < 2) return fail(c, UMGS_ERR_STATE, "umgs_sort: frame not binned");
  hipError_t e = launch_tile_lists(c);
  if (e != hipSuccess) return hip_check(c, e, "tile lists launch");
  c->stage = 3;
  return UMGS_OK;
}

umgs_status umgs_blend(umgs_ctx *ctx, float *image, float *T_final, int32_t *n_contrib,
                       float *T_entity_in) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (c->stage < 3) return fail(c, UMGS_ERR_STATE, "umgs_blend: frame not sorted");
  if (!image) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_blend: NULL image");
  umgs_status s = hip_check(c, launch_blend(c, image, T_final, n_contrib, T_entity_in), "blend launch");
  if (s == UMGS_OK) c->stage = 4;
  return s;
}

umgs_status umgs_render_batched(umgs_ctx *ctx, int32_t V, const umgs_camera *cams,
                                const int64_t *view_offsets, int32_t N, const float *means,
                                const float *cov3d, const float *scales, const float *quats,
                                const float *opacity, const float *sh, int32_t T,
                                const float *tri_xyz, const float *tri_rgb, const float *tri_alpha,
                                float *image, float *T_final, int32_t *n_contrib,
                                float *T_entity_in) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (!image) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_render_batched: NULL image");
  c->view_offsets = view_offsets;
  umgs_status s = umgs_project(ctx, V, cams, N, means, cov3d, scales, quats, opacity, sh, T,
                               tri_xyz, tri_rgb, tri_alpha);
  c->view_offsets = nullptr;
  if (s != UMGS_OK) return s;
  if ((s = umgs_bin(ctx)) != UMGS_OK || (s = umgs_sort(ctx)) != UMGS_OK) return s;
  const int32_t sched = c->opt.schedule;
  c->opt.schedule = UMGS_SCHEDULE_PERSISTENT;
  s = umgs_blend(ctx, image, T_final, n_contrib, T_entity_in);
  c->opt.schedule = sched;
  return s;
}

umgs_status umgs_backward(umgs_ctx *ctx, const float *dL_dimage, const float *T_final,
                          const int32_t *n_contrib, const float *T_entity_in, const float *means,
                          const float *scales, const float *quats, const float *xform,
                          const float *sh, float *dL_dmeans, float *dL_dscales, float *dL_dquats,
                          float *dL_dopacity, float *dL_dsh, float *dL_dxform, int32_t accumulate) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (c->stage < 4) return fail(c, UMGS_ERR_STATE, "umgs_backward: no blended frame on this context");
  if (c->mode != UMGS_MODE_UNIMGS && c->mode != UMGS_MODE_DIRECT)
    return fail(c, UMGS_ERR_UNSUPPORTED, "umgs_backward: mode %d has no backward", c->mode);
  if (!dL_dimage || !T_final || !n_contrib || !T_entity_in)
    return fail(c, UMGS_ERR_INVALID_ARG, "umgs_backward: NULL per-pixel array");
  if (c->N > 0 && (!means || !scales || !quats || !sh || !dL_dmeans || !dL_dscales || !dL_dquats ||
                   !dL_dopacity || !dL_dsh))
    return fail(c, UMGS_ERR_INVALID_ARG, "umgs_backward: NULL Gaussian array");
  umgs_status s = ensure(c, c->g2d, sizeof(float) * 9 * std::max<int64_t>((int64_t)c->V * c->N, 1),
                         "2D gradients");
  if (s != UMGS_OK) return s;
  return hip_check(c, launch_backward(c, dL_dimage, T_final, n_contrib, T_entity_in, means, scales,
                                      quats, xform, sh, dL_dmeans, dL_dscales, dL_dquats,
                                      dL_dopacity, dL_dsh, dL_dxform, accumulate != 0),
                   "backward launch");
}

umgs_status umgs_backward_transfer(umgs_ctx *ctx, const float *V_def, int32_t N,
                                   const int32_t *bind_face, const float *bind_bary,
                                   const float *dL_dmeans, const float *dL_dxform,
                                   float *dL_dV_def, int32_t accumulate) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (c->nV == 0)
    return fail(c, UMGS_ERR_STATE, "umgs_backward_transfer: no proxy (call umgs_set_proxy)");
  if (N < 0) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_backward_transfer: N=%d", N);
  if (!V_def || !dL_dV_def)
    return fail(c, UMGS_ERR_INVALID_ARG, "umgs_backward_transfer: NULL V_def or dL_dV_def");
  if (N > 0 && (!bind_face || !bind_bary))
    return fail(c, UMGS_ERR_INVALID_ARG, "umgs_backward_transfer: NULL binding array");
  const int64_t M = std::max<int64_t>((int64_t)N * c->opt.k_bind, 1);
  if (M >= (1LL << 31))
    return fail(c, UMGS_ERR_CAPACITY, "umgs_backward_transfer: N*K = %lld corners", (long long)M);
  const int64_t hb = (int64_t)radix_hist_bytes((uint64_t)M);
  umgs_status s;
  if ((s = ensure(c, c->tb_face, sizeof(float) * 36 * (size_t)c->nF, "per-face gradient sums")) ||
      (s = ensure(c, c->tb_g, sizeof(float) * kGRow * (size_t)std::max<int32_t>(N, 1), "Gaussian gradient rows")) ||
      (s = ensure(c, c->tb_key[0], sizeof(uint32_t) * (size_t)M, "corner keys")) ||
      (s = ensure(c, c->tb_key[1], sizeof(uint32_t) * (size_t)M, "corner keys")) ||
      (s = ensure(c, c->tb_val[0], sizeof(uint32_t) * (size_t)M, "corner ids")) ||
      (s = ensure(c, c->tb_val[1], sizeof(uint32_t) * (size_t)M, "corner ids")) ||
      (s = ensure(c, c->hist, (size_t)hb, "radix histograms")) ||
      (s = ensure(c, c->scan_tmp, scan_tmp_bytes(std::max<int64_t>({M + 1, 1 << 20, hb / 4})),
                  "scan scratch")))
    return s;
  return hip_check(c, launch_transfer_backward(c, V_def, N, bind_face, bind_bary, dL_dmeans,
                                               dL_dxform, dL_dV_def, accumulate != 0),
                   "transfer backward launch");
}

umgs_status umgs_backward_triangles(umgs_ctx *ctx, const float *dL_dimage, const float *T_final,
                                    const int32_t *n_contrib, const float *T_entity_in,
                                    float *dL_dtri_rgb, float *dL_dtri_alpha, int32_t accumulate) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (c->stage < 4)
    return fail(c, UMGS_ERR_STATE, "umgs_backward_triangles: no blended frame on this context");
  if (c->mode != UMGS_MODE_UNIMGS && c->mode != UMGS_MODE_DIRECT)
    return fail(c, UMGS_ERR_UNSUPPORTED, "umgs_backward_triangles: mode %d has no backward", c->mode);
  if (!dL_dimage || !T_final || !n_contrib || !T_entity_in)
    return fail(c, UMGS_ERR_INVALID_ARG, "umgs_backward_triangles: NULL per-pixel array");
  if (c->T > 0 && (!dL_dtri_rgb || !dL_dtri_alpha))
    return fail(c, UMGS_ERR_INVALID_ARG, "umgs_backward_triangles: NULL triangle array");
  return hip_check(c, launch_backward_triangles(c, dL_dimage, T_final, n_contrib, T_entity_in,
                                                dL_dtri_rgb, dL_dtri_alpha, accumulate != 0),
                   "triangle backward launch");
}

// Reads the device frame info into the host copies (synchronizes).
static umgs_status read_frame_info(Ctx *c, FrameInfo *out) {
  memset(out, 0, sizeof *out);
  if (!c->finfo.p) return UMGS_OK;
  hipError_t e = hipMemcpyAsync(out, c->finfo.p, sizeof *out, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_check(c, e, "frame info readback");
  if (out->fault)
    return fail(c, UMGS_ERR_HIP, "a device scan gave up waiting for an earlier tile (look-back "
                "limit); the frame's lists are not valid");
  if (c->stage >= 2) c->n_dup = out->n_dup;
  return UMGS_OK;
}

umgs_status umgs_query(umgs_ctx *ctx, int64_t *n_dup, int64_t *n_tiles, int64_t *n_records,
                       int32_t *overflow) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (c->capturing) return fail(c, UMGS_ERR_STATE, "umgs_query: the stream is being captured");
  FrameInfo fi;
  umgs_status s = read_frame_info(c, &fi);
  if (s != UMGS_OK) return s;
  if (n_dup) *n_dup = (int64_t)c->n_dup;
  if (n_tiles) *n_tiles = c->n_tiles;
  if (n_records) *n_records = c->n_records;
  if (overflow) {
    *overflow = fi.overflow ? 1 : 0;
    if (fi.overflow) {
      hipError_t e = launch_fill_u32(c, (uint32_t *)c->finfo.p + offsetof(FrameInfo, overflow) / 4, 1, 0u);
      if (e != hipSuccess) return hip_check(c, e, "overflow reset");
    }
  }
  return UMGS_OK;
}

umgs_status umgs_query_bins(umgs_ctx *ctx, int64_t *n_supertiles, int64_t *n_entries) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (c->capturing) return fail(c, UMGS_ERR_STATE, "umgs_query_bins: the stream is being captured");
  if (c->stage < 2) return fail(c, UMGS_ERR_STATE, "umgs_query_bins: frame not binned");
  FrameInfo fi;
  umgs_status s = read_frame_info(c, &fi);
  if (s != UMGS_OK) return s;
  if (n_supertiles) *n_supertiles = c->n_st;
  if (n_entries) *n_entries = (int64_t)fi.n1;
  return UMGS_OK;
}

umgs_status umgs_copy_state(umgs_ctx *ctx, int32_t which, void *dst, int64_t cap_bytes) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (!dst) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_copy_state: NULL destination");
  if (c->capturing) return fail(c, UMGS_ERR_STATE, "umgs_copy_state: the stream is being captured");
  FrameInfo fi;
  umgs_status st = read_frame_info(c, &fi);
  if (st != UMGS_OK) return st;
  const void *src = nullptr;
  int64_t bytes = 0;
  int need = 1;
  switch (which) {
    case UMGS_STATE_KEYS: src = c->keys.p; bytes = 4 * c->n_records; need = 1; break;
    case UMGS_STATE_SORTED_KEYS: src = nullptr; bytes = 8 * (int64_t)fi.n_dup; need = 3; break;
    case UMGS_STATE_GRAD2D: src = c->g2d.p; bytes = 36 * (int64_t)c->V * c->N; need = 4; break;
    case UMGS_STATE_SORTED_VALS: src = c->v0.p; bytes = 4 * (int64_t)fi.n_dup; need = 3; break;
    case UMGS_STATE_RANGES: src = c->ranges.p; bytes = 8 * c->n_tiles; need = 3; break;
    case UMGS_STATE_TRI_FIXED: src = c->trec.p; bytes = 24 * (int64_t)c->V * c->T; need = 1; break;
    default: return fail(c, UMGS_ERR_INVALID_ARG, "umgs_copy_state: unknown state %d", which);
  }
  if (c->stage < need) return fail(c, UMGS_ERR_STATE, "umgs_copy_state: state %d not computed", which);
  if (cap_bytes < bytes) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_copy_state: need %lld bytes", (long long)bytes);
  if (bytes == 0) return UMGS_OK;
  hipError_t e;
  if (which == UMGS_STATE_SORTED_KEYS) {
    e = launch_expand_keys(c, (uint64_t *)dst);
  } else if (which == UMGS_STATE_TRI_FIXED) {
    // 2D copy: the first 24 bytes of every record
    e = hipMemcpy2DAsync(dst, 24, src, sizeof(TriRec), 24, (size_t)c->V * c->T,
                         hipMemcpyDeviceToDevice, c->stream);
  } else {
    e = hipMemcpyAsync(dst, src, (size_t)bytes, hipMemcpyDeviceToDevice, c->stream);
  }
  return hip_check(c, e, "umgs_copy_state copy");
}

umgs_status umgs_blend_pairs(umgs_ctx *ctx, float *image, int64_t *pairs) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (c->stage < 3) return fail(c, UMGS_ERR_STATE, "umgs_blend_pairs: frame not sorted");
  if (!image || !pairs) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_blend_pairs: NULL argument");
  if (c->capturing) return fail(c, UMGS_ERR_STATE, "umgs_blend_pairs: capturing");
  umgs_status s = ensure(c, c->pair_count, 4 * sizeof(uint64_t), "pair counters");
  if (s != UMGS_OK) return s;
  hipError_t e = launch_fill_u32(c, (uint32_t *)c->pair_count.p, 8, 0u);
  if (e == hipSuccess)
    e = launch_blend(c, image, nullptr, nullptr, nullptr, (unsigned long long *)c->pair_count.p);
  if (e == hipSuccess)
    e = hipMemcpyAsync(pairs, c->pair_count.p, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return hip_check(c, e, "umgs_blend_pairs");
}

umgs_status umgs_reserve(umgs_ctx *ctx, int64_t max_dup) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (c->capturing) return fail(c, UMGS_ERR_STATE, "umgs_reserve: the stream is being captured");
  if (max_dup < 0 || (uint64_t)max_dup >= 0xFFFF0000ull)
    return fail(c, UMGS_ERR_INVALID_ARG, "umgs_reserve: max_dup=%lld", (long long)max_dup);
  if (max_dup == 0) {
    c->fixed_cap = false;
    return UMGS_OK;
  }
  // first-level capacity: the last eager frame's entries per duplicate (a
  // quarter before any), with 25% headroom
  const double ratio = c->st_ratio > 0.0 ? c->st_ratio : 0.25;
  const uint64_t st = std::min<uint64_t>(
      (uint64_t)max_dup, std::max<uint64_t>((uint64_t)(1.25 * ratio * (double)max_dup) + 1, 1u << 16));
  umgs_status s = ensure_lists(c, (uint64_t)max_dup, st);
  if (s != UMGS_OK) return s;
  c->key_cap = (uint64_t)max_dup;
  c->st_cap = st;
  c->fixed_cap = true;
  return UMGS_OK;
}

umgs_status umgs_graph_begin(umgs_ctx *ctx) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (c->capturing) return fail(c, UMGS_ERR_STATE, "umgs_graph_begin: already capturing");
  if (!c->fixed_cap) return fail(c, UMGS_ERR_STATE, "umgs_graph_begin: call umgs_reserve first");
  if (c->prof.on) return fail(c, UMGS_ERR_STATE, "umgs_graph_begin: profiling is on");
  if (c->views.empty()) return fail(c, UMGS_ERR_STATE, "umgs_graph_begin: render one eager frame first");
  if (!c->stream) return fail(c, UMGS_ERR_STATE, "umgs_graph_begin: the null stream cannot be captured");
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return hip_check(c, e, "hipStreamBeginCapture");
  c->capturing = true;
  return UMGS_OK;
}

umgs_status umgs_graph_end(umgs_ctx *ctx) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (!c->capturing) return fail(c, UMGS_ERR_STATE, "umgs_graph_end: not capturing");
  c->capturing = false;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (e != hipSuccess) return hip_check(c, e, "hipStreamEndCapture");
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph = g;
  c->graph_exec = nullptr;
  e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
  return hip_check(c, e, "hipGraphInstantiate");
}

umgs_status umgs_graph_launch(umgs_ctx *ctx) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (!c->graph_exec) return fail(c, UMGS_ERR_STATE, "umgs_graph_launch: no graph");
  if (c->capturing) return fail(c, UMGS_ERR_STATE, "umgs_graph_launch: capturing");
  return hip_check(c, hipGraphLaunch(c->graph_exec, c->stream), "hipGraphLaunch");
}

umgs_status umgs_update_views(umgs_ctx *ctx, int32_t V, const umgs_camera *old_cams,
                              const umgs_camera *new_cams) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (c->capturing) return fail(c, UMGS_ERR_STATE, "umgs_update_views: capturing");
  if (!old_cams || !new_cams || V < 1)
    return fail(c, UMGS_ERR_INVALID_ARG, "umgs_update_views: NULL cameras or V=%d", V);
  std::vector<ViewParams> oldv, newv;
  int64_t tiles = 0, pix = 0, tiles2 = 0, pix2 = 0;
  umgs_status s = build_views(c, V, old_cams, oldv, tiles, pix);
  if (s == UMGS_OK) s = build_views(c, V, new_cams, newv, tiles2, pix2);
  if (s != UMGS_OK) return s;
  for (int v = 0; v < V; ++v)
    if (oldv[v].W != newv[v].W || oldv[v].H != newv[v].H)
      return fail(c, UMGS_ERR_INVALID_ARG, "umgs_update_views: view %d changed size", v);
  for (size_t k = 0; k < c->view_sets.size(); ++k) {
    std::vector<ViewParams> &t = c->view_sets[k];
    if ((int)t.size() != V) continue;
    // a table keeps its pixel placement (packed, or the caller's offsets)
    for (int v = 0; v < V; ++v) oldv[v].pix_base = newv[v].pix_base = t[v].pix_base;
    if (memcmp(t.data(), oldv.data(), sizeof(ViewParams) * V) != 0) continue;
    t = newv;
    ViewParams *dv = (ViewParams *)c->d_views.p + c->view_set_off[k];
    if (dv == c->cur_views) c->views = newv;
    return hip_check(c, hipMemcpyAsync(dv, newv.data(), sizeof(ViewParams) * V,
                                       hipMemcpyHostToDevice, c->stream),
                     "view upload");
  }
  return fail(c, UMGS_ERR_STATE, "umgs_update_views: no stored view table matches old_cams");
}

umgs_status umgs_view_dups(umgs_ctx *ctx, int64_t *dups) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (!dups) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_view_dups: NULL output");
  if (c->stage < 1) return fail(c, UMGS_ERR_STATE, "umgs_view_dups: no projected frame");
  if (c->capturing) return fail(c, UMGS_ERR_STATE, "umgs_view_dups: capturing");
  std::vector<uint64_t> b(c->V);
  hipError_t e = launch_view_sums(c, (unsigned long long *)c->view_sums.p);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b.data(), c->view_sums.p, sizeof(uint64_t) * c->V, hipMemcpyDeviceToHost,
                       c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_check(c, e, "umgs_view_dups");
  for (int v = 0; v < c->V; ++v) dups[v] = (int64_t)b[v];
  return UMGS_OK;
}

umgs_status umgs_set_profiling(umgs_ctx *ctx, int32_t enable) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  umgs_status s = drain_profile(c);
  if (s != UMGS_OK) return s;
  for (int k = 0; k < K_COUNT; ++k) {
    c->prof.ms[k] = 0.0;
    c->prof.n[k] = 0;
  }
  c->prof.on = enable != 0;
  return UMGS_OK;
}

umgs_status umgs_profile_read(umgs_ctx *ctx, int32_t kernel, int64_t *launches, double *total_ms) {
  if (!ctx) return UMGS_ERR_INVALID_ARG;
  Ctx *c = &ctx->c;
  if (kernel < 0 || kernel >= K_COUNT) return fail(c, UMGS_ERR_INVALID_ARG, "umgs_profile_read: kernel %d", kernel);
  umgs_status s = drain_profile(c);
  if (s != UMGS_OK) return s;
  if (launches) *launches = c->prof.n[kernel];
  if (total_ms) *total_ms = c->prof.ms[kernel];
  return UMGS_OK;
}

}  // extern "C"
