// Internal declarations of the unimgs HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/unimgs.h"

namespace umgs {

// 3DGS constants that the rasterizer follows (Section 3.2 builds on them).
constexpr float kAlphaMin = 1.0f / 255.0f;   // a fragment contributes iff alpha >= this
constexpr float kAlphaMax = 0.99f;           // alpha clamp
constexpr float kTStop = 1e-4f;              // early termination threshold
constexpr float kNear = 0.2f;                // near plane (view z)
constexpr float kDilation = 0.3f;            // EWA low-pass, px^2
constexpr float kFrustumClamp = 1.3f;        // J evaluated at x/z clamped to 1.3 tan(fov/2)
constexpr int kSubpx = 256;                  // fixed-point vertex resolution: 1/256 px
constexpr int kCoordLimit = 1 << 24;         // |snapped coordinate| bound (1/256 px)
constexpr uint32_t kCulled = 0xFFFFFFFFu;    // depth key of a culled primitive

constexpr int64_t kViewSlots = 8192;   // ViewParams the device table store holds
constexpr int kMinMaxSlots = 4096;     // slot pairs of the frame's depth-key range
// Supertiles: blocks of kST x kST tiles (kST = 8, so a supertile's tiles
// index the 64 bits of a mask), the unit of the first binning level.
constexpr int kSTLog = 3;
constexpr int kST = 1 << kSTLog;

// Floats per row of the proxy backward's per-Gaussian gradient table: the
// row's 12 terms padded to 64 B, one aligned memory sector per gather.
constexpr int kGRow = 16;

// Per-view parameters in device memory.
struct ViewParams {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float tanx, tany;      // W/(2 fx), H/(2 fy)
  int32_t W, H;
  int32_t ntx, nty;      // tile grid
  uint32_t tile_base;    // first global tile id of this view
  uint32_t st_base;      // first global supertile id of this view (8 x 8 tiles each)
  int64_t pix_base;      // first pixel of this view in the packed per-pixel arrays
};

// Projected Gaussian as the blend stage reads it (48 B, 16-B aligned).  The
// power coefficients are stored times log2(e) next to lo = log2(opacity), so
// that p = (qa dx^2 + qb dx dy + qc dy^2) + lo is log2(o exp(power)) and
// alpha = min(0.99, 2^p) takes one exp2 and no further products.
struct __align__(16) GaussRec {
  float mx, my;          // mean in pixels
  float qa, qb, qc;      // log2(e) x power coefficients (power = -d^T conic d / 2)
  float opacity;
  float r, g, b;
  float lo;              // log2(opacity)
  float inv_o;           // 1 / opacity
  float pad;
};

constexpr float kLog2e = 1.44269504088896341f;
constexpr float kLn2 = 0.69314718055994531f;
constexpr float kLog2_255 = 7.99435343685885793f;   // log2(255): alpha >= 1/255 iff p >= -this

// Set-up triangle (112 B): snapped vertices after orientation normalisation,
// per-vertex 1/z, colour/z and texture coordinates/z for perspective-correct
// interpolation, alpha, and the edge ownership bits of the tie rule.
struct __align__(16) TriRec {
  int32_t X[3], Y[3];
  float iz[3];
  float ciz[9];
  float alpha;
  uint32_t owned;        // bit k: edge k owns samples exactly on it
  float uviz[6];         // (u, v) / z per vertex (zeros without a texture)
  uint32_t swapped;      // 1: record vertices 1, 2 are input vertices 2, 1
  float pad;
};

// The triangles' RGBA texture as the blend kernels read it (no texture:
// texels == nullptr).
struct TexView {
  const float4 *texels;  // (h, w) row-major
  int32_t w, h;
};

// Kernel ids for the event-based profiler (same order as UMGS_K_* in unimgs.h).
enum KernelId {
  K_VERTEX_FRAMES = 0, K_TRANSFER, K_PROJECT, K_TRIANGLES, K_SCAN, K_EMIT, K_SORT_UPSWEEP,
  K_SORT_SCAN, K_SORT_DOWNSWEEP, K_RANGES, K_BLEND, K_BLEND_BWD, K_PROJECT_BWD, K_DEPTH_SORT,
  K_TILE_COUNT, K_TILE_SCATTER, K_ST_MASK, K_BLEND_BWD_TRI, K_TRANSFER_BWD, K_COUNT
};

struct Prof {
  bool on = false;
  std::vector<hipEvent_t> pool;
  struct Pending { int id; hipEvent_t a, b; };
  std::vector<Pending> pending;
  double ms[K_COUNT] = {};
  int64_t n[K_COUNT] = {};
};

// Per-frame sizes that the kernels after the count scan read on the device,
// so a captured graph needs no host synchronisation.
struct FrameInfo {
  uint32_t n_dup;        // duplicates (clamped to the capacity of v0)
  uint32_t depth_base;   // smallest depth-key bits of the frame
  int32_t depth_bits;    // significant bits of (depth key - depth_base)
  uint32_t n1;           // supertile entries (clamped to their capacity)
  int32_t sorted_in;     // 0: tile lists in v0 (1: in v1)
  uint32_t overflow;     // sticky: duplicates or entries exceeded a capacity
  uint32_t queue;        // reserved (kept zero)
  uint32_t n_chunks;     // second-level chunks of the frame
  uint32_t fault;        // sticky: a single-launch scan's look-back gave up (never expected)
};

// State of the single-launch scan: per tile, its total with a ready flag in
// the high word; the tile ticket and the finished-tile count.  The last tile
// of every scan leaves it all zero for the next one.
constexpr int kLbMaxTiles = 1024;
struct LbState {
  unsigned long long status[kLbMaxTiles];
  uint32_t ticket, done;
};

// Device buffer that only grows.
struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
};

struct Ctx {
  umgs_options opt;
  hipStream_t stream = nullptr;
  int device = 0;
  int num_cu = 256;
  std::string err;

  // proxy mesh
  int32_t nV = 0, nF = 0;
  DevBuf V_rest, faces, vf_ptr, vf_idx, vtab;
  DevBuf ftab;   // per face: its three vertex rows (9 float4, 144 B)
  // transfer backward: per-Gaussian gradient rows (12 floats), corner sort
  // keys and ids (ping-pong), per-face sums (36 floats)
  DevBuf tb_g, tb_key[2], tb_val[2], tb_face;   // tb_g: N rows of kGRow floats
  // BVH of the rest proxy for the binding association (rebuilt per call)
  DevBuf bvh_code[2], bvh_id[2];  // nF uint32: Morton codes / face ids (ping-pong sort)
  DevBuf bvh_tri;                 // nF x 3 float4: leaf triangles in Morton order
  DevBuf bvh_node;                // max(nF-1,1) x 4 float4: both children's boxes + links
  DevBuf bvh_aux;                 // centroid bounds, fault flag, camera centres
  DevBuf cast_code[2], cast_id[2]; // N uint32: Gaussians in Morton order of their means

  // per-frame state
  int stage = 0;         // 0 none, 1 projected, 2 binned, 3 sorted, 4 blended
  int32_t V = 0, N = 0, T = 0;
  int32_t tile_w = 16, tile_h = 16, frag_batch = 128, mode = 0, sh_degree = 0;
  float bg[3] = {0, 0, 0};
  int64_t n_records = 0;   // V * (N + T)
  int64_t n_tiles = 0;
  int64_t n_pixels = 0;
  uint64_t n_dup = 0;         // duplicates of the frame as last read on the host
  int64_t n_st = 0;           // supertiles of the frame
  int64_t n_st_max = 0;       // most supertiles of any frame so far (sizes the chunk counts)
  int st_bits = 1;            // bits of a global supertile id
  bool st_key16 = false;      // supertile ids fit 16 bits: sk holds uint16 keys
  int st_sorted = 0;          // which of sk/sv holds the sorted entries
  uint64_t st_launch = 0;     // entries the first-level grids cover (n1, or the capacity)
  uint64_t st_cap = 0;        // entries the first-level buffers hold
  // sizes of the last list-buffer growth (duplicates, entries, supertiles):
  // the buffers hold at least these, so a later eager frame can bin into
  // them before its own counts reach the host
  uint64_t list_key = 0, list_st = 0;
  int64_t list_nst = 0;
  hipEvent_t ev_totals = nullptr;   // the frame totals' readback has landed
  double st_ratio = 0.0;      // entries / duplicates of the last eager frame
  const int64_t *view_offsets = nullptr;   // caller's per-view pixel offsets (render_batched)
  DevBuf lb;           // LbState of the single-launch scan (zero between scans)
  bool lb_zeroed = false;
  DevBuf minmax;       // 2 x kMinMaxSlots uint32: min / max depth-key bits (folded in bin)
  bool minmax_ready = false;   // reset once; the bin stage resets as it folds
  DevBuf finfo;        // FrameInfo (device)
  DevBuf tile_order;   // 64 bucket counters + n_tiles tile ids (persistent blend)
  DevBuf bwd_order;    // 128 bucket counters + n_tiles keys + n_tiles tile ids + n_tiles mask words (backward)
  DevBuf pair_count;   // 4 uint64: blend work counters (measurement)
  DevBuf view_sums;    // V uint64: duplicates per view
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  uint64_t key_cap = 0;      // duplicates the key buffers hold
  bool capturing = false;    // a graph capture is in progress on the stream
  bool fixed_cap = false;    // key capacity reserved: no host readback in umgs_bin
  std::vector<ViewParams> views;
  std::vector<int32_t> view_first_tile_x;  // host copy helpers
  DevBuf d_views;            // kViewSlots view tables, appended as new camera sets appear
  std::vector<std::vector<ViewParams>> view_sets;   // host copies of the stored tables
  std::vector<int64_t> view_set_off;                // offset of each table in d_views
  int64_t view_used = 0;                            // ViewParams stored
  const ViewParams *cur_views = nullptr;            // table of the current frame
  DevBuf keys;         // n_records uint32 depth bits
  DevBuf rects;        // n_records uint2: (tx0 | ty0 << 16, tx1 | ty1 << 16) inclusive-exclusive
  DevBuf counts;       // n_records uint64: tiles | supertile entries << 32
  DevBuf dk[2], dv[2]; // n_records uint32: depth-sort keys / record ids (ping-pong)
  DevBuf offs;         // n_records + 1 uint64: supertile-entry counts in depth order, scanned
  DevBuf totals;       // 2 uint64: the frame's duplicates and supertile entries
  DevBuf grec;         // V*N GaussRec
  DevBuf trec;         // V*T TriRec
  DevBuf tex, tex_uv;  // triangle texture (tex_h, tex_w) float4 and (tex_T, 3, 2) coordinates
  int32_t tex_w = 0, tex_h = 0, tex_T = 0;
  DevBuf scan_tmp;
  DevBuf sk[2], sv[2]; // st_cap supertile ids (uint16 or uint32) / record ids (ping-pong)
  DevBuf masks[2];     // st_cap uint64: tiles of its supertile an entry reaches (ping-pong)
  DevBuf st_rng;       // n_st uint2: [start, end) of each supertile's sorted entries
  DevBuf chunk_base;   // n_st + 1 uint32: scanned second-level chunks per supertile
  DevBuf cnt2;         // chunks x 64 uint32: per-chunk tile counts / prefixes
  DevBuf chunk_tab;    // chunks x 16 B: each chunk's entries, view and supertile
  DevBuf tstart;       // n_tiles + 1 uint32: tile counts, scanned
  DevBuf v0;           // key_cap uint32: record ids in tile order (the tile lists)
  DevBuf v1;           // unused (kept null: the lists always land in v0)
  DevBuf hist;         // radix per-block histograms
  DevBuf ranges;       // n_tiles uint2
  DevBuf g2d;          // V*N x 9 per-view 2D gradients (backward)
  DevBuf host_pinned;  // not a device buffer: pinned host scratch for small readbacks
  Prof prof;
};

// Records a HIP event pair around the kernels launched in its scope when the
// context's profiler is on.
struct ScopedTimer {
  Ctx *c;
  int id;
  hipEvent_t a = nullptr, b = nullptr;
  ScopedTimer(Ctx *ctx, int kid);
  ~ScopedTimer();
};

// error helpers
umgs_status fail(Ctx *c, umgs_status s, const char *fmt, ...);
umgs_status hip_check(Ctx *c, hipError_t e, const char *what);
umgs_status ensure(Ctx *c, DevBuf &b, size_t bytes, const char *what);

// launchers (each returns the launch status)
hipError_t launch_project_gaussians(Ctx *c, const float *means, const float *cov3d,
                                    const float *scales, const float *quats,
                                    const float *opacity, const float *sh);
hipError_t launch_setup_triangles(Ctx *c, const float *tri_xyz, const float *tri_rgb,
                                  const float *tri_alpha);
hipError_t launch_exclusive_scan_u32(Ctx *c, uint32_t *data, int64_t n, uint32_t *tmp);
hipError_t launch_exclusive_scan_u64(Ctx *c, uint64_t *data, int64_t n, uint64_t *tmp);
hipError_t launch_fill_u32(Ctx *c, uint32_t *p, int64_t n, uint32_t v);
hipError_t launch_minmax_reset(Ctx *c);
size_t scan_tmp_bytes(int64_t n);
hipError_t launch_view_sums(Ctx *c, unsigned long long *sums);
hipError_t launch_depth_order(Ctx *c);
hipError_t launch_st_bin(Ctx *c);
hipError_t launch_tile_lists(Ctx *c);
uint64_t max_chunks(uint64_t n1, int64_t n_st);
size_t chunk_rec_bytes();
hipError_t launch_radix_sort_u32(Ctx *c, uint32_t *keys[2], uint32_t *vals[2], uint64_t n_launch,
                                 const uint32_t *n_dev, const int32_t *bits_dev, int bits,
                                 int kid_up, int kid_scan, int kid_down);
hipError_t launch_radix_sort_pay_u32(Ctx *c, uint32_t *keys[2], uint32_t *vals[2],
                                     uint64_t *pay[2], uint64_t n_launch, const uint32_t *n_dev,
                                     int bits, int kid_up, int kid_scan, int kid_down);
hipError_t launch_radix_sort_pay_u16(Ctx *c, uint16_t *keys[2], uint32_t *vals[2],
                                     uint64_t *pay[2], uint64_t n_launch, const uint32_t *n_dev,
                                     int bits, int kid_up, int kid_scan, int kid_down);
int radix_passes(int bits);
size_t radix_hist_bytes(uint64_t n);
hipError_t launch_expand_keys(Ctx *c, uint64_t *dst);
hipError_t launch_bvh_build(Ctx *c);
hipError_t launch_raycast(Ctx *c, int32_t N, const float *means, const float *scales,
                          const float *quats, int32_t K, int32_t C, int32_t *bind_face,
                          float *bind_bary, float *dist);
size_t bvh_aux_bytes(int32_t C);
uint32_t *bvh_fault_flag(Ctx *c);
float *bvh_cam_slots(Ctx *c);
hipError_t launch_blend(Ctx *c, float *image, float *T_final, int32_t *n_contrib,
                        float *T_entity_in, unsigned long long *pairs = nullptr);
// The context's triangle texture as the blend kernels take it.
inline TexView frame_texture(const Ctx *c) {
  TexView t;
  t.texels = c->tex_w > 0 ? (const float4 *)c->tex.p : nullptr;
  t.w = c->tex_w;
  t.h = c->tex_h;
  return t;
}
// Heaviest-first tile order of the backward walks (bwd_order: 128 bucket
// counters, n_tiles keys, n_tiles tile ids, n_tiles mask words); returns the
// order array through *order.  Tiles whose mask word is 0 (mask given) get
// key 0 and go last.
hipError_t launch_walk_order(Ctx *c, const int32_t *nc, const uint32_t **order,
                             const uint32_t *mask = nullptr);
hipError_t launch_backward_triangles(Ctx *c, const float *dL, const float *Tf, const int32_t *nc,
                                     const float *Te, float *d_rgb, float *d_alpha,
                                     bool accumulate);
hipError_t launch_backward(Ctx *c, const float *dL, const float *Tf, const int32_t *nc,
                           const float *Te, const float *means, const float *scales,
                           const float *quats, const float *xform, const float *sh,
                           float *d_means, float *d_scales, float *d_quats, float *d_opac,
                           float *d_sh, float *d_xform, bool accumulate);
// Allocation-free transfer: its scratch is a static device array of
// kNoAllocScratchBytes per GPU, whose address noalloc_scratch_init looks up
// once per device (with that device current) and noalloc_scratch returns.
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch_init(int device);
void *noalloc_scratch(int device);
size_t noalloc_transfer_bytes(int64_t nV, int64_t nF, bool vertex_table_in_scratch);
hipError_t launch_transfer_noalloc(Ctx *c, void *scratch_base, const float *V_def, int32_t N,
                                   const int32_t *bind_face, const float *bind_bary,
                                   const float *means, const float *quats, const float *scales,
                                   float *means_out, float *quats_out, float *cov3d_out,
                                   float *xform_out, float *vertex_out);
hipError_t launch_transfer_backward(Ctx *c, const float *V_def, int32_t N,
                                    const int32_t *bind_face, const float *bind_bary,
                                    const float *dL_dmeans, const float *dL_dxform,
                                    float *dL_dV_def, bool accumulate);
hipError_t launch_transfer(Ctx *c, const float *V_def, int32_t N, const int32_t *bind_face,
                           const float *bind_bary, const float *means, const float *quats,
                           const float *scales, float *means_out, float *quats_out,
                           float *cov3d_out, float *xform_out, float *vertex_out);

inline unsigned ceil_div(uint64_t a, uint64_t b) { return (unsigned)((a + b - 1) / b); }

// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each
// with its own L2.  Give every XCD a contiguous range of logical block ids so
// that neighbouring blocks -- whose outputs abut in memory -- share an L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t bid, uint32_t nb) {
  const uint32_t xcd = bid & 7u, k = bid >> 3;
  const uint32_t per = nb >> 3, rem = nb & 7u;
  return xcd * per + min(xcd, rem) + k;
}

// The same for a grid of at least nb workgroups of which only the first nb
// logical blocks have work (a grid sized for a capacity, the count known on
// the device): those nb are spread over all 8 XCDs, each a contiguous range,
// and every other workgroup gets 0xFFFFFFFF.  A bijection onto [0, nb)
// whatever the grid size >= nb.
__device__ __forceinline__ uint32_t xcd_block_n(uint32_t bid, uint32_t nb) {
  const uint32_t xcd = bid & 7u, k = bid >> 3;
  const uint32_t per = nb >> 3, rem = nb & 7u;
  return k < per + (xcd < rem ? 1u : 0u) ? xcd * per + min(xcd, rem) + k : 0xFFFFFFFFu;
}

// Wave-wide minimum / maximum of a uint32 (wave64).
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  for (int o = 32; o >= 1; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
  return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  for (int o = 32; o >= 1; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
  return v;
}

}  // namespace umgs

struct umgs_ctx {
  umgs::Ctx c;
};
