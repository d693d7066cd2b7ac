/*
 * unimgs.h -- C ABI of the MI355X (gfx950) mixed Gaussian/triangle rasterizer.
 *
 * The library renders 3D Gaussian splats and anti-aliased triangles in one
 * rasterization pass (the paper's Section 3.2, Eq. 1-11) after moving bound
 * Gaussians with a deformed proxy mesh (Section 3.3.2, Eq. 12-13).  Every
 * step runs in hand-written HIP kernels on the stream given to umgs_create.
 *
 * Conventions shared by all entry points
 *   - Arrays marked [device] are device pointers, FP32 (or int32) row-major
 *     and contiguous unless stated; [host] marks host memory.  The library
 *     never frees caller memory and never keeps caller pointers after a call
 *     returns.  Internal work buffers belong to the context.
 *   - Calls are asynchronous on the context's stream unless stated.  One
 *     context per stream; a context is not thread-safe.
 *   - Every call validates its arguments before enqueueing anything; on any
 *     error nothing has been enqueued by that call and umgs_last_error()
 *     describes it.  No C++ exception crosses the ABI.
 *   - Camera: world->camera rotation R (row-major 3x3) and translation t,
 *     OpenCV axes (x right, y down, z forward).  Pixel (i, j) covers
 *     [i, i+1) x [j, j+1); a point projects to u = fx x/z + cx,
 *     v = fy y/z + cy.
 *   - Gaussians: means (N,3); scales (N,3) linear; quats (N,4) (w,x,y,z),
 *     normalised inside; opacity (N,) in (0,1); sh (N,(deg+1)^2,3) real SH
 *     coefficients (degree-0 colour = sh0 * 0.28209479 + 0.5, clamped >= 0);
 *     cov3d (N,6) optional packed world covariance (xx,xy,xz,yy,yz,zz).
 *   - Triangles: tri_xyz (T,3,3) world vertices, tri_rgb (T,3,3) per-vertex
 *     colour, tri_alpha (T,) opacity.  Global fragment ids: Gaussians
 *     0..N-1, triangles N..N+T-1; equal depth keys order by ascending id.
 *   - Per-view outputs are packed view after view: image (3,H,W) per view
 *     (planar RGB), per-pixel arrays (H,W) per view.
 */
#ifndef UNIMGS_H
#define UNIMGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  UMGS_OK = 0,
  UMGS_ERR_INVALID_ARG = -1,  /* bad pointer, size, option or shape        */
  UMGS_ERR_CAPACITY = -2,     /* a size exceeds what the library supports   */
  UMGS_ERR_HIP = -3,          /* a HIP runtime call or launch failed        */
  UMGS_ERR_STATE = -4,        /* call out of order (e.g. blend before sort) */
  UMGS_ERR_UNSUPPORTED = -5
} umgs_status;

typedef struct umgs_ctx umgs_ctx;

typedef struct {
  float R[9];       /* world -> camera rotation, row-major                 */
  float t[3];       /* world -> camera translation                         */
  float fx, fy;     /* focal lengths in pixels                             */
  float cx, cy;     /* principal point in pixels                           */
  int32_t width, height;  /* 1 .. 16384                                    */
} umgs_camera;

typedef struct {
  int32_t tile_w, tile_h;  /* 8x8, 16x16 or 32x8                               */
  int32_t frag_batch;      /* fragments staged in LDS per batch: 32,64,128,256 */
  int32_t sh_degree;       /* 0..3                                             */
  int32_t k_bind;          /* bindings per Gaussian: 1 (centre) or 8 (corners) */
  int32_t mode;            /* compositing rule, UMGS_MODE_*                    */
  int32_t schedule;        /* blend schedule, UMGS_SCHEDULE_*                  */
  float bg[3];             /* opaque background colour                         */
} umgs_options;

/* Blend schedules: one workgroup per screen tile, or a persistent grid that
 * takes tiles from a queue ordered by fragment-list length, longest first
 * (evens out many views of uneven size and cost). */
enum { UMGS_SCHEDULE_TILE_GRID = 0, UMGS_SCHEDULE_PERSISTENT = 1 };

/* Compositing rules (Section 3.2, Fig. 3).  UMGS_MODE_UNIMGS is the paper's
 * method; the others are its ablations. */
enum {
  UMGS_MODE_UNIMGS = 0,      /* depth-adjacent triangles form one entity (Fig. 3d)   */
  UMGS_MODE_DIRECT = 1,      /* triangles alpha-blended like Gaussians (Fig. 3a)     */
  UMGS_MODE_ONE_ENTITY = 2,  /* all triangles of a pixel one entity (Fig. 3b/c)      */
  UMGS_MODE_LITERAL_T = 3    /* entity with pixel T updated per Eq. 6 with Eq. 8's O */
};

/* Default options: 16x16 tiles, batch 128, SH degree 0, K = 8, UniMGS mode,
 * one workgroup per tile, black background. */
void umgs_default_options(umgs_options *opt);

/* Create a context bound to a HIP stream (hipStream_t passed as void*, NULL =
 * the null stream).  *out receives the context.  Errors: INVALID_ARG for a
 * NULL out/opt or options outside the ranges above; HIP if the device cannot
 * be queried. */
umgs_status umgs_create(umgs_ctx **out, const umgs_options *opt, void *hip_stream);
void umgs_destroy(umgs_ctx *ctx);
/* Text of the last error on this context ("" if none).  Owned by ctx. */
const char *umgs_last_error(const umgs_ctx *ctx);
/* Replace the options; takes effect at the next umgs_project. */
umgs_status umgs_set_options(umgs_ctx *ctx, const umgs_options *opt);

/* ---- deformation transfer (Section 3.3.2, Eq. 12-13) ------------------- */

/* Upload the rest proxy mesh (setup, once): V_rest [host] (nV,3), faces
 * [host] (nF,3) int32, outward oriented.  Builds the vertex->face adjacency.
 * Synchronous.  Errors: INVALID_ARG (NULL, nV < 3, nF < 1, face index out of
 * range, a vertex without faces). */
umgs_status umgs_set_proxy(umgs_ctx *ctx, int32_t nV, const float *V_rest, int32_t nF,
                           const int32_t *faces);

/* Move N bound Gaussians with the deformed proxy V_def [device] (nV,3).
 * Per vertex: offset, cotangent-weighted 1-ring deformation gradient (with a
 * normal pair), polar decomposition and rotation log; per Gaussian: Eq. 12
 * over its K = k_bind bindings bind_face [device] (N,K) int32 and bind_bary
 * [device] (N,K,2) = (u,v) with w = 1-u-v, then Eq. 13.
 * Outputs [device]: means_out (N,3), quats_out (N,4) = quat(R') * q,
 * cov3d_out (N,6) = A Sigma A^T packed, xform_out (N,9) = A = R'S' row-major;
 * vertex_out (nV,12) = (Delta 3, log R 3, S xx,xy,xz,yy,yz,zz) may be NULL
 * (else 16-byte aligned).
 * A binding whose face index lies outside [0, nF) -- umgs_bind_raycast
 * writes -1 where no ray crosses the proxy -- is unbound (Section 3.3.1
 * leaves such corners open): Eq. 13 then averages over the k_b bound
 * bindings only, and a Gaussian with none keeps its rest pose (mu' = mu,
 * R' = S' = A = I, Sigma' = Sigma, q' = q/|q|); the barycentrics of an
 * unbound binding must be finite, their values are otherwise unused.
 * means_out follows a fixed FP32 operation order (the deformed mean orders
 * the Gaussians): Delta = V'-V; w = (1-u)-v; Delta_i = (u Da + v Db) + w Dc;
 * s = ((Delta_a + Delta_b) + ...) over the bound bindings in binding order;
 * mu' = mu + s * (1/k_b), 1/k_b rounded to FP32.
 * Errors: STATE without umgs_set_proxy; INVALID_ARG for NULL inputs,
 * N < 0, a misaligned vertex_out, or (K = 8) bind_face / bind_bary not
 * 16-byte aligned. */
umgs_status umgs_bind_transfer(umgs_ctx *ctx, const float *V_def, int32_t N,
                               const int32_t *bind_face, const float *bind_bary,
                               const float *means, const float *quats, const float *scales,
                               float *means_out, float *quats_out, float *cov3d_out,
                               float *xform_out, float *vertex_out);

/* umgs_bind_transfer for callers that cannot allocate device memory during
 * the call (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): same arguments, kernels, results and errors, but the
 * per-vertex table and the face rows live in a static device array of
 * 16 MiB (16,777,216 bytes) that every GPU the library runs on holds until
 * the process ends, instead of context buffers; the call allocates nothing
 * and synchronizes nothing.  It needs 48 * nV bytes (rounded up to 256; none
 * when vertex_out is given) + 144 * nF bytes of that array, and fails with
 * CAPACITY, before any launch, for a proxy that needs more.  All calls on
 * one GPU share the array (it keeps the last call's contents, every byte of
 * it a call reads is written by that call first): calls that overlap on one
 * GPU -- on two streams, or from two contexts -- race and must be ordered by
 * the caller. */
umgs_status umgs_bind_transfer_noalloc(umgs_ctx *ctx, const float *V_def, int32_t N,
                                       const int32_t *bind_face, const float *bind_bary,
                                       const float *means, const float *quats,
                                       const float *scales, float *means_out, float *quats_out,
                                       float *cov3d_out, float *xform_out, float *vertex_out);

/* Binding association by ray casting (Section 3.3.1), a setup step run
 * before deformation.  Each Gaussian has K target points: K = 1 its mean,
 * K = 8 the corners mu + R(q) diag(3 s) (sx, sy, sz) of its bounding box,
 * signs +-1 with the x sign varying fastest, then y, then z (q normalised
 * inside).  From each of the C camera centres cam_centers [host] (C,3) a ray
 * o + t (P - o), t > 0, is cast through the target P (at t = 1).  Every
 * crossing of a face of the rest proxy (umgs_set_proxy) is a candidate,
 * edges and vertices included; the target binds to the crossing nearest to
 * it, |t - 1| |P - o|, over all faces and cameras -- not to the first
 * crossing seen from the camera.  Ties go to the lower camera, then the lower
 * face index.
 * Inputs [device]: means (N,3); scales (N,3) and quats (N,4) (w,x,y,z), read
 * only for K = 8 (may be NULL for K = 1).
 * Outputs [device]: bind_face (N,K) int32 (-1 where no ray crosses the
 * proxy), bind_bary (N,K,2) = (u,v) with crossing = u V[f0] + v V[f1] +
 * (1-u-v) V[f2] ((0,0) for -1), the layout umgs_bind_transfer reads (which
 * leaves -1 corners out of Eq. 13); dist
 * (N,K) the distance from the crossing to the target (+inf for -1), may be
 * NULL.
 * The call builds a BVH of the proxy on the device (linear BVH over the
 * Morton codes of the face centroids) into context buffers, casts in FP32,
 * and returns after the stream has finished (synchronous).
 * Errors: STATE without a proxy or during graph capture; INVALID_ARG (N < 0,
 * K not 1 or 8, C < 1 or C > 2^20, a NULL array, a non-finite camera
 * centre); CAPACITY (N*K >= 2^31, or a traversal past its stack or step
 * bound, which the hierarchy's depth bound -- at most 30 + log2(nF) levels --
 * keeps it from reaching); HIP. */
umgs_status umgs_bind_raycast(umgs_ctx *ctx, int32_t N, const float *means, const float *scales,
                              const float *quats, int32_t K, int32_t C, const float *cam_centers,
                              int32_t *bind_face, float *bind_bary, float *dist);

/* ---- forward rasterization (Section 3.2) ---------------------------------- */

/* Project N Gaussians (EWA splatting: 2D covariance J W Sigma W^T J^T + 0.3 I,
 * conic, SH colour; the inputs to Eq. 1-2) and set up T triangles (4x
 * rotated-grid sub-sample coverage with 1/256-px fixed-point vertices: the
 * o_i^j of Eq. 4/7) for V views cams [host] (V entries).  cov3d may be NULL,
 * then scales and quats are used (else they may be NULL).  N or T may be 0
 * (their pointers may then be NULL).  Records stay in the context until the
 * next umgs_project.  Errors: INVALID_ARG (NULL where required, sizes < 0,
 * V < 1, bad camera size); CAPACITY if V*(N+T) >= 2^31. */
umgs_status umgs_project(umgs_ctx *ctx, int32_t V, const umgs_camera *cams, int32_t N,
                         const float *means, const float *cov3d, const float *scales,
                         const float *quats, const float *opacity, const float *sh,
                         int32_t T, const float *tri_xyz, const float *tri_rgb,
                         const float *tri_alpha);

/* Texture the triangles (the paper's Section 1: textured meshes carrying an
 * opacity attribute).  tex_rgba [device] (tex_h, tex_w, 4) FP32 RGBA, row j
 * of texels at v = (j + 1/2)/tex_h, column i at u = (i + 1/2)/tex_w;
 * tri_uv [device] (T,3,2) texture coordinates (u, v) of each triangle's
 * vertices.  Both are copied into the context (asynchronously on its
 * stream: the caller may free them after the stream reaches this call).
 * Every later umgs_project / umgs_render_batched of T triangles then shades a
 * triangle at each pixel centre with the perspective-correct interpolation
 * of its texture coordinates: a bilinear fetch (addresses clamped to the
 * edge texels), colour = per-vertex colour x texel RGB, opacity =
 * tri_alpha x texel alpha; sub-sample coverage and depth keys do not change.
 * tex_rgba NULL removes the texture (untextured shading).  Not while
 * capturing a graph.  Errors: INVALID_ARG (sizes outside 1..16384, T < 0, a
 * NULL tri_uv with T > 0), STATE, CAPACITY, HIP; umgs_project then fails
 * with INVALID_ARG if its triangle count is not T. */
umgs_status umgs_set_texture(umgs_ctx *ctx, int32_t tex_w, int32_t tex_h, const float *tex_rgba,
                             int32_t T, const float *tri_uv);

/* Bin (first level of the mixed depth sort of Section 3.2): the projected
 * primitives in (depth key, record id) order, then one (supertile, record)
 * entry for every supertile -- a block of 8 x 8 tiles -- that the
 * primitive's support reaches, stably sorted by supertile id, so each
 * supertile's entries are front to back.  Without a reservation it
 * synchronizes the stream once to size the buffers of the duplicates (one
 * per (tile, primitive) pair the support reaches) and of the entries; after
 * umgs_reserve it does not synchronize, and duplicates or entries beyond the
 * reserved capacity are dropped and flagged (see umgs_query).  Errors:
 * STATE before umgs_project; CAPACITY if the duplicate or entry count
 * reaches 2^32 - 2^16 or a buffer cannot be allocated. */
umgs_status umgs_bin(umgs_ctx *ctx);

/* Sort (second level): every tile's list of record ids, front to back --
 * the order of the (tile, depth key, record id) keys, ties by ascending id --
 * and every tile's [start, end) range in it.  Each supertile's entries are
 * split into the tiles they reach by a counting sort, so each duplicate is
 * written once, to its final place.  Errors: STATE before umgs_bin. */
umgs_status umgs_sort(umgs_ctx *ctx);

/* Blend every tile front to back (Eq. 1-2 for Gaussians, Eq. 7-9 for
 * triangle entities, Eq. 10-11 background) with early termination.
 * Outputs [device], packed per view: image (3,H,W) FP32, T_final (H,W),
 * n_contrib (H,W) int32 = 1 + position in the tile's sorted list of the last
 * blended fragment (0 if none), T_entity_in (H,W) = transmittance in front of
 * the last blended unit -- a Gaussian, or a whole triangle entity (a single
 * triangle in UMGS_MODE_DIRECT) -- (1 if none); the backward pass needs it
 * when that unit is opaque.  T_final, n_contrib and
 * T_entity_in may be NULL.  Errors: STATE before umgs_sort. */
umgs_status umgs_blend(umgs_ctx *ctx, float *image, float *T_final, int32_t *n_contrib,
                       float *T_entity_in);

/* Batched frame of V views (Section 3.2's renderer over many views at
 * once): umgs_project, umgs_bin, umgs_sort and umgs_blend in one call, the
 * blend with the persistent longest-list-first schedule, which evens out
 * views of very different size.  view_offsets [host, V + 1 entries; NULL =
 * views packed in order] places view v's pixels at element view_offsets[v]
 * of the per-pixel outputs (and at 3 x that of image, whose views are
 * (3,H,W) blocks); view v must end at or before view_offsets[v + 1], and
 * view_offsets[V] is the outputs' length in pixels.  Elements between views
 * are not written.  The other arguments are those of umgs_project and
 * umgs_blend.  Like every call it may be captured into a graph between
 * umgs_graph_begin and umgs_graph_end (after umgs_reserve).  Errors: those
 * of the four calls; INVALID_ARG, before any launch, for offsets that
 * decrease or let views overlap or overrun view_offsets[V]. */
umgs_status umgs_render_batched(umgs_ctx *ctx, int32_t V, const umgs_camera *cams,
                                const int64_t *view_offsets, int32_t N, const float *means,
                                const float *cov3d, const float *scales, const float *quats,
                                const float *opacity, const float *sh, int32_t T,
                                const float *tri_xyz, const float *tri_rgb, const float *tri_alpha,
                                float *image, float *T_final, int32_t *n_contrib,
                                float *T_entity_in);

/* ---- backward (gradients through the blend of Section 3.2) ----------------- */

/* Gradients of a loss L with respect to the Gaussians of the last blended
 * frame on this context, given dL_dimage [device] (same layout as image).
 * T_final, n_contrib and T_entity_in are the per-pixel outputs of that
 * umgs_blend call (the backward recovers the transmittance in front of every
 * fragment from them instead of storing per-fragment state).  means are the
 * means that were projected; the projected covariance must have been
 * A Sigma(scales, quats) A^T with A = xform [device] (N,9) row-major, or
 * Sigma(scales, quats) when xform is NULL (deformed scenes pass the A
 * written by umgs_bind_transfer; the mean offset is constant, so the
 * gradient of the rest mean equals that of the deformed mean).
 * Outputs [device]: dL_dmeans (N,3), dL_dscales (N,3) w.r.t. linear scales,
 * dL_dquats (N,4) w.r.t. the raw quaternion before normalisation,
 * dL_dopacity (N,), dL_dsh (N,(deg+1)^2,3); dL_dxform (N,9) w.r.t. A when
 * both xform and dL_dxform are non-NULL (what umgs_backward_transfer takes
 * on to the proxy vertices; ignored otherwise); written when accumulate is
 * 0, added to their contents otherwise (to sum over groups of views
 * rendered by separate frames).
 * Triangle gradients come from umgs_backward_triangles.  Float atomics make the summation order,
 * hence the last bits, run-dependent.  Errors: STATE without a blended
 * frame; UNSUPPORTED for UMGS_MODE_ONE_ENTITY and UMGS_MODE_LITERAL_T;
 * INVALID_ARG for NULL arrays. */
umgs_status umgs_backward(umgs_ctx *ctx, const float *dL_dimage, const float *T_final,
                          const int32_t *n_contrib, const float *T_entity_in, const float *means,
                          const float *scales, const float *quats, const float *xform,
                          const float *sh, float *dL_dmeans, float *dL_dscales, float *dL_dquats,
                          float *dL_dopacity, float *dL_dsh, float *dL_dxform, int32_t accumulate);

/* Gradient with respect to the deformed proxy vertices V_def [device]
 * (nV,3) of a loss given its gradients with respect to the transfer's
 * outputs (Section 3.3.2): dL_dmeans (N,3) w.r.t. the deformed means mu'
 * and dL_dxform (N,9) w.r.t. A = R'S' (as umgs_backward writes them for a
 * frame whose Gaussians came from umgs_bind_transfer with this V_def and
 * these bindings; either may be NULL, meaning zero).  Eq. 12-13 and the
 * per-vertex transform (the 1-ring least squares D, the polar D = RS, the
 * principal log of R) are differentiated exactly, the per-vertex part in
 * FP64; the bindings are the same arrays as umgs_bind_transfer's (corners
 * outside [0, nF) unbound and without gradient).  Output dL_dV_def (nV,3)
 * [device], written when accumulate is 0, added to otherwise.  Float
 * atomics make the last bits run-dependent.  Capturable once an eager call
 * with the same N has sized its buffers.  Errors: STATE without a proxy;
 * INVALID_ARG for N < 0 or NULL arrays; CAPACITY (also when capturing a
 * call that would need larger buffers). */
umgs_status umgs_backward_transfer(umgs_ctx *ctx, const float *V_def, int32_t N,
                                   const int32_t *bind_face, const float *bind_bary,
                                   const float *dL_dmeans, const float *dL_dxform,
                                   float *dL_dV_def, int32_t accumulate);

/* Gradients of L with respect to the triangles of the last blended frame:
 * their per-vertex colours and opacity attributes, through the sub-sample
 * entity blend of Eq. 7-9 (UMGS_MODE_UNIMGS) or the per-triangle blend of
 * UMGS_MODE_DIRECT, with coverage held fixed (a step function of the
 * geometry, whose derivative is zero almost everywhere).  The per-pixel
 * inputs are those of umgs_backward.  A textured triangle's colour is
 * rgb x texel RGB and its opacity alpha x texel alpha; the texels are
 * constants here (no texture gradient).
 * Outputs [device]: dL_dtri_rgb (T,3,3) in the vertex order of tri_rgb,
 * dL_dtri_alpha (T,); summed over the frame's views; written when
 * accumulate is 0, added to their contents otherwise.  Independent of
 * umgs_backward (either may run first, or alone).  Float atomics make the
 * last bits run-dependent.  Errors: STATE without a blended frame;
 * UNSUPPORTED for UMGS_MODE_ONE_ENTITY and UMGS_MODE_LITERAL_T;
 * INVALID_ARG for NULL arrays. */
umgs_status umgs_backward_triangles(umgs_ctx *ctx, const float *dL_dimage, const float *T_final,
                                    const int32_t *n_contrib, const float *T_entity_in,
                                    float *dL_dtri_rgb, float *dL_dtri_alpha, int32_t accumulate);

/* ---- graphs: capture one step, replay it ----------------------------------- */

/* Reserve the tile lists for max_dup duplicates and stop synchronizing in
 * umgs_bin (the later stages then read the frame's sizes on the device); 0
 * returns to the synchronizing mode.  The supertile entries get 1.25 x
 * max_dup x the entries-per-duplicate ratio of the last eager frame (at
 * least 2^16, at most max_dup).  Call it after one eager frame of the same
 * shape (which sizes every other buffer).  Errors: CAPACITY. */
umgs_status umgs_reserve(umgs_ctx *ctx, int64_t max_dup);
/* Begin capturing the context stream into a graph: the entry points called
 * until umgs_graph_end are recorded, not run.  Requires a reservation,
 * profiling off, a non-null stream, and umgs_project calls with camera sets
 * that eager frames have used before (the context keeps one device table per
 * distinct camera set; a frame rendered in several view groups has one per
 * group).  Any entry point that would allocate or synchronize while
 * capturing fails with STATE or CAPACITY.  Errors: STATE, HIP. */
umgs_status umgs_graph_begin(umgs_ctx *ctx);
/* End the capture and instantiate the graph (replacing any previous one). */
umgs_status umgs_graph_end(umgs_ctx *ctx);
/* Launch the instantiated graph on the context stream (asynchronous). */
umgs_status umgs_graph_launch(umgs_ctx *ctx);
/* Replace the stored camera set old_cams [host] (V views) by new_cams for the
 * next replays; every view keeps its width and height.  Asynchronous on the
 * stream.  Errors: INVALID_ARG, STATE (no stored set equals old_cams). */
umgs_status umgs_update_views(umgs_ctx *ctx, int32_t V, const umgs_camera *old_cams,
                              const umgs_camera *new_cams);
/* Upper bound of the duplicates each view of the projected frame will
 * produce, dups [host] (V entries): the tiles of its primitives' bounding
 * rectangles (the tile lists keep those the support reaches), known before
 * umgs_bin allocates anything: used to split a batch whose duplicates exceed
 * the 32-bit positions of one frame into view groups.  Synchronous.
 * Errors: STATE. */
umgs_status umgs_view_dups(umgs_ctx *ctx, int64_t *dups);

/* Measurement: blend the sorted frame again into image [device] while
 * counting; pairs [host, 4 entries] receives {Gaussian pairs, triangle
 * pairs, wave iterations, staged fragments}: the (pixel, fragment) pairs
 * evaluated before each pixel is done, the fragment-loop iterations of all
 * 64-lane waves, and the fragments loaded into LDS.  The algorithmic work of
 * the blend is the pair counts times the per-pair operation counts; 64 times
 * the wave iterations over the pairs is the SIMD-lane occupancy lost to
 * pixels of one wave finishing at different depths.  Synchronous.  Errors:
 * STATE before umgs_sort. */
umgs_status umgs_blend_pairs(umgs_ctx *ctx, float *image, int64_t *pairs);

/* Sizes of the current frame: n_dup (duplicates in the tile lists after
 * umgs_sort, at most the reserved capacity; after umgs_bin alone, the
 * rectangles' upper bound), n_tiles (all views), the record count V*(N+T) and
 * overflow (1 if duplicates were dropped since the flag was last read; the
 * flag is cleared by reading it).  Any pointer may be NULL.  Synchronous. */
umgs_status umgs_query(umgs_ctx *ctx, int64_t *n_dup, int64_t *n_tiles, int64_t *n_records,
                       int32_t *overflow);

/* First-level sizes of the last binned frame: supertiles (blocks of 8 x 8
 * tiles over all views) and (supertile, primitive) entries.  Synchronizes
 * the stream.  Errors: STATE before umgs_bin or while capturing. */
umgs_status umgs_query_bins(umgs_ctx *ctx, int64_t *n_supertiles, int64_t *n_entries);

/* Copy internal per-frame state into caller memory [device] (for tests):
 *   UMGS_STATE_KEYS    n_records uint32 depth-key bits (0xFFFFFFFF = culled)
 *   UMGS_STATE_SORTED_KEYS  n_dup uint64 sorted keys
 *   UMGS_STATE_SORTED_VALS  n_dup uint32 record ids in sorted order
 *   UMGS_STATE_RANGES  n_tiles x 2 uint32 [start, end) per global tile
 *   UMGS_STATE_TRI_FIXED  V*T x 6 int32 snapped vertices (X0,X1,X2,Y0,Y1,Y2)
 *                         after orientation normalisation (0 when culled)
 *   UMGS_STATE_GRAD2D  V*N x 9 float gradients of the last umgs_backward with
 *                      respect to each projected Gaussian: mean (2), power
 *                      coefficients of dx^2, dx dy, dy^2 (3), opacity, rgb (3)
 * cap_bytes must hold the whole array.  Errors: INVALID_ARG, STATE. */
enum { UMGS_STATE_KEYS = 0, UMGS_STATE_SORTED_KEYS = 1, UMGS_STATE_SORTED_VALS = 2,
       UMGS_STATE_RANGES = 3, UMGS_STATE_TRI_FIXED = 4, UMGS_STATE_GRAD2D = 5 };
umgs_status umgs_copy_state(umgs_ctx *ctx, int32_t which, void *dst, int64_t cap_bytes);

/* ---- kernel timing -------------------------------------------------------- */

/* Per-kernel timing with HIP events recorded on the context stream around
 * each launch (UMGS_K_* ids).  umgs_set_profiling enables or disables it and
 * clears the totals; umgs_profile_read synchronizes the stream and returns
 * the number of timed launches and their total duration.  Keep profiling off
 * while a stream is being captured into a graph. */
enum { UMGS_K_VERTEX_FRAMES = 0, UMGS_K_TRANSFER = 1, UMGS_K_PROJECT = 2, UMGS_K_TRIANGLES = 3,
       UMGS_K_SCAN = 4, UMGS_K_EMIT = 5, UMGS_K_SORT_UPSWEEP = 6, UMGS_K_SORT_SCAN = 7,
       UMGS_K_SORT_DOWNSWEEP = 8, UMGS_K_RANGES = 9, UMGS_K_BLEND = 10, UMGS_K_BLEND_BWD = 11,
       UMGS_K_PROJECT_BWD = 12, UMGS_K_DEPTH_SORT = 13, UMGS_K_TILE_COUNT = 14,
       UMGS_K_TILE_SCATTER = 15, UMGS_K_ST_MASK = 16, UMGS_K_BLEND_BWD_TRI = 17,
       UMGS_K_TRANSFER_BWD = 18, UMGS_K_COUNT = 19 };
umgs_status umgs_set_profiling(umgs_ctx *ctx, int32_t enable);
umgs_status umgs_profile_read(umgs_ctx *ctx, int32_t kernel, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* UNIMGS_H */
