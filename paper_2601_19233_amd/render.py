"""Python binding of the C ABI (argument marshalling only).

Every step of the path runs in the HIP kernels of libunimgs.so; PyTorch only
provides device memory and the stream.  Names follow the C entry points.
"""
from __future__ import annotations

import contextlib
import ctypes as C
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _f32(x, device) -> Optional[torch.Tensor]:
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.float32).contiguous()
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(device)


def _i32(x, device) -> Optional[torch.Tensor]:
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.int32).contiguous()
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).to(device)


def camera_struct(cam) -> L.Camera:
    c = L.Camera()
    R = np.asarray(cam.R, np.float32).reshape(9)
    t = np.asarray(cam.t, np.float32).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def make_options(tile=(16, 16), frag_batch=128, sh_degree=0, k_bind=8, mode=0, schedule=0,
                 bg=(0.0, 0.0, 0.0)) -> L.Options:
    o = L.Options()
    o.tile_w, o.tile_h = int(tile[0]), int(tile[1])
    o.frag_batch = int(frag_batch)
    o.sh_degree = int(sh_degree)
    o.k_bind = int(k_bind)
    o.mode = int(mode)
    o.schedule = int(schedule)
    for k in range(3):
        o.bg[k] = float(bg[k])
    return o


class Rasterizer:
    """One library context bound to a stream on one device.

    By default the context uses the caller's current stream.  With
    ``own_stream=True`` (needed for graph capture, since the null stream
    cannot be captured) it gets a stream of its own at default priority, and
    every call orders it after the caller's current stream and the caller's
    stream after it."""

    def __init__(self, device="cuda:0", stream: Optional[torch.cuda.Stream] = None,
                 own_stream: bool = False, **opts):
        self.lib = L.load()
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        if stream is None:
            stream = torch.cuda.Stream(self.device) if own_stream else torch.cuda.current_stream(self.device)
        self.stream = stream
        self._capturing = False
        self.opts = make_options(**opts)
        h = C.c_void_p()
        st = self.lib.umgs_create(C.byref(h), C.byref(self.opts), C.c_void_p(self.stream.cuda_stream))
        if st != L.UMGS_OK:
            raise L.UmgsError(st, "umgs_create failed (invalid options or no HIP device)")
        self.h = h
        self.views: List = []
        self.N = self.T = 0
        self._keep: list = []

    def close(self):
        if getattr(self, "h", None):
            self.lib.umgs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != L.UMGS_OK:
            raise L.UmgsError(st, self.lib.umgs_last_error(self.h).decode())

    @contextlib.contextmanager
    def _on_stream(self):
        """Run library calls on the context stream, ordered after the caller's
        current stream (inputs) and before it (outputs); no cross-stream
        waits while a graph is being captured."""
        cur = torch.cuda.current_stream(self.device)
        other = cur.cuda_stream != self.stream.cuda_stream
        if other and not self._capturing:
            self.stream.wait_stream(cur)
        with torch.cuda.stream(self.stream):
            yield
        if other and not self._capturing:
            cur.wait_stream(self.stream)

    def set_options(self, **opts):
        self.opts = make_options(**opts)
        self._check(self.lib.umgs_set_options(self.h, C.byref(self.opts)))

    # ---- deformation transfer -------------------------------------------
    def set_proxy(self, V_rest, faces):
        V = np.ascontiguousarray(V_rest, np.float32)
        F = np.ascontiguousarray(faces, np.int32)
        self.nV = V.shape[0]
        self.nF = F.shape[0]
        self._check(self.lib.umgs_set_proxy(self.h, V.shape[0], V.ctypes.data_as(C.c_void_p),
                                            F.shape[0], F.ctypes.data_as(C.c_void_p)))

    def bind_raycast(self, means, scales, quats, K: int, cam_centers) -> Dict[str, torch.Tensor]:
        """Section 3.3.1 binding association on the GPU: rays from the camera
        centres (C,3) through each Gaussian's K = 1 centre or K = 8 box
        corners into the rest proxy; returns face (N,K) int32, bary (N,K,2)
        and dist (N,K), ready for bind_transfer."""
        d = self.device
        means, scales, quats = (_f32(x, d) for x in (means, scales, quats))
        oc = np.ascontiguousarray(np.asarray(cam_centers, np.float32).reshape(-1, 3))
        N = means.shape[0]
        out = dict(face=torch.empty((N, K), dtype=torch.int32, device=d),
                   bary=torch.empty((N, K, 2), device=d), dist=torch.empty((N, K), device=d))
        with self._on_stream():
            self._check(self.lib.umgs_bind_raycast(
                self.h, N, _ptr(means), _ptr(scales), _ptr(quats), K, oc.shape[0],
                oc.ctypes.data_as(C.POINTER(C.c_float)), _ptr(out["face"]), _ptr(out["bary"]),
                _ptr(out["dist"])))
        return out

    def bind_transfer(self, V_def, bind_face, bind_bary, means, quats, scales,
                      with_vertex: bool = False, out: Optional[Dict] = None,
                      noalloc: bool = False) -> Dict[str, torch.Tensor]:
        """Eq. 12-13 transfer (umgs_bind_transfer; umgs_bind_transfer_noalloc
        with ``noalloc``, whose scratch is the library's static per-GPU array)."""
        d = self.device
        V_def, means, quats, scales = (_f32(x, d) for x in (V_def, means, quats, scales))
        bind_face = _i32(bind_face, d)
        bind_bary = _f32(bind_bary, d)
        N = means.shape[0]
        K = self.opts.k_bind
        if bind_face.numel() != N * K or bind_bary.numel() != 2 * N * K:
            raise ValueError(f"bindings must be (N, {K}) faces and (N, {K}, 2) barycentrics")
        if out is None:
            out = dict(means=torch.empty((N, 3), device=d), quats=torch.empty((N, 4), device=d),
                       cov3d=torch.empty((N, 6), device=d), xform=torch.empty((N, 9), device=d))
        vert = torch.empty((self.nV, 12), device=d) if with_vertex else None
        with self._on_stream():
            fn = self.lib.umgs_bind_transfer_noalloc if noalloc else self.lib.umgs_bind_transfer
            self._check(fn(
                self.h, _ptr(V_def), N, _ptr(bind_face), _ptr(bind_bary), _ptr(means), _ptr(quats),
                _ptr(scales), _ptr(out["means"]), _ptr(out["quats"]), _ptr(out["cov3d"]),
                _ptr(out["xform"]), _ptr(vert)))
        if vert is not None:
            out["vertex"] = vert
        return out

    # ---- textured triangles ---------------------------------------------------
    def set_texture(self, tex=None, tri_uv=None):
        """RGBA texture (H, W, 4) and per-vertex texture coordinates (T, 3, 2)
        of the triangles for the following frames (umgs_set_texture); None
        removes the texture."""
        if tex is None:
            self._check(self.lib.umgs_set_texture(self.h, 0, 0, None, 0, None))
            self._tex = None
            return
        d = self.device
        tex = _f32(tex, d)
        uv = _f32(tri_uv, d)
        if tex.dim() != 3 or tex.shape[2] != 4:
            raise ValueError("the texture must be (H, W, 4) RGBA")
        T = 0 if uv is None else uv.numel() // 6
        if uv is not None and uv.numel() != 6 * T:
            raise ValueError("tri_uv must be (T, 3, 2)")
        with self._on_stream():
            self._check(self.lib.umgs_set_texture(self.h, tex.shape[1], tex.shape[0], _ptr(tex), T,
                                                  _ptr(uv)))
        self._tex = (tex, uv)       # kept alive until the copies on the stream are done

    # ---- forward ------------------------------------------------------------
    def _scene_args(self, means=None, opacity=None, sh=None, scales=None, quats=None, cov3d=None,
                    tri_xyz=None, tri_rgb=None, tri_alpha=None):
        """Device float32 copies of the scene arrays, checked against the sizes
        the kernels read (N Gaussians, T triangles)."""
        d = self.device
        means, opacity, sh, scales, quats, cov3d = (_f32(x, d) for x in (means, opacity, sh, scales, quats, cov3d))
        tri_xyz, tri_rgb, tri_alpha = (_f32(x, d) for x in (tri_xyz, tri_rgb, tri_alpha))
        N = 0 if means is None else means.shape[0]
        T = 0 if tri_xyz is None else tri_xyz.shape[0]
        nc = 3 * (self.opts.sh_degree + 1) ** 2
        if N and (sh is None or sh.numel() != N * nc):
            raise ValueError(f"sh must hold {nc} floats per Gaussian for sh_degree {self.opts.sh_degree}")
        if N and opacity is None:
            raise ValueError("opacity is required")
        if N and cov3d is None and (scales is None or quats is None):
            raise ValueError("give cov3d, or scales and quats")
        for name, t, w in (("means", means, 3), ("opacity", opacity, 1), ("scales", scales, 3),
                           ("quats", quats, 4), ("cov3d", cov3d, 6)):
            if N and t is not None and t.numel() != N * w:
                raise ValueError(f"{name} must hold {w} floats per Gaussian")
        for name, t, w in (("tri_rgb", tri_rgb, 9), ("tri_alpha", tri_alpha, 1)):
            if T and (t is None or t.numel() != T * w):
                raise ValueError(f"{name} must hold {w} floats per triangle")
        if T and tri_xyz.numel() != T * 9:
            raise ValueError("tri_xyz must hold 9 floats per triangle")
        g = dict(means=means, opacity=opacity, sh=sh, scales=scales, quats=quats, cov3d=cov3d,
                 tri_xyz=tri_xyz, tri_rgb=tri_rgb, tri_alpha=tri_alpha)
        return g, N, T

    def project(self, cams: Sequence, means=None, opacity=None, sh=None, scales=None, quats=None,
                cov3d=None, tri_xyz=None, tri_rgb=None, tri_alpha=None):
        g, N, T = self._scene_args(means, opacity, sh, scales, quats, cov3d, tri_xyz, tri_rgb, tri_alpha)
        means, opacity, sh, scales, quats, cov3d = (g[k] for k in ("means", "opacity", "sh", "scales",
                                                                  "quats", "cov3d"))
        tri_xyz, tri_rgb, tri_alpha = g["tri_xyz"], g["tri_rgb"], g["tri_alpha"]
        arr = (L.Camera * len(cams))(*[camera_struct(c) for c in cams])
        self._keep = [means, opacity, sh, scales, quats, cov3d, tri_xyz, tri_rgb, tri_alpha]
        with self._on_stream():
            self._check(self.lib.umgs_project(self.h, len(cams), arr, N, _ptr(means), _ptr(cov3d),
                                              _ptr(scales), _ptr(quats), _ptr(opacity), _ptr(sh), T,
                                              _ptr(tri_xyz), _ptr(tri_rgb), _ptr(tri_alpha)))
        self.views = [(int(c.width), int(c.height)) for c in cams]
        self.N, self.T = N, T
        self.frame_id = getattr(self, "frame_id", 0) + 1

    def bin(self):
        with self._on_stream():
            self._check(self.lib.umgs_bin(self.h))

    def sort(self):
        with self._on_stream():
            self._check(self.lib.umgs_sort(self.h))

    def alloc_outputs(self, want_state: bool = True) -> Dict[str, torch.Tensor]:
        d = self.device
        npix = sum(w * h for w, h in self.views)
        return dict(image=torch.empty(3 * npix, device=d),
                    T_final=torch.empty(npix, device=d) if want_state else None,
                    n_contrib=torch.empty(npix, device=d, dtype=torch.int32) if want_state else None,
                    T_entity_in=torch.empty(npix, device=d) if want_state else None)

    def blend(self, want_state: bool = True, out: Optional[Dict] = None) -> Dict[str, torch.Tensor]:
        if out is None:
            out = self.alloc_outputs(want_state)
        npix = sum(w * h for w, h in self.views)
        for name, per in (("image", 3), ("T_final", 1), ("n_contrib", 1), ("T_entity_in", 1)):
            t = out.get(name)
            if t is not None and (t.numel() != per * npix or not t.is_contiguous()):
                raise ValueError(f"blend output {name} must be contiguous with {per * npix} elements")
        with self._on_stream():
            self._check(self.lib.umgs_blend(self.h, _ptr(out["image"]), _ptr(out["T_final"]),
                                            _ptr(out["n_contrib"]), _ptr(out["T_entity_in"])))
        return out

    def backward(self, dL_dimage: torch.Tensor, fwd: Dict[str, torch.Tensor], means, scales, quats,
                 sh, xform=None, out: Optional[Dict] = None, accumulate: bool = False
                 ) -> Dict[str, torch.Tensor]:
        """Gradients of the last blended frame (umgs_backward).  ``fwd`` is the
        dict returned by blend(); ``means`` are the projected means."""
        d = self.device
        means, scales, quats, sh, xform = (_f32(x, d) for x in (means, scales, quats, sh, xform))
        dL = _f32(dL_dimage, d)
        N = self.N
        nc = 3 * (self.opts.sh_degree + 1) ** 2
        if out is None:
            out = dict(means=torch.empty((N, 3), device=d), scales=torch.empty((N, 3), device=d),
                       quats=torch.empty((N, 4), device=d), opacity=torch.empty((N,), device=d),
                       sh=torch.empty((N, nc), device=d))
            if xform is not None:
                out["xform"] = torch.empty((N, 9), device=d)
        if dL.numel() != fwd["image"].numel():
            raise ValueError("dL_dimage must have the image's shape")
        with self._on_stream():
            self._check(self.lib.umgs_backward(
                self.h, _ptr(dL), _ptr(fwd["T_final"]), _ptr(fwd["n_contrib"]), _ptr(fwd["T_entity_in"]),
                _ptr(means), _ptr(scales), _ptr(quats), _ptr(xform), _ptr(sh), _ptr(out["means"]),
                _ptr(out["scales"]), _ptr(out["quats"]), _ptr(out["opacity"]), _ptr(out["sh"]),
                _ptr(out.get("xform")), 1 if accumulate else 0))
        return out

    def backward_transfer(self, V_def, bind_face, bind_bary, dL_dmeans=None, dL_dxform=None,
                          out: Optional[torch.Tensor] = None, accumulate: bool = False) -> torch.Tensor:
        """dL/dV_def (nV,3) of the deformed proxy from the gradients with
        respect to the transferred means and A (umgs_backward_transfer):
        ``dL_dmeans`` and ``dL_dxform`` as backward() returns them as
        "means" and "xform" for a frame whose Gaussians came from
        bind_transfer(V_def, bind_face, bind_bary, ...)."""
        d = self.device
        V_def = _f32(V_def, d)
        face = _i32(bind_face, d)
        bary = _f32(bind_bary, d)
        N = int(face.shape[0])
        dm = None if dL_dmeans is None else _f32(dL_dmeans, d)
        dx = None if dL_dxform is None else _f32(dL_dxform, d)
        nV = int(V_def.numel() // 3)
        if out is None:
            out = torch.empty((nV, 3), device=d)
        with self._on_stream():
            self._check(self.lib.umgs_backward_transfer(
                self.h, _ptr(V_def), N, _ptr(face), _ptr(bary), _ptr(dm), _ptr(dx), _ptr(out),
                1 if accumulate else 0))
        return out

    def backward_triangles(self, dL_dimage: torch.Tensor, fwd: Dict[str, torch.Tensor],
                           out: Optional[Dict] = None, accumulate: bool = False
                           ) -> Dict[str, torch.Tensor]:
        """Gradients of the last blended frame with respect to the triangles'
        per-vertex colours (T,3,3) and opacity attributes (T,)
        (umgs_backward_triangles); ``fwd`` is the dict returned by blend()."""
        d = self.device
        dL = _f32(dL_dimage, d)
        T = self.T
        if out is None:
            out = dict(tri_rgb=torch.empty((T, 3, 3), device=d), tri_alpha=torch.empty((T,), device=d))
        if dL.numel() != fwd["image"].numel():
            raise ValueError("dL_dimage must have the image's shape")
        with self._on_stream():
            self._check(self.lib.umgs_backward_triangles(
                self.h, _ptr(dL), _ptr(fwd["T_final"]), _ptr(fwd["n_contrib"]), _ptr(fwd["T_entity_in"]),
                _ptr(out["tri_rgb"]), _ptr(out["tri_alpha"]), 1 if accumulate else 0))
        return out

    def render_batched(self, cams: Sequence, view_offsets: Optional[Sequence[int]] = None,
                       out: Optional[Dict] = None, **scene) -> Dict[str, torch.Tensor]:
        """umgs_render_batched: project, bin, sort and blend V views in one
        call with the persistent blend schedule.  ``view_offsets`` (V + 1
        pixel offsets: view v starts at element offs[v] of the per-pixel
        outputs and must end by offs[v + 1]; offs[V] is their length) places
        each view inside the outputs; by default views are packed in order."""
        d = self.device
        g, N, T = self._scene_args(**scene)
        sizes = [int(c.width) * int(c.height) for c in cams]
        if view_offsets is None:
            offs = None
            npix = sum(sizes)
        else:
            offs = [int(o) for o in view_offsets]
            if len(offs) != len(cams) + 1:
                raise ValueError("view_offsets needs V + 1 entries")
            npix = offs[-1]
        if out is None:
            out = dict(image=torch.zeros(3 * npix, device=d), T_final=torch.zeros(npix, device=d),
                       n_contrib=torch.zeros(npix, device=d, dtype=torch.int32),
                       T_entity_in=torch.zeros(npix, device=d))
        for name, per in (("image", 3), ("T_final", 1), ("n_contrib", 1), ("T_entity_in", 1)):
            tt = out.get(name)
            if tt is not None and (tt.numel() < per * npix or not tt.is_contiguous()):
                raise ValueError(f"output {name} must be contiguous with at least {per * npix} elements")
        arr = (L.Camera * len(cams))(*[camera_struct(c) for c in cams])
        off_arr = (C.c_int64 * len(offs))(*offs) if offs is not None else None
        self._keep = list(g.values())
        with self._on_stream():
            self._check(self.lib.umgs_render_batched(
                self.h, len(cams), arr, off_arr, N, _ptr(g["means"]), _ptr(g["cov3d"]),
                _ptr(g["scales"]), _ptr(g["quats"]), _ptr(g["opacity"]), _ptr(g["sh"]), T,
                _ptr(g["tri_xyz"]), _ptr(g["tri_rgb"]), _ptr(g["tri_alpha"]), _ptr(out["image"]),
                _ptr(out.get("T_final")), _ptr(out.get("n_contrib")), _ptr(out.get("T_entity_in"))))
        self.views = [(int(c.width), int(c.height)) for c in cams]
        self.N, self.T = N, T
        self.frame_id = getattr(self, "frame_id", 0) + 1
        return out

    def render(self, cams, **scene) -> Dict[str, torch.Tensor]:
        self.project(cams, **scene)
        self.bin()
        self.sort()
        return self.blend()

    def split_views(self, flat: torch.Tensor, channels: int) -> List[torch.Tensor]:
        out, o = [], 0
        for w, h in self.views:
            n = channels * w * h
            out.append(flat[o:o + n].view(channels, h, w) if channels > 1 else flat[o:o + n].view(h, w))
            o += n
        return out

    # ---- kernel timing ------------------------------------------------------
    def set_profiling(self, on: bool):
        self._check(self.lib.umgs_set_profiling(self.h, 1 if on else 0))

    def profile(self) -> Dict[str, tuple]:
        """{kernel name: (launches, total ms)} since profiling was enabled."""
        out = {}
        for k, name in enumerate(L.KERNEL_NAMES):
            n, ms = C.c_int64(), C.c_double()
            self._check(self.lib.umgs_profile_read(self.h, k, C.byref(n), C.byref(ms)))
            if n.value:
                out[name] = (n.value, ms.value)
        return out

    # ---- inspection ---------------------------------------------------------
    def query(self):
        """(n_dup, n_tiles, n_records); synchronizes."""
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self.lib.umgs_query(self.h, C.byref(a), C.byref(b), C.byref(c), None))
        return a.value, b.value, c.value

    def query_bins(self):
        """(supertiles, supertile entries) of the last binned frame; synchronizes."""
        a, b = C.c_int64(), C.c_int64()
        self._check(self.lib.umgs_query_bins(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def overflowed(self) -> bool:
        """Whether duplicates were dropped for lack of reserved capacity since
        the last call (clears the flag); synchronizes."""
        f = C.c_int32()
        self._check(self.lib.umgs_query(self.h, None, None, None, C.byref(f)))
        return bool(f.value)

    def blend_pairs(self) -> Dict[str, int]:
        """Work counters of the blend on the sorted frame: Gaussian and
        triangle (pixel, fragment) pairs evaluated, wave iterations of the
        fragment loop, fragments staged into LDS."""
        out = self.alloc_outputs(False)
        pairs = (C.c_int64 * 4)()
        with self._on_stream():
            self._check(self.lib.umgs_blend_pairs(self.h, _ptr(out["image"]), pairs))
        return dict(gauss=int(pairs[0]), tri=int(pairs[1]), wave_iters=int(pairs[2]),
                    staged=int(pairs[3]))

    def backward_pairs(self, n_contrib: torch.Tensor, triangles: bool = False) -> Dict[str, int]:
        """(pixel, fragment) pairs the backward walks on the sorted frame: every
        pixel the positions 1..n_contrib of its tile's list (n_contrib as
        written by the blend, views packed in order), split into Gaussian and
        triangle fragments.  triangles=True: the pairs of the triangle
        backward, whose walk ends at the tile's first triangle fragment and
        skips tiles that blend none."""
        ranges = self.copy_state(L.STATE_RANGES).long()
        vals = self.copy_state(L.STATE_SORTED_VALS).long() & 0xFFFFFFFF
        per_view = max(1, self.N + self.T)
        is_tri = (vals % per_view) >= self.N
        pref = torch.zeros(vals.numel() + 1, dtype=torch.int64, device=vals.device)
        pref[1:] = torch.cumsum(is_tri.long(), 0)
        tw, th = self.opts.tile_w, self.opts.tile_h
        nc_all = n_contrib.reshape(-1).long()
        g = t = 0
        pix0 = tile0 = 0
        for W, H in self.views:
            ntx, nty = (W + tw - 1) // tw, (H + th - 1) // th
            nc = nc_all[pix0:pix0 + W * H].view(H, W)
            ys = torch.arange(H, device=nc.device)[:, None]
            xs = torch.arange(W, device=nc.device)[None, :]
            tiles = tile0 + (ys // th) * ntx + (xs // tw)
            start = ranges[tiles, 0]
            lo = torch.zeros_like(nc)
            if triangles:
                n_t = ntx * nty
                flat = (tiles - tile0).reshape(-1)
                mx = torch.zeros(n_t, dtype=torch.int64, device=nc.device)
                mx = mx.scatter_reduce(0, flat, nc.reshape(-1), reduce="amax")
                s0 = ranges[tile0:tile0 + n_t, 0]
                tri_idx = torch.nonzero(is_tri).reshape(-1)
                big = torch.full_like(s0, 1 << 40)
                if tri_idx.numel():
                    k = torch.searchsorted(tri_idx, s0)
                    fpos = torch.where(k < tri_idx.numel(),
                                       tri_idx[k.clamp(max=tri_idx.numel() - 1)] - s0, big)
                else:
                    fpos = big
                active = fpos < mx                           # the tile walks at all
                lo = torch.where(active, fpos, 0)[flat].view(H, W)
                act = active[flat].view(H, W)
                lo = torch.where(act, lo, nc)                # inactive: no pairs
                nc = torch.maximum(nc, lo)
            nt = pref[start + nc] - pref[start + lo]
            t += int(nt.sum())
            g += int((nc - lo).sum()) - int(nt.sum())
            pix0 += W * H
            tile0 += ntx * nty
        return dict(gauss=g, tri=t)

    # ---- graphs ---------------------------------------------------------------
    def reserve(self, max_dup: int):
        self._check(self.lib.umgs_reserve(self.h, int(max_dup)))

    def capture(self, fn):
        """Record the library calls that ``fn()`` makes into a graph (after
        an eager frame of the same shape and a reserve()).  Output tensors
        that fn allocates must be kept alive by the caller: replays write
        into them."""
        if self.stream.cuda_stream == 0:
            raise ValueError("graph capture needs a Rasterizer with its own stream (own_stream=True)")
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        self._check(self.lib.umgs_graph_begin(self.h))
        self._capturing = True
        try:
            out = fn()
        except BaseException:
            self._capturing = False
            self.lib.umgs_graph_end(self.h)
            raise
        self._capturing = False
        self._check(self.lib.umgs_graph_end(self.h))
        return out

    def replay(self):
        with self._on_stream():
            self._check(self.lib.umgs_graph_launch(self.h))

    def update_views(self, old_cams, new_cams):
        """Replace a stored camera set (same sizes) for the next replays."""
        if len(old_cams) != len(new_cams):
            raise ValueError("old and new camera sets differ in length")
        a = (L.Camera * len(old_cams))(*[camera_struct(c) for c in old_cams])
        b = (L.Camera * len(new_cams))(*[camera_struct(c) for c in new_cams])
        with self._on_stream():
            self._check(self.lib.umgs_update_views(self.h, len(old_cams), a, b))

    def view_dups(self) -> List[int]:
        """Duplicates per view of the projected frame (before bin())."""
        arr = (C.c_int64 * len(self.views))()
        with self._on_stream():
            self._check(self.lib.umgs_view_dups(self.h, arr))
        return [int(x) for x in arr]

    def copy_state(self, which: int) -> torch.Tensor:
        n_dup, n_tiles, n_rec = self.query()
        d = self.device
        if which == L.STATE_KEYS:
            t = torch.empty(n_rec, dtype=torch.int32, device=d)
        elif which == L.STATE_SORTED_KEYS:
            t = torch.empty(n_dup, dtype=torch.int64, device=d)
        elif which == L.STATE_SORTED_VALS:
            t = torch.empty(n_dup, dtype=torch.int32, device=d)
        elif which == L.STATE_RANGES:
            t = torch.empty((n_tiles, 2), dtype=torch.int32, device=d)
        elif which == L.STATE_TRI_FIXED:
            t = torch.empty((len(self.views) * self.T, 6), dtype=torch.int32, device=d)
        elif which == L.STATE_GRAD2D:
            t = torch.empty((len(self.views) * self.N, 9), dtype=torch.float32, device=d)
        else:
            raise ValueError(which)
        with self._on_stream():
            self._check(self.lib.umgs_copy_state(self.h, which, _ptr(t), t.numel() * t.element_size()))
        torch.cuda.synchronize(d)
        return t


def scene_inputs(scene, cov3d=None, means=None) -> Dict:
    """Keyword arguments of Rasterizer.project for a generated scene."""
    kw = dict(means=scene.means if means is None else means, opacity=scene.opacity,
              sh=scene.sh.reshape(scene.N, -1), tri_xyz=scene.tri_xyz.reshape(scene.T, 9),
              tri_rgb=scene.tri_rgb.reshape(scene.T, 9), tri_alpha=scene.tri_alpha)
    if cov3d is not None:
        kw["cov3d"] = cov3d
    else:
        kw["scales"] = scene.scales
        kw["quats"] = scene.quats
    return kw


class _RenderFunction(torch.autograd.Function):
    """Differentiable render through the C ABI: Gaussians, the deformed
    proxy's vertices, and the triangles' per-vertex colours and opacities."""

    @staticmethod
    def forward(ctx, means, scales, quats, opacity, sh, V_def, tri_rgb, tri_alpha, rast, cams,
                tri_xyz, binding):
        with torch.no_grad():
            if binding is not None:
                dt = rast.bind_transfer(V_def, binding["bind_face"], binding["bind_bary"],
                                        means, quats, scales)
                pm, cov, xform = dt["means"], dt["cov3d"], dt["xform"]
            else:
                pm, cov, xform = means, None, None
            rast.project(cams, means=pm, cov3d=cov, scales=None if cov is not None else scales,
                         quats=None if cov is not None else quats, opacity=opacity,
                         sh=sh.reshape(sh.shape[0], -1), tri_xyz=tri_xyz, tri_rgb=tri_rgb,
                         tri_alpha=tri_alpha)
            rast.bin()
            rast.sort()
            out = rast.blend(want_state=True)
        ctx.rast = rast
        ctx.frame_id = rast.frame_id
        ctx.fwd = out
        empty = torch.empty(0, device=means.device)
        ctx.save_for_backward(pm.detach(), scales.detach(), quats.detach(), sh.detach(),
                              xform if xform is not None else empty)
        ctx.has_xform = xform is not None
        ctx.binding = binding
        ctx.V_def = V_def.detach() if isinstance(V_def, torch.Tensor) else V_def
        ctx.tri_shapes = (tuple(tri_rgb.shape) if isinstance(tri_rgb, torch.Tensor) else None,
                          tuple(tri_alpha.shape) if isinstance(tri_alpha, torch.Tensor) else None)
        ctx.sh_shape = sh.shape
        return out["image"]

    @staticmethod
    def backward(ctx, dL_dimage):
        rast = ctx.rast
        if rast.frame_id != ctx.frame_id:
            raise RuntimeError("the rasterizer has projected another frame since this forward; "
                               "run backward before the next forward on the same Rasterizer")
        pm, scales, quats, sh, xform = ctx.saved_tensors
        dL = dL_dimage.contiguous()
        g = rast.backward(dL, ctx.fwd, pm, scales, quats, sh.reshape(sh.shape[0], -1),
                          xform if ctx.has_xform else None)
        dV = d_rgb = d_alpha = None
        if ctx.has_xform and ctx.needs_input_grad[5]:
            dV = rast.backward_transfer(ctx.V_def, ctx.binding["bind_face"], ctx.binding["bind_bary"],
                                        g["means"], g["xform"]).reshape(ctx.V_def.shape)
        if ctx.needs_input_grad[6] or ctx.needs_input_grad[7]:
            tg = rast.backward_triangles(dL, ctx.fwd)
            if ctx.needs_input_grad[6]:
                d_rgb = tg["tri_rgb"].reshape(ctx.tri_shapes[0])
            if ctx.needs_input_grad[7]:
                d_alpha = tg["tri_alpha"].reshape(ctx.tri_shapes[1])
        return (g["means"], g["scales"], g["quats"], g["opacity"], g["sh"].reshape(ctx.sh_shape),
                dV, d_rgb, d_alpha, None, None, None, None)


def render_differentiable(rast: Rasterizer, cams, means, scales, quats, opacity, sh, tri_xyz=None,
                          tri_rgb=None, tri_alpha=None, deform: Optional[Dict] = None) -> torch.Tensor:
    """Packed image (3,H,W per view) as a differentiable function of the
    Gaussians' means, linear scales, raw quaternions, opacities and SH
    coefficients, and of the triangles' per-vertex colours and opacities
    when those are tensors that require gradients.  ``deform`` =
    dict(V_def, bind_face, bind_bary) moves the Gaussians with the proxy set
    by ``rast.set_proxy`` first (gradients are then with respect to the rest
    parameters, and to V_def when it requires them).  The backward must run
    before the next forward on the same Rasterizer."""
    V_def, binding = None, None
    if deform is not None:
        V_def = deform["V_def"]
        binding = dict(bind_face=deform["bind_face"], bind_bary=deform["bind_bary"])
    return _RenderFunction.apply(means, scales, quats, opacity, sh, V_def, tri_rgb, tri_alpha, rast,
                                 list(cams), tri_xyz, binding)
