"""Python binding of the C ABI (argument marshalling only).

Every step of the path runs in the HIP kernels of libunimgs.so; PyTorch only
provides device memory and the stream.  Names follow the C entry points.
"""
from __future__ import annotations

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


def make_options(tile=(16, 16), frag_batch=128, sh_degree=0, k_bind=8, mode=0,
                 bg=(0.0, 0.0, 0.0)) -> L.Options:
    o = L.Options()
    o.tile_w, o.tile_h = int(tile[0]), int(tile[1])
    o.frag_batch = int(frag_batch)
    o.sh_degree = int(sh_degree)
    o.k_bind = int(k_bind)
    o.mode = int(mode)
    for k in range(3):
        o.bg[k] = float(bg[k])
    return o


class Rasterizer:
    """One library context bound to a torch stream on one device."""

    def __init__(self, device="cuda:0", stream: Optional[torch.cuda.Stream] = None, **opts):
        self.lib = L.load()
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
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

    def bind_transfer(self, V_def, bind_face, bind_bary, means, quats, scales,
                      with_vertex: bool = False) -> Dict[str, torch.Tensor]:
        d = self.device
        V_def, means, quats, scales = (_f32(x, d) for x in (V_def, means, quats, scales))
        if isinstance(bind_face, np.ndarray) and bind_face.size and (
                bind_face.min() < 0 or bind_face.max() >= self.nF):
            raise ValueError("bind_face holds a face index outside the proxy")
        bind_face = _i32(bind_face, d)
        bind_bary = _f32(bind_bary, d)
        N = means.shape[0]
        K = self.opts.k_bind
        if bind_face.numel() != N * K or bind_bary.numel() != 2 * N * K:
            raise ValueError(f"bindings must be (N, {K}) faces and (N, {K}, 2) barycentrics")
        out = dict(means=torch.empty((N, 3), device=d), quats=torch.empty((N, 4), device=d),
                   cov3d=torch.empty((N, 6), device=d), xform=torch.empty((N, 9), device=d))
        vert = torch.empty((self.nV, 12), device=d) if with_vertex else None
        with torch.cuda.stream(self.stream):
            self._check(self.lib.umgs_bind_transfer(
                self.h, _ptr(V_def), N, _ptr(bind_face), _ptr(bind_bary), _ptr(means), _ptr(quats),
                _ptr(scales), _ptr(out["means"]), _ptr(out["quats"]), _ptr(out["cov3d"]),
                _ptr(out["xform"]), _ptr(vert)))
        if vert is not None:
            out["vertex"] = vert
        return out

    # ---- forward ------------------------------------------------------------
    def project(self, cams: Sequence, means=None, opacity=None, sh=None, scales=None, quats=None,
                cov3d=None, tri_xyz=None, tri_rgb=None, tri_alpha=None):
        d = self.device
        means, opacity, sh, scales, quats, cov3d = (_f32(x, d) for x in (means, opacity, sh, scales, quats, cov3d))
        tri_xyz, tri_rgb, tri_alpha = (_f32(x, d) for x in (tri_xyz, tri_rgb, tri_alpha))
        N = 0 if means is None else means.shape[0]
        T = 0 if tri_xyz is None else tri_xyz.shape[0]
        nc = 3 * (self.opts.sh_degree + 1) ** 2
        if N and (sh is None or sh.numel() != N * nc):
            raise ValueError(f"sh must hold {nc} floats per Gaussian for sh_degree {self.opts.sh_degree}")
        for name, t, w in (("means", means, 3), ("opacity", opacity, 1), ("scales", scales, 3),
                           ("quats", quats, 4), ("cov3d", cov3d, 6)):
            if N and t is not None and t.numel() != N * w:
                raise ValueError(f"{name} must hold {w} floats per Gaussian")
        for name, t, w in (("tri_rgb", tri_rgb, 9), ("tri_alpha", tri_alpha, 1)):
            if T and (t is None or t.numel() != T * w):
                raise ValueError(f"{name} must hold {w} floats per triangle")
        if T and tri_xyz.numel() != T * 9:
            raise ValueError("tri_xyz must hold 9 floats per triangle")
        arr = (L.Camera * len(cams))(*[camera_struct(c) for c in cams])
        self._keep = [means, opacity, sh, scales, quats, cov3d, tri_xyz, tri_rgb, tri_alpha]
        self._check(self.lib.umgs_project(self.h, len(cams), arr, N, _ptr(means), _ptr(cov3d), _ptr(scales),
                                          _ptr(quats), _ptr(opacity), _ptr(sh), T, _ptr(tri_xyz),
                                          _ptr(tri_rgb), _ptr(tri_alpha)))
        self.views = [(int(c.width), int(c.height)) for c in cams]
        self.N, self.T = N, T

    def bin(self):
        self._check(self.lib.umgs_bin(self.h))

    def sort(self):
        self._check(self.lib.umgs_sort(self.h))

    def blend(self, want_state: bool = True) -> Dict[str, torch.Tensor]:
        d = self.device
        npix = sum(w * h for w, h in self.views)
        image = torch.empty(3 * npix, device=d)
        Tf = torch.empty(npix, device=d) if want_state else None
        nc = torch.empty(npix, device=d, dtype=torch.int32) if want_state else None
        Te = torch.empty(npix, device=d) if want_state else None
        self._check(self.lib.umgs_blend(self.h, _ptr(image), _ptr(Tf), _ptr(nc), _ptr(Te)))
        return dict(image=image, T_final=Tf, n_contrib=nc, T_entity_in=Te)

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
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self.lib.umgs_query(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

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
        else:
            raise ValueError(which)
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
