"""Seeded synthetic inputs for the mixed Gaussian/triangle rasterizer.

This module only *draws* inputs: Gaussian parameters, triangle meshes, proxy
meshes and their deformations, cameras, and the host-side association of each
Gaussian (or each corner of its bounding box) with the nearest proxy face.
It contains none of the rendering or deformation-transfer arithmetic, so both
the GPU path and the CPU oracle can consume what it returns without sharing
any of the method's code.

Workloads (all FP32 arrays, seeded by ``numpy.random.default_rng``):

0. 64x64, 1 view: 2,000 Gaussians uniform in [-1,1]^3, an opaque icosphere
   (frequency 4, 320 faces, radius 0.3) and a 2-triangle quad at z=0.2 with
   alpha 0.5; camera at distance 3, vertical FOV 60 degrees.
1. 1920x1080, 1 view: 1M Gaussians within 0.02 of a 20,480-face proxy sphere,
   bound to their nearest faces (8 bounding-box corners), proxy bent by
   0.2*sin(2*pi*x); 100,128 occluder triangles (8 opaque icospheres of
   frequency 16 plus 4 semi-transparent 86x86 planes).
2. 800x800, 1 view: 300k Gaussians with SH degree 3, 50,176 triangles.
3. 64 orbit views of uneven size (256^2 .. 1920x1080), 500k Gaussians and
   30,084 triangles.
4. 16 orbit views at 1920x1080: 2M Gaussians (SH degree 3) bound to a 50k-face
   proxy deformed by three Gaussian bumps, 200k occluder triangles.

``make_config(i, scale=...)`` can shrink the primitive counts and resolution of
a workload while keeping its structure (used for parity tests that the CPU
oracle must finish in seconds).
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import List, Optional

import numpy as np

# sqrt(4*pi): a degree-0 SH coefficient of (rgb - 0.5) * sqrt(4*pi) makes the
# view-independent colour equal to rgb (input distribution parameter only).
_DC_SCALE = math.sqrt(4.0 * math.pi)


@dataclasses.dataclass
class Camera:
    """Pinhole camera, world->camera rotation R (3x3) and translation t.

    OpenCV axes: x right, y down, z forward.  Pixel (i, j) covers
    [i, i+1) x [j, j+1); its centre is (i + 0.5, j + 0.5).
    """
    R: np.ndarray            # (3,3) float32
    t: np.ndarray            # (3,) float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def center(self) -> np.ndarray:
        return -(self.R.astype(np.float64).T @ self.t.astype(np.float64))


@dataclasses.dataclass
class Proxy:
    """Proxy mesh: rest vertices, faces and a deformed copy of the vertices."""
    V_rest: np.ndarray        # (nV,3) float32
    faces: np.ndarray         # (nF,3) int32, outward orientation
    V_def: np.ndarray         # (nV,3) float32


@dataclasses.dataclass
class Scene:
    name: str
    means: np.ndarray          # (N,3) float32
    scales: np.ndarray         # (N,3) float32, linear (exp of log-scales)
    quats: np.ndarray          # (N,4) float32, (w,x,y,z), unit length
    opacity: np.ndarray        # (N,) float32 in (0,1)
    sh: np.ndarray             # (N, (deg+1)^2, 3) float32
    sh_degree: int
    tri_xyz: np.ndarray        # (T,3,3) float32 world-space vertices
    tri_rgb: np.ndarray        # (T,3,3) float32 per-vertex colour
    tri_alpha: np.ndarray      # (T,) float32
    cams: List[Camera]
    proxy: Optional[Proxy] = None
    bind_face: Optional[np.ndarray] = None   # (N,K) int32
    bind_bary: Optional[np.ndarray] = None   # (N,K,2) float32 (u,v); w = 1-u-v
    bg: tuple = (0.0, 0.0, 0.0)

    @property
    def N(self) -> int:
        return int(self.means.shape[0])

    @property
    def T(self) -> int:
        return int(self.tri_xyz.shape[0])


# ----------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------

def look_at(eye, width: int, height: int, target=(0.0, 0.0, 0.0),
            fov_y_deg: float = 60.0) -> Camera:
    """Camera at ``eye`` looking at ``target`` with world up +y."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    up = np.array([0.0, 1.0, 0.0])
    if abs(f @ up) > 0.999:
        up = np.array([0.0, 0.0, 1.0])
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f]).astype(np.float32)
    t = (-(R.astype(np.float64) @ eye)).astype(np.float32)
    foc = height / (2.0 * math.tan(math.radians(fov_y_deg) / 2.0))
    return Camera(R=R, t=t, fx=float(np.float32(foc)), fy=float(np.float32(foc)),
                  cx=width / 2.0, cy=height / 2.0, width=int(width), height=int(height))


def orbit_cameras(rng, n: int, sizes, dist_range=(2.5, 4.0)) -> List[Camera]:
    cams = []
    for i in range(n):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        dist = rng.uniform(*dist_range)
        w, h = sizes[i]
        cams.append(look_at(d * dist, w, h))
    return cams


def uneven_sizes(rng, n: int, lo=(256, 256), hi=(1920, 1080)):
    """log-area uniform between lo and hi, aspect U[1, 16/9]."""
    a0, a1 = math.log(lo[0] * lo[1]), math.log(hi[0] * hi[1])
    out = []
    for _ in range(n):
        area = math.exp(rng.uniform(a0, a1))
        aspect = rng.uniform(1.0, 16.0 / 9.0)
        w = int(round(math.sqrt(area * aspect)))
        h = int(round(area / w))
        out.append((max(w, 1), max(h, 1)))
    return out


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------

def _icosahedron():
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
                  [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
                  [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], np.float64)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


def icosphere(freq: int, radius: float = 1.0, center=(0.0, 0.0, 0.0)):
    """Geodesic sphere of frequency ``freq``: 20*freq^2 faces, 10*freq^2+2 vertices.

    Each icosahedron face is split into a barycentric grid of freq^2
    triangles; shared edge vertices are merged by their exact integer grid
    label, then every vertex is pushed to the sphere.
    """
    V0, F0 = _icosahedron()
    n = freq
    key_to_idx = {}
    verts = []

    def vid(a, b, c, i, j, k):
        # point = (i*Va + j*Vb + k*Vc)/n with i+j+k = n; label it by the
        # sorted (vertex, weight) pairs with non-zero weight.
        lab = tuple(sorted((vv, ww) for vv, ww in ((a, i), (b, j), (c, k)) if ww))
        idx = key_to_idx.get(lab)
        if idx is None:
            idx = len(verts)
            key_to_idx[lab] = idx
            verts.append((i * V0[a] + j * V0[b] + k * V0[c]) / n)
        return idx

    faces = []
    for a, b, c in F0:
        grid = {}
        for i in range(n + 1):
            for j in range(n + 1 - i):
                grid[(i, j)] = vid(a, b, c, n - i - j, i, j)
        for i in range(n):
            for j in range(n - i):
                p0, p1, p2 = grid[(i, j)], grid[(i + 1, j)], grid[(i, j + 1)]
                faces.append((p0, p1, p2))
                if j < n - i - 1:
                    q0, q1, q2 = grid[(i + 1, j)], grid[(i + 1, j + 1)], grid[(i, j + 1)]
                    faces.append((q0, q1, q2))
    V = np.array(verts, np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    V = V * radius + np.asarray(center, np.float64)
    F = np.array(faces, np.int64)
    # outward orientation
    c = V[F].mean(axis=1) - np.asarray(center, np.float64)
    nrm = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    flip = (nrm * c).sum(axis=1) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def grid_plane(n: int, side: float, center, normal):
    """n x n grid of squares (2 n^2 triangles) of the given side length."""
    normal = np.asarray(normal, np.float64)
    normal /= np.linalg.norm(normal)
    a = np.cross(normal, [1.0, 0.0, 0.0])
    if np.linalg.norm(a) < 1e-3:
        a = np.cross(normal, [0.0, 1.0, 0.0])
    a /= np.linalg.norm(a)
    b = np.cross(normal, a)
    s = np.linspace(-side / 2, side / 2, n + 1)
    uu, vv = np.meshgrid(s, s, indexing="ij")
    V = (np.asarray(center, np.float64)[None, :]
         + uu.reshape(-1, 1) * a[None, :] + vv.reshape(-1, 1) * b[None, :])
    idx = np.arange((n + 1) * (n + 1)).reshape(n + 1, n + 1)
    q0, q1 = idx[:-1, :-1].ravel(), idx[1:, :-1].ravel()
    q2, q3 = idx[1:, 1:].ravel(), idx[:-1, 1:].ravel()
    F = np.concatenate([np.stack([q0, q1, q2], 1), np.stack([q0, q2, q3], 1)])
    return V, F


def _tri_soup(V, F):
    return V[F].astype(np.float32)


# ----------------------------------------------------------------------------
# Gaussians
# ----------------------------------------------------------------------------

def _gaussian_stats(rng, n, sh_degree):
    log_s = rng.normal(-3.0, 0.5, size=(n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    o = 1.0 / (1.0 + np.exp(-rng.normal(size=n)))
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    nc = (sh_degree + 1) ** 2
    sh = np.zeros((n, nc, 3))
    sh[:, 0, :] = (rgb - 0.5) * _DC_SCALE
    if nc > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.1, size=(n, nc - 1, 3))
    return (np.exp(log_s).astype(np.float32), q.astype(np.float32),
            o.astype(np.float32), sh.astype(np.float32))


def _sample_on_mesh(rng, V, F, n, offset):
    """Points with face chosen by area, uniform barycentric, normal offset."""
    e1 = V[F[:, 1]] - V[F[:, 0]]
    e2 = V[F[:, 2]] - V[F[:, 0]]
    cr = np.cross(e1, e2)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    nrm = cr / (2.0 * area[:, None])
    f = rng.choice(F.shape[0], size=n, p=area / area.sum())
    r1, r2 = rng.uniform(size=n), rng.uniform(size=n)
    s = np.sqrt(r1)
    b0, b1, b2 = 1 - s, s * (1 - r2), s * r2
    P = (b0[:, None] * V[F[f, 0]] + b1[:, None] * V[F[f, 1]] + b2[:, None] * V[F[f, 2]])
    P += nrm[f] * rng.uniform(-offset, offset, size=n)[:, None]
    return P


# ----------------------------------------------------------------------------
# host-side binding association (setup step, not per frame)
# ----------------------------------------------------------------------------

def _closest_on_triangles(P, A, B, C):
    """Closest point on triangles (A,B,C) to P, vectorised: the projection onto
    the plane when it falls inside the triangle, else the nearest point on the
    three edges.  Returns barycentrics (u, v, w) w.r.t. (A, B, C) and the
    squared distance."""
    ab, ac, ap = B - A, C - A, P - A
    d00 = (ab * ab).sum(-1)
    d01 = (ab * ac).sum(-1)
    d11 = (ac * ac).sum(-1)
    d20 = (ap * ab).sum(-1)
    d21 = (ap * ac).sum(-1)
    den = d00 * d11 - d01 * d01
    with np.errstate(divide="ignore", invalid="ignore"):
        bv = (d11 * d20 - d01 * d21) / den
        bw = (d00 * d21 - d01 * d20) / den
    bu = 1.0 - bv - bw
    inside = (bu >= 0) & (bv >= 0) & (bw >= 0)

    def seg(X, Y):
        xy = Y - X
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.clip(((P - X) * xy).sum(-1) / (xy * xy).sum(-1), 0.0, 1.0)
        t = np.nan_to_num(t)
        Q = X + t[..., None] * xy
        return t, ((P - Q) ** 2).sum(-1)

    t_ab, e_ab = seg(A, B)
    t_bc, e_bc = seg(B, C)
    t_ca, e_ca = seg(C, A)
    best = np.argmin(np.stack([e_ab, e_bc, e_ca], -1), axis=-1)
    z = np.zeros_like(t_ab)
    eu = np.choose(best, [1 - t_ab, z, t_ca])
    ev = np.choose(best, [t_ab, 1 - t_bc, z])
    ew = np.choose(best, [z, t_bc, 1 - t_ca])
    u = np.where(inside, bu, eu)
    v = np.where(inside, bv, ev)
    w = np.where(inside, bw, ew)
    Q = u[..., None] * A + v[..., None] * B + w[..., None] * C
    return u, v, w, ((P - Q) ** 2).sum(-1)


def bind_nearest(points, V, F, candidates: int = 8, chunk: int = 1 << 15):
    """Associate each point with the nearest proxy face (among the faces whose
    centroids are the ``candidates`` nearest), returning (face, u, v) with
    the closest point = u*V[f0] + v*V[f1] + (1-u-v)*V[f2].  Chunks run on a
    thread pool (NumPy releases the GIL in its array operations)."""
    from concurrent.futures import ThreadPoolExecutor
    from scipy.spatial import cKDTree
    cen = V[F].mean(axis=1)
    tree = cKDTree(cen)
    n = points.shape[0]
    face = np.empty(n, np.int32)
    bu = np.empty(n, np.float32)
    bv = np.empty(n, np.float32)

    def work(s):
        P = points[s:s + chunk]
        _, cand = tree.query(P, k=candidates)
        A, B, C = V[F[cand, 0]], V[F[cand, 1]], V[F[cand, 2]]
        u, v, w, d2 = _closest_on_triangles(P[:, None, :], A, B, C)
        best = np.argmin(d2, axis=1)
        r = np.arange(P.shape[0])
        face[s:s + chunk] = cand[r, best]
        bu[s:s + chunk] = u[r, best]
        bv[s:s + chunk] = v[r, best]

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(work, range(0, n, chunk)))
    return face, bu, bv


def bbox_corners(means, scales, quats):
    """Corners mu + R(q) diag(3 s) (+-1,+-1,+-1) in a fixed order (x fastest)."""
    w, x, y, z = [quats[:, i].astype(np.float64) for i in range(4)]
    R = np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)
    signs = np.array([[sx, sy, sz] for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)],
                     np.float64)
    loc = signs[None, :, :] * (3.0 * scales.astype(np.float64))[:, None, :]
    return means.astype(np.float64)[:, None, :] + np.einsum("nij,nkj->nki", R, loc)


def make_binding(means, scales, quats, V, F, K: int):
    if K == 1:
        pts = means.astype(np.float64)
    else:
        pts = bbox_corners(means, scales, quats).reshape(-1, 3)
    f, u, v = bind_nearest(pts, V, F)
    N = means.shape[0]
    return f.reshape(N, K), np.stack([u, v], -1).reshape(N, K, 2).astype(np.float32)


# ----------------------------------------------------------------------------
# deformations of the proxy (analytic; stand-ins for an editing tool)
# ----------------------------------------------------------------------------

def bend(V, amplitude=0.2, wavelength=1.0):
    D = V.copy()
    D[:, 1] += amplitude * np.sin(2 * math.pi * V[:, 0] / wavelength)
    return D


def rbf_bumps(rng, V, n=3):
    D = V.copy()
    for _ in range(n):
        c = V[rng.integers(V.shape[0])]
        r = rng.uniform(0.3, 0.6)
        a = rng.normal(size=3)
        a = a / np.linalg.norm(a) * rng.uniform(0.1, 0.25)
        D += np.exp(-((V - c) ** 2).sum(1) / (2 * r * r))[:, None] * a[None, :]
    return D


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def _assemble_tris(parts):
    xyz = np.concatenate([p[0] for p in parts]) if parts else np.zeros((0, 3, 3), np.float32)
    rgb = np.concatenate([p[1] for p in parts]) if parts else np.zeros((0, 3, 3), np.float32)
    al = np.concatenate([p[2] for p in parts]) if parts else np.zeros((0,), np.float32)
    return xyz.astype(np.float32), rgb.astype(np.float32), al.astype(np.float32)


def _mesh_part(rng, V, F, alpha):
    xyz = _tri_soup(V, F)
    rgb = rng.uniform(0.0, 1.0, size=(V.shape[0], 3))[F].astype(np.float32)
    al = np.broadcast_to(np.asarray(alpha, np.float32), (F.shape[0],)).astype(np.float32)
    return xyz, rgb, al


def _random_spheres(rng, count, freq, r_range, c_range=1.5, alpha_fn=None):
    parts = []
    for _ in range(count):
        r = rng.uniform(*r_range)
        c = rng.uniform(-c_range, c_range, size=3)
        V, F = icosphere(freq, r, c)
        alpha = 1.0 if alpha_fn is None else alpha_fn(F.shape[0])
        parts.append(_mesh_part(rng, V, F, alpha))
    return parts


def _random_planes(rng, count, n, side=2.0):
    parts = []
    for _ in range(count):
        nrm = rng.normal(size=3)
        c = rng.uniform(-1.0, 1.0, size=3)
        V, F = grid_plane(n, side, c, nrm)
        parts.append(_mesh_part(rng, V, F, rng.uniform(0.3, 0.7)))
    return parts


def _scaled(n, scale, lo=1):
    return max(lo, int(round(n * scale)))


def make_config(index: int, seed: Optional[int] = None, scale: float = 1.0,
                res_scale: float = 1.0, n_views: Optional[int] = None,
                K: Optional[int] = None) -> Scene:
    """Build workload ``index`` (0..4).

    ``scale`` multiplies the Gaussian count and the mesh subdivision density
    (triangle counts scale with it); ``res_scale`` multiplies image width and
    height; ``n_views`` overrides the number of views of workloads 3 and 4.
    The full-size workloads are ``scale = res_scale = 1``.  If the
    environment variable UMGS_SCENE_CACHE names a directory, generated scenes
    are stored there (pickle-free .npz) and reused.
    """
    cache = os.environ.get("UMGS_SCENE_CACHE")
    if cache:
        key = f"cfg{index}_s{seed}_x{scale}_r{res_scale}_v{n_views}_k{K}.npz"
        path = os.path.join(cache, key)
        if os.path.exists(path):
            return _load_scene(path)
        sc = _make_config(index, seed, scale, res_scale, n_views, K)
        os.makedirs(cache, exist_ok=True)
        _save_scene(sc, path)
        return sc
    return _make_config(index, seed, scale, res_scale, n_views, K)


_CAM_FIELDS = ("fx", "fy", "cx", "cy", "width", "height")


def _save_scene(sc: Scene, path: str):
    d = dict(name=np.array(sc.name), means=sc.means, scales=sc.scales, quats=sc.quats,
             opacity=sc.opacity, sh=sc.sh, sh_degree=np.array(sc.sh_degree), tri_xyz=sc.tri_xyz,
             tri_rgb=sc.tri_rgb, tri_alpha=sc.tri_alpha, bg=np.array(sc.bg, np.float64),
             cam_R=np.stack([c.R for c in sc.cams]), cam_t=np.stack([c.t for c in sc.cams]),
             cam_k=np.array([[getattr(c, f) for f in _CAM_FIELDS] for c in sc.cams], np.float64))
    if sc.proxy is not None:
        d.update(V_rest=sc.proxy.V_rest, faces=sc.proxy.faces, V_def=sc.proxy.V_def,
                 bind_face=sc.bind_face, bind_bary=sc.bind_bary)
    tmp = path + ".tmp.npz"
    np.savez(tmp, **d)
    os.replace(tmp, path)


def _load_scene(path: str) -> Scene:
    z = np.load(path)          # allow_pickle stays False
    cams = [Camera(R=z["cam_R"][i], t=z["cam_t"][i], fx=float(k[0]), fy=float(k[1]), cx=float(k[2]),
                   cy=float(k[3]), width=int(k[4]), height=int(k[5]))
            for i, k in enumerate(z["cam_k"])]
    proxy = None
    bf = bb = None
    if "V_rest" in z:
        proxy = Proxy(z["V_rest"], z["faces"], z["V_def"])
        bf, bb = z["bind_face"], z["bind_bary"]
    return Scene(str(z["name"]), z["means"], z["scales"], z["quats"], z["opacity"], z["sh"],
                 int(z["sh_degree"]), z["tri_xyz"], z["tri_rgb"], z["tri_alpha"], cams, proxy=proxy,
                 bind_face=bf, bind_bary=bb, bg=tuple(z["bg"].tolist()))


def _make_config(index, seed, scale, res_scale, n_views, K) -> Scene:
    seed = index if seed is None else seed
    rng = np.random.default_rng(seed)

    def res(w, h):
        return max(1, int(round(w * res_scale))), max(1, int(round(h * res_scale)))

    def freq(f):
        return max(1, int(round(f * math.sqrt(scale))))

    if index == 0:
        n = _scaled(2000, scale)
        means = rng.uniform(-1, 1, size=(n, 3)).astype(np.float32)
        s, q, o, sh = _gaussian_stats(rng, n, 0)
        V, F = icosphere(4, 0.3)
        parts = [_mesh_part(rng, V, F, 1.0)]
        qv = np.array([[-0.5, -0.5, 0.2], [0.5, -0.5, 0.2], [0.5, 0.5, 0.2], [-0.5, 0.5, 0.2]])
        qf = np.array([[0, 1, 2], [0, 2, 3]])
        parts.append(_mesh_part(rng, qv, qf, 0.5))
        xyz, rgb, al = _assemble_tris(parts)
        W, H = res(64, 64)
        return Scene("quad_sphere_2k_64px", means, s, q, o, sh, 0, xyz, rgb, al,
                     [look_at((0, 0, 3), W, H)])

    if index == 1 or index == 4:
        big = index == 4
        pf = freq(50 if big else 32)
        Vp, Fp = icosphere(pf, 1.0)
        n = _scaled(2_000_000 if big else 1_000_000, scale)
        means = _sample_on_mesh(rng, Vp, Fp, n, 0.02).astype(np.float32)
        s, q, o, sh = _gaussian_stats(rng, n, 3 if big else 0)
        Vd = rbf_bumps(rng, Vp) if big else bend(Vp)
        k = K if K is not None else 8
        bf, bb = make_binding(means, s, q, Vp, Fp, k)
        if big:
            def alpha_fn(nf):
                a = np.ones(nf)
                m = rng.uniform(size=nf) < 0.2
                a[m] = rng.uniform(0.2, 0.8, size=int(m.sum()))
                return a
            parts = _random_spheres(rng, 16, freq(25), (0.1, 0.3), alpha_fn=alpha_fn)
        else:
            parts = _random_spheres(rng, 8, freq(16), (0.15, 0.35))
            parts += _random_planes(rng, 4, freq(86))
        xyz, rgb, al = _assemble_tris(parts)
        proxy = Proxy(Vp.astype(np.float32), Fp.astype(np.int32), Vd.astype(np.float32))
        if big:
            nv = 16 if n_views is None else n_views
            cams = orbit_cameras(rng, nv, [res(1920, 1080)] * nv)
            name = "deformed_2m_sh3_16x1080p"
        else:
            W, H = res(1920, 1080)
            cams = [look_at((0, 0, 3), W, H)]
            name = "deformed_1m_100k_tris_1080p"
        return Scene(name, means, s, q, o, sh, 3 if big else 0, xyz, rgb, al, cams,
                     proxy=proxy, bind_face=bf, bind_bary=bb)

    if index == 2:
        n = _scaled(300_000, scale)
        means = rng.uniform(-1, 1, size=(n, 3)).astype(np.float32)
        s, q, o, sh = _gaussian_stats(rng, n, 3)
        parts = _random_spheres(rng, 8, freq(16), (0.15, 0.35))
        parts += _random_planes(rng, 2, freq(48))
        xyz, rgb, al = _assemble_tris(parts)
        W, H = res(800, 800)
        return Scene("sh3_300k_800px", means, s, q, o, sh, 3, xyz, rgb, al,
                     [look_at((0, 0, 3), W, H)])

    if index == 3:
        n = _scaled(500_000, scale)
        means = rng.uniform(-1, 1, size=(n, 3)).astype(np.float32)
        s, q, o, sh = _gaussian_stats(rng, n, 0)
        parts = _random_spheres(rng, 4, freq(16), (0.15, 0.35))
        parts += _random_planes(rng, 2, freq(49))
        xyz, rgb, al = _assemble_tris(parts)
        nv = 64 if n_views is None else n_views
        lo = res(256, 256)
        hi = res(1920, 1080)
        cams = orbit_cameras(rng, nv, uneven_sizes(rng, nv, lo, hi))
        return Scene("uneven_64_views_500k", means, s, q, o, sh, 0, xyz, rgb, al, cams)

    raise ValueError(f"unknown workload {index}")


def perturbed(scene: Scene, seed: int, sigma: float = 0.01) -> Scene:
    """Copy of ``scene`` whose raw Gaussian parameters (mean, log-scale,
    quaternion, logit-opacity, SH) are perturbed by N(0, sigma)."""
    rng = np.random.default_rng(seed)
    n = scene.N
    means = scene.means + rng.normal(0, sigma, size=(n, 3)).astype(np.float32)
    scales = np.exp(np.log(scene.scales.astype(np.float64))
                    + rng.normal(0, sigma, size=(n, 3))).astype(np.float32)
    q = scene.quats.astype(np.float64) + rng.normal(0, sigma, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    o = scene.opacity.astype(np.float64)
    lo = np.log(o / (1 - o)) + rng.normal(0, sigma, size=n)
    sh = scene.sh + rng.normal(0, sigma, size=scene.sh.shape).astype(np.float32)
    return dataclasses.replace(scene, means=means, scales=scales,
                               quats=q.astype(np.float32),
                               opacity=(1 / (1 + np.exp(-lo))).astype(np.float32),
                               sh=sh.astype(np.float32))
