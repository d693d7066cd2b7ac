"""Forward oracle of the single-pass mixed rasterizer (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
use this module.  It is written from the paper's Section 3.2 (Eq. 1-11) and
the 3DGS projection conventions it extends; it shares no code with the GPU
library.  Everything continuous is evaluated in FP64.  The few values that
*decide* something discrete -- the view depth that culls and orders a
primitive, the snapped triangle vertices that decide sample coverage -- are
evaluated in FP32 with one rounding per operation in a fixed order, so that
the GPU path, which computes the same decision values in FP32, can be
compared bit for bit.

Per pixel, the oracle gathers *every* primitive that contributes to it (no
tiles), sorts them by (depth key, global id) and blends front to back:

* Gaussian fragment (Eq. 1-2): alpha = min(0.99, o exp(power)); it
  contributes iff alpha >= 1/255.  If T (1 - alpha) < 1e-4 the pixel stops
  before blending it; otherwise C += T alpha c, T *= 1 - alpha.  A Gaussian
  closes any open triangle entity.
* Triangle fragment (Eq. 7-9): contributes iff it covers at least one of the
  M = 4 sub-samples.  Consecutive triangle fragments (no contributing
  Gaussian between them) form one entity: at its first triangle
  T_in = T and t^j = 1; each triangle adds T_in O alpha c with
  O = (1/M) sum_j o^j t^j (Eq. 8) and updates t^j *= 1 - o^j alpha (Eq. 7).
  Pixel transmittance after each triangle is T = T_in (1/M) sum_j t^j
  (reading of "still updated" for later blending); the pixel stops after
  blending a triangle that leaves T < 1e-4.
* Background (Eq. 10-11 with an opaque background): C += T C_bg.

A triangle's colour and opacity are evaluated at the pixel centre: the
per-vertex colour interpolated perspective-correctly, and the triangle's
opacity attribute.  A textured mesh (the paper's Section 1 assigns an
opacity attribute to textured meshes) also interpolates per-vertex texture
coordinates with the same weights and samples an RGBA texture bilinearly:
colour = vertex colour x texel RGB, opacity = attribute x texel alpha (the
texel alpha is the per-texel opacity).  Sub-sample coverage is unaffected.

Besides C and T the oracle reports, per pixel, the transmittance in front of
the last blended unit (a Gaussian, or a whole triangle entity), which the
backward pass needs when that unit is opaque.

Global ids: Gaussians 0..N-1, triangles N..N+T-1.  Equal depth keys are
ordered by ascending id.

Global constants follow 3DGS: EWA low-pass dilation 0.3 px^2, alpha clamp
0.99, contribution threshold 1/255, stop threshold 1e-4, near plane 0.2,
frustum clamp 1.3 x tan(fov/2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import sh as _sh

F32 = np.float32

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_STOP = 1e-4
NEAR = 0.2
DILATION = 0.3
FRUSTUM_CLAMP = 1.3
M_SAMPLES = 4
SUBPX = 256                       # fixed-point sub-pixel resolution (1/256 px)
COORD_LIMIT = 1 << 24             # |snapped coordinate| bound, in 1/256 px
# 4x rotated-grid sample offsets from the pixel centre, in 1/256 px
SAMPLE_OFFSETS = ((-32, -96), (96, -32), (-96, 32), (32, 96))

MODE_UNIMGS = 0        # depth-adjacent triangles form one entity (Fig. 3d)
MODE_DIRECT = 1        # triangles blended like Gaussians, centre coverage (Fig. 3a)
MODE_ONE_ENTITY = 2    # all triangles of a pixel form one entity (Fig. 3b/c)
MODE_LITERAL_T = 3     # entity with pixel T updated by Eq. 6 with Eq. 8's O


# ---------------------------------------------------------------------------
# pinned FP32 decision values
# ---------------------------------------------------------------------------

def _cam32(cam):
    R = np.asarray(cam.R, F32)
    t = np.asarray(cam.t, F32)
    return R, t, F32(cam.fx), F32(cam.fy), F32(cam.cx), F32(cam.cy)


def view_row_f32(R, t, P, row):
    """((R[r,0] x + R[r,1] y) + R[r,2] z) + t[r] in float32, one rounding per op."""
    P = np.asarray(P, F32)
    a = R[row, 0] * P[:, 0]
    b = R[row, 1] * P[:, 1]
    c = R[row, 2] * P[:, 2]
    return ((a + b) + c) + t[row]


def pixel_f32(f, c, xv, zv):
    """u = (f x) / z + c in float32 (correctly rounded division)."""
    return (f * xv) / zv + c


# ---------------------------------------------------------------------------
# Gaussians: EWA projection (3DGS conventions)
# ---------------------------------------------------------------------------

def quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrices of (w,x,y,z) quaternions, normalised first."""
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def cov3d_from_scale_rot(scales, quats):
    Rq = quat_to_rot(np.asarray(quats, np.float64))
    S2 = np.asarray(scales, np.float64) ** 2
    return np.einsum("nij,nj,nkj->nik", Rq, S2, Rq)


def cov3d_from_packed(c6):
    c = np.asarray(c6, np.float64)
    return np.stack([np.stack([c[:, 0], c[:, 1], c[:, 2]], -1),
                     np.stack([c[:, 1], c[:, 3], c[:, 4]], -1),
                     np.stack([c[:, 2], c[:, 4], c[:, 5]], -1)], -2)


@dataclass
class GaussProj:
    valid: np.ndarray        # (N,) bool
    key: np.ndarray          # (N,) float32 depth key (pinned)
    mean2d: np.ndarray       # (N,2) fp64
    cov2d: np.ndarray        # (N,3) fp64 (a, b, c) of the dilated 2D covariance
    conic: np.ndarray        # (N,3) fp64 inverse of cov2d (a, b, c)
    opacity: np.ndarray      # (N,)
    rgb: np.ndarray          # (N,3)
    depth: np.ndarray        # (N,) fp64 view z


def project_gaussians(cam, means, opacity, sh, sh_degree, scales=None, quats=None,
                      cov3d=None) -> GaussProj:
    """EWA splatting of each Gaussian into the view (3DGS, the paper's Eq. 1 input).

    cov3d, if given, is the packed (xx, xy, xz, yy, yz, zz) world covariance
    (e.g. after deformation transfer); otherwise Sigma = R(q) diag(s^2) R(q)^T.
    """
    means64 = np.asarray(means, np.float64)      # continuous path (FP64 inputs allowed)
    means = np.asarray(means, F32)                # the depth key is pinned in FP32
    n = means.shape[0]
    R32, t32, fx32, fy32, cx32, cy32 = _cam32(cam)
    z32 = view_row_f32(R32, t32, means, 2)
    valid = z32 > F32(NEAR)

    W = R32.astype(np.float64)
    tv = t32.astype(np.float64)
    fx, fy = float(fx32), float(fy32)
    cx, cy = float(cx32), float(cy32)
    p = means64 @ W.T + tv
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    zs = np.where(valid, z, 1.0)
    Sigma = cov3d_from_packed(cov3d) if cov3d is not None else cov3d_from_scale_rot(scales, quats)

    tanx = cam.width / (2.0 * fx)
    tany = cam.height / (2.0 * fy)
    limx, limy = FRUSTUM_CLAMP * tanx, FRUSTUM_CLAMP * tany
    txc = np.clip(x / zs, -limx, limx) * zs
    tyc = np.clip(y / zs, -limy, limy) * zs
    J = np.zeros((n, 2, 3))
    J[:, 0, 0] = fx / zs
    J[:, 0, 2] = -fx * txc / (zs * zs)
    J[:, 1, 1] = fy / zs
    J[:, 1, 2] = -fy * tyc / (zs * zs)
    M = J @ W[None, :, :]
    S2 = M @ Sigma @ np.transpose(M, (0, 2, 1))
    a = S2[:, 0, 0] + DILATION
    b = S2[:, 0, 1]
    c = S2[:, 1, 1] + DILATION
    det = a * c - b * b
    valid &= det > 0
    dets = np.where(det > 0, det, 1.0)
    conic = np.stack([c / dets, -b / dets, a / dets], -1)
    mean2d = np.stack([fx * x / zs + cx, fy * y / zs + cy], -1)

    cam_c = -(W.T @ tv)
    d = means64 - cam_c[None, :]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rgb = _sh.colour(np.asarray(sh), d, sh_degree)
    return GaussProj(valid=valid, key=z32, mean2d=mean2d, cov2d=np.stack([a, b, c], -1),
                     conic=conic, opacity=np.asarray(opacity, np.float64), rgb=rgb, depth=z)


# ---------------------------------------------------------------------------
# Triangles: fixed-point coverage setup
# ---------------------------------------------------------------------------

@dataclass
class TriSetup:
    valid: np.ndarray        # (T,) bool
    key: np.ndarray          # (T,) float32 depth key (pinned)
    X: np.ndarray            # (T,3) int64 snapped x in 1/256 px, positive orientation
    Y: np.ndarray            # (T,3) int64
    area2: np.ndarray        # (T,) int64 > 0 for valid triangles
    z: np.ndarray            # (T,3) fp64 view z, same vertex order as X/Y
    rgb: np.ndarray          # (T,3,3) per-vertex colour, same vertex order
    alpha: np.ndarray        # (T,)
    uv: Optional[np.ndarray] = None    # (T,3,2) texture coordinates, same vertex order
    order: Optional[np.ndarray] = None # (T,3) input vertex index of each set-up vertex


def setup_triangles(cam, tri_xyz, tri_rgb, tri_alpha, tri_uv=None) -> TriSetup:
    tri_xyz = np.asarray(tri_xyz, F32)
    T = tri_xyz.shape[0]
    R32, t32, fx32, fy32, cx32, cy32 = _cam32(cam)
    P = tri_xyz.reshape(-1, 3)
    xv = view_row_f32(R32, t32, P, 0).reshape(T, 3)
    yv = view_row_f32(R32, t32, P, 1).reshape(T, 3)
    zv = view_row_f32(R32, t32, P, 2).reshape(T, 3)
    valid = np.all(zv > F32(NEAR), axis=1)
    zsafe = np.where(zv > F32(NEAR), zv, F32(1.0))
    with np.errstate(over="ignore", invalid="ignore"):
        u = pixel_f32(fx32, cx32, xv, zsafe)
        v = pixel_f32(fy32, cy32, yv, zsafe)
        us = np.rint(u * F32(SUBPX))
        vs = np.rint(v * F32(SUBPX))
    inrange = (np.abs(us) <= COORD_LIMIT) & (np.abs(vs) <= COORD_LIMIT)
    valid &= np.all(inrange, axis=1)
    X = np.where(valid[:, None], us, 0).astype(np.int64)
    Y = np.where(valid[:, None], vs, 0).astype(np.int64)
    key = ((zv[:, 0] + zv[:, 1]) + zv[:, 2]) * F32(1.0 / 3.0)
    area2 = (X[:, 1] - X[:, 0]) * (Y[:, 2] - Y[:, 0]) - (Y[:, 1] - Y[:, 0]) * (X[:, 2] - X[:, 0])
    valid &= area2 != 0
    # normalise orientation: swap vertices 1 and 2 of negatively oriented triangles
    neg = area2 < 0
    order = np.where(neg[:, None], np.array([0, 2, 1]), np.array([0, 1, 2]))
    r = np.arange(T)[:, None]
    X, Y = X[r, order], Y[r, order]
    area2 = np.abs(area2)
    p64 = tri_xyz.astype(np.float64) @ R32.astype(np.float64).T + t32.astype(np.float64)
    z64 = p64[:, :, 2][r, order]
    rgb = np.asarray(tri_rgb, np.float64)[r, order]
    uv = None if tri_uv is None else np.asarray(tri_uv, F32).astype(np.float64).reshape(T, 3, 2)[r, order]
    return TriSetup(valid=valid, key=key, X=X, Y=Y, area2=area2, z=z64, rgb=rgb,
                    alpha=np.asarray(tri_alpha, np.float64), uv=uv, order=order)


def _edges(X, Y):
    """Edge k is opposite vertex k: (a, b) = (1,2), (2,0), (0,1)."""
    return ((1, 2), (2, 0), (0, 1))


def edge_values(ts: TriSetup, idx, Px, Py):
    """Exact integer edge functions E_k(P) = (Xb-Xa)(Py-Ya) - (Yb-Ya)(Px-Xa)
    for triangles idx at points (Px, Py) in 1/256 px; returns (len(idx), 3)."""
    X, Y = ts.X[idx], ts.Y[idx]
    out = []
    for a, b in _edges(X, Y):
        dx = X[:, b] - X[:, a]
        dy = Y[:, b] - Y[:, a]
        out.append(dx * (Py - Y[:, a]) - dy * (Px - X[:, a]))
    return np.stack(out, -1)


def edge_owned(ts: TriSetup, idx):
    """Tie rule for samples exactly on an edge: an edge a->b owns its points
    iff dy > 0, or dy == 0 and dx < 0 (equivalent to nudging every sample by
    an infinitesimal (-1, -eps)); two triangles sharing an edge traverse it
    in opposite directions, so exactly one of them owns it."""
    X, Y = ts.X[idx], ts.Y[idx]
    out = []
    for a, b in _edges(X, Y):
        dx = X[:, b] - X[:, a]
        dy = Y[:, b] - Y[:, a]
        out.append((dy > 0) | ((dy == 0) & (dx < 0)))
    return np.stack(out, -1)


def sample_coverage(ts: TriSetup, idx, px: int, py: int) -> np.ndarray:
    """o^j for the M = 4 sub-samples of pixel (px, py): (len(idx), 4) bool."""
    owned = edge_owned(ts, idx)
    cov = []
    for ox, oy in SAMPLE_OFFSETS:
        Sx = px * SUBPX + SUBPX // 2 + ox
        Sy = py * SUBPX + SUBPX // 2 + oy
        E = edge_values(ts, idx, Sx, Sy)
        cov.append(np.all((E > 0) | ((E == 0) & owned), axis=1))
    return np.stack(cov, -1)


def centre_coverage(ts: TriSetup, idx, px: int, py: int) -> np.ndarray:
    owned = edge_owned(ts, idx)
    E = edge_values(ts, idx, px * SUBPX + SUBPX // 2, py * SUBPX + SUBPX // 2)
    return np.all((E > 0) | ((E == 0) & owned), axis=1)


def _perspective_weights(ts: TriSetup, idx, px: int, py: int) -> np.ndarray:
    """Perspective-correct barycentric weights at the pixel centre: screen
    barycentrics b_k = E_k(centre) / area2 from the snapped vertices,
    negative ones clamped to 0 and renormalised, then weighted by 1/z_k."""
    E = edge_values(ts, idx, px * SUBPX + SUBPX // 2, py * SUBPX + SUBPX // 2).astype(np.float64)
    b = np.maximum(E, 0.0) / ts.area2[idx, None].astype(np.float64)
    b /= b.sum(axis=1, keepdims=True)
    w = b / ts.z[idx]
    return w / w.sum(axis=1, keepdims=True)


def triangle_colour(ts: TriSetup, idx, px: int, py: int) -> np.ndarray:
    """Perspective-correct per-vertex colour at the pixel centre."""
    lam = _perspective_weights(ts, idx, px, py)
    return np.einsum("nk,nkc->nc", lam, ts.rgb[idx])


def texture_sample(tex: np.ndarray, uv: np.ndarray) -> np.ndarray:
    """Bilinear RGBA of texture tex (H, W, 4) at texture coordinates uv (n, 2):
    texel (i, j) -- column i, row j -- is centred at ((i + 1/2)/W, (j + 1/2)/H),
    addresses clamp to the edge texels, and each interpolation step is
    a + f (b - a) (so a constant texture returns its value exactly)."""
    tex = np.asarray(tex, np.float64)
    H, W = tex.shape[0], tex.shape[1]
    x = uv[:, 0] * W - 0.5
    y = uv[:, 1] * H - 0.5
    x0, y0 = np.floor(x), np.floor(y)
    fx, fy = (x - x0)[:, None], (y - y0)[:, None]
    i0 = np.clip(x0, 0, W - 1).astype(np.int64)
    i1 = np.clip(x0 + 1, 0, W - 1).astype(np.int64)
    j0 = np.clip(y0, 0, H - 1).astype(np.int64)
    j1 = np.clip(y0 + 1, 0, H - 1).astype(np.int64)
    top = tex[j0, i0] + fx * (tex[j0, i1] - tex[j0, i0])
    bot = tex[j1, i0] + fx * (tex[j1, i1] - tex[j1, i0])
    return top + fy * (bot - top)


def triangle_shade(ts: TriSetup, idx, px: int, py: int, tex=None):
    """Colour (n, 3) and opacity (n,) of triangles idx at the pixel centre.
    Untextured: the perspective-correct per-vertex colour and the triangle's
    opacity attribute.  Textured (the paper's Section 1: an opacity attribute
    on textured meshes): the texture coordinates are interpolated with the
    same perspective-correct weights, the texture is sampled bilinearly, the
    colour is the per-vertex colour times the texel RGB and the opacity the
    triangle's attribute times the texel alpha."""
    lam = _perspective_weights(ts, idx, px, py)
    col = np.einsum("nk,nkc->nc", lam, ts.rgb[idx])
    alpha = ts.alpha[idx].astype(np.float64)
    if tex is None or ts.uv is None:
        return col, alpha
    uv = np.einsum("nk,nkc->nc", lam, ts.uv[idx])
    t = texture_sample(tex, uv)
    return col * t[:, :3], alpha * t[:, 3]


# ---------------------------------------------------------------------------
# per-pixel gather, sort and blend
# ---------------------------------------------------------------------------

@dataclass
class PixelResult:
    C: np.ndarray                 # (3,)
    T: float                      # final transmittance (before background)
    n_blended: int                # fragments blended
    last_id: int                  # global id of the last blended fragment, -1 if none
    T_entity_in: float            # T before the last blended unit (a Gaussian, or a whole
                                  # triangle entity; a triangle in direct mode), 1 if none
    order: List[int]              # global ids of the blended fragments, in order
    contributors: List[int]       # all contributors in (key, id) order
    margin: float                 # smallest relative decision margin met
    ambiguous: List[Tuple[str, int]] = field(default_factory=list)
    T_trace: List[float] = field(default_factory=list)   # T after each blended fragment


class Frame:
    """All projected primitives of one view, ready for per-pixel queries."""

    def __init__(self, cam, means, opacity, sh, sh_degree, tri_xyz, tri_rgb, tri_alpha,
                 scales=None, quats=None, cov3d=None, bg=(0.0, 0.0, 0.0),
                 mode: int = MODE_UNIMGS, tri_uv=None, tex=None):
        self.cam = cam
        self.N = int(np.asarray(means).shape[0])
        self.g = project_gaussians(cam, means, opacity, sh, sh_degree, scales, quats, cov3d)
        self.t = setup_triangles(cam, tri_xyz, tri_rgb, tri_alpha, tri_uv)
        self.tex = None if tex is None else np.asarray(tex, F32)
        self.bg = np.asarray(bg, np.float64)
        self.mode = mode
        g = self.g
        # conservative pixel boxes for prefiltering (exact tests follow)
        with np.errstate(divide="ignore", invalid="ignore"):
            L = np.log(np.maximum(g.opacity, 1e-30) * 255.0)
        L = np.where(np.isfinite(L), L, -1.0)
        self.g_live = np.flatnonzero(g.valid & (L > -1e-3))
        Lp = np.maximum(L, 0.0) * (1.0 + 1e-3) + 1e-3
        hx = np.sqrt(2.0 * Lp * np.maximum(g.cov2d[:, 0], 0)) + 1.0
        hy = np.sqrt(2.0 * Lp * np.maximum(g.cov2d[:, 2], 0)) + 1.0
        self.g_box = np.stack([g.mean2d[:, 0] - hx, g.mean2d[:, 0] + hx,
                               g.mean2d[:, 1] - hy, g.mean2d[:, 1] + hy], -1)
        t = self.t
        self.t_live = np.flatnonzero(t.valid)
        self.t_box = np.stack([t.X.min(1) / SUBPX - 1, t.X.max(1) / SUBPX + 1,
                               t.Y.min(1) / SUBPX - 1, t.Y.max(1) / SUBPX + 1], -1)

    # -- candidate gathering ------------------------------------------------
    def _gauss_at(self, px, py, margin_rel):
        cxp, cyp = px + 0.5, py + 0.5
        gl = self.g_live
        bx = self.g_box[gl]
        m = (bx[:, 0] <= cxp) & (cxp <= bx[:, 1]) & (bx[:, 2] <= cyp) & (cyp <= bx[:, 3])
        idx = gl[m]
        g = self.g
        dx = g.mean2d[idx, 0] - cxp
        dy = g.mean2d[idx, 1] - cyp
        con = g.conic[idx]
        power = -0.5 * (con[:, 0] * dx * dx + con[:, 2] * dy * dy) - con[:, 1] * dx * dy
        raw = g.opacity[idx] * np.exp(np.minimum(power, 0.0))
        alpha = np.minimum(ALPHA_MAX, raw)
        ok = power <= 0
        contrib = ok & (alpha >= ALPHA_MIN)
        rel = np.abs(raw - ALPHA_MIN) / ALPHA_MIN
        amb = ok & (rel < margin_rel)
        return idx, alpha, contrib, amb, rel

    def _tris_at(self, px, py):
        cxp, cyp = px + 0.5, py + 0.5
        tl = self.t_live
        bx = self.t_box[tl]
        m = (bx[:, 0] <= cxp) & (cxp <= bx[:, 1]) & (bx[:, 2] <= cyp) & (cyp <= bx[:, 3])
        idx = tl[m]
        if self.mode == MODE_DIRECT:
            cov = centre_coverage(self.t, idx, px, py)[:, None] if idx.size else np.zeros((0, 1), bool)
            hit = cov[:, 0]
        else:
            cov = sample_coverage(self.t, idx, px, py) if idx.size else np.zeros((0, 4), bool)
            hit = cov.any(axis=1)
        return idx[hit], cov[hit]

    # -- the blend ----------------------------------------------------------
    def pixel(self, px: int, py: int, margin_rel: float = 1e-4,
              flips: frozenset = frozenset()) -> PixelResult:
        """Blend pixel (px, py).  ``flips`` names decisions to invert, each
        ('a', gid) for a Gaussian's alpha >= 1/255 test or ('s', gid) for the
        stop test at fragment gid; used to enumerate the valid outcomes of
        decisions that sit within ``margin_rel`` of their threshold."""
        N = self.N
        gidx, galpha, gcon, gamb, grel = self._gauss_at(px, py, margin_rel)
        ambiguous = [("a", int(i)) for i in gidx[gamb]]
        margin = float(grel[gcon | gamb].min()) if np.any(gcon | gamb) else math.inf
        if flips:
            fa = np.array([("a", int(i)) in flips for i in gidx], bool)
            gcon = gcon ^ fa
            galpha = np.where(fa & (galpha < ALPHA_MIN), ALPHA_MIN, galpha)
        g_ids = gidx[gcon]
        g_alpha = dict(zip(g_ids.tolist(), galpha[gcon].tolist()))
        tidx, tcov = self._tris_at(px, py)
        ids = np.concatenate([g_ids, tidx + N]).astype(np.int64)
        keys = np.concatenate([self.g.key[g_ids], self.t.key[tidx]]).astype(F32)
        order = np.lexsort((ids, keys))
        ids = ids[order]
        tri_cov = {int(t) + N: tcov[i] for i, t in enumerate(tidx)}
        tri_col, tri_al = {}, {}
        if tidx.size:
            cols, als = triangle_shade(self.t, tidx, px, py, self.tex)
            tri_col = {int(t) + N: cols[i] for i, t in enumerate(tidx)}
            tri_al = {int(t) + N: float(als[i]) for i, t in enumerate(tidx)}

        C = np.zeros(3)
        T = 1.0
        T_in = 1.0
        T_ent = 1.0
        t_sub = np.ones(M_SAMPLES)
        in_entity = False
        blended: List[int] = []
        trace: List[float] = []
        mode = self.mode
        for gid in ids.tolist():
            if gid < N:
                a = g_alpha[gid]
                test_T = T * (1.0 - a)
                rel = abs(test_T - T_STOP) / T_STOP
                margin = min(margin, rel)
                if rel < margin_rel:
                    ambiguous.append(("s", gid))
                stop = test_T < T_STOP
                if ("s", gid) in flips:
                    stop = not stop
                if stop:
                    break
                T_ent = T
                C += T * a * self.g.rgb[gid]
                T = test_T
                blended.append(gid)
                trace.append(T)
                if mode != MODE_ONE_ENTITY:
                    in_entity = False
            else:
                al = tri_al[gid]
                col = tri_col[gid]
                if mode == MODE_DIRECT:
                    # like a Gaussian, but blended before the stop test (an
                    # opaque triangle must still show its colour)
                    T_ent = T
                    C += T * al * col
                    T = T * (1.0 - al)
                    blended.append(gid)
                    trace.append(T)
                    rel = abs(T - T_STOP) / T_STOP
                    margin = min(margin, rel)
                    if rel < margin_rel:
                        ambiguous.append(("s", gid))
                    if (T < T_STOP) != (("s", gid) in flips):
                        break
                    continue
                o = tri_cov[gid].astype(np.float64)
                if not in_entity:
                    T_in = T
                    T_ent = T
                    t_sub = np.ones(M_SAMPLES)
                    in_entity = True
                O = float(np.mean(o * t_sub))
                C += T_in * O * al * col
                if mode == MODE_LITERAL_T:
                    T = T * (1.0 - O * al)
                    t_sub = t_sub * (1.0 - o * al)
                else:
                    t_sub = t_sub * (1.0 - o * al)
                    T = T_in * float(np.mean(t_sub))
                blended.append(gid)
                trace.append(T)
                rel = abs(T - T_STOP) / T_STOP
                margin = min(margin, rel)
                if rel < margin_rel:
                    ambiguous.append(("s", gid))
                stop = (T < T_STOP) != (("s", gid) in flips)
                if stop:
                    break
        C_pix = C + T * self.bg
        return PixelResult(C=C_pix, T=T, n_blended=len(blended),
                           last_id=blended[-1] if blended else -1,
                           T_entity_in=T_ent, order=blended, contributors=ids.tolist(),
                           margin=margin, ambiguous=ambiguous, T_trace=trace)

    def pixel_variants(self, px, py, margin_rel=1e-4, max_flips=2):
        """Nominal result plus the results with up to ``max_flips`` of the
        pixel's near-threshold decisions inverted (all equally valid)."""
        base = self.pixel(px, py, margin_rel)
        out = [base]
        amb = list(dict.fromkeys(base.ambiguous))
        if not amb:
            return out
        import itertools
        for k in range(1, max_flips + 1):
            for combo in itertools.combinations(amb, k):
                out.append(self.pixel(px, py, margin_rel, frozenset(combo)))
        return out


def render(cam, means, opacity, sh, sh_degree, tri_xyz, tri_rgb, tri_alpha, scales=None,
           quats=None, cov3d=None, bg=(0.0, 0.0, 0.0), pixels: Optional[np.ndarray] = None,
           mode: int = MODE_UNIMGS, margin_rel: float = 1e-4, tri_uv=None,
           tex=None) -> Dict[str, np.ndarray]:
    """Render a full view (or the listed pixels, an (n,2) array of (px, py)).

    Returns image (3,H,W) or (n,3), T_final, n_blended, last_id, T_entity_in,
    margin (per pixel) and the per-pixel blended order (list of lists)."""
    fr = Frame(cam, means, opacity, sh, sh_degree, tri_xyz, tri_rgb, tri_alpha,
               scales, quats, cov3d, bg, mode, tri_uv=tri_uv, tex=tex)
    full = pixels is None
    if full:
        yy, xx = np.mgrid[0:cam.height, 0:cam.width]
        pixels = np.stack([xx.ravel(), yy.ravel()], -1)
    res = [fr.pixel(int(p[0]), int(p[1]), margin_rel) for p in pixels]
    C = np.stack([r.C for r in res])
    out = dict(
        image=C, T_final=np.array([r.T for r in res]),
        n_blended=np.array([r.n_blended for r in res]),
        last_id=np.array([r.last_id for r in res]),
        T_entity_in=np.array([r.T_entity_in for r in res]),
        margin=np.array([r.margin for r in res]),
        order=[r.order for r in res], frame=fr, pixels=pixels)
    if full:
        H, W = cam.height, cam.width
        out["image"] = C.T.reshape(3, H, W)
        for k in ("T_final", "n_blended", "last_id", "T_entity_in", "margin"):
            out[k] = out[k].reshape(H, W)
    return out
