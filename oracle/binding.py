"""Binding association by ray casting (Section 3.3.1): CPU FP64 oracle.

Test infrastructure: only the tests, the smoke check and the CPU baseline use
this module; the library never calls it.

What is computed.  Every Gaussian has K target points: K = 1, its mean; K = 8,
the corners of its bounding box, mu + R(q) diag(3 s) (sx, sy, sz) with signs
+-1, the x sign varying fastest, then y, then z (q normalised first).  From the
centre o_c of every camera c a ray x(t) = o_c + t (P - o_c), t > 0, is cast
towards the target P, which lies at t = 1.  Each proxy face the ray crosses is
a candidate, recorded with the barycentric coordinates of the crossing and its
distance |t - 1| |P - o_c| to the target.  The target is bound to the
candidate nearest to it over all faces and all cameras.

Readings where the text leaves a choice (each also listed in the design notes):
  * every crossing along the ray counts, not only the first one seen from the
    camera (a ray through an outer layer still binds to the inner face that
    lies next to the target);
  * crossings behind the camera (t <= 0) do not count; crossings on a face's
    edge or vertex do (closed triangles);
  * ties in distance go to the lower camera index, then the lower face index;
  * a target that no ray reaches gets face -1, barycentrics (0, 0) and an
    infinite distance;
  * barycentrics (u, v) follow the binding layout of Eq. 12: the crossing is
    u V[f0] + v V[f1] + (1 - u - v) V[f2].

The crossing is the solution (b, g, t) of the 3 x 3 system
A + b (B - A) + g (C - A) = o + t d, written out with Cramer's rule; parity is
pinned against numpy's dense solver, closed-form crossings, surface points
that must bind to their own face and a two-layer mesh that separates "nearest
to the target" from "first hit".
"""
from __future__ import annotations

import numpy as np


def target_points(means, scales, quats, K: int):
    """(N, K, 3) FP64 target points: the means (K = 1) or the eight corners of
    mu + R(q) diag(3 s) [-1, 1]^3 (K = 8), x sign fastest."""
    mu = np.asarray(means, np.float64)
    if K == 1:
        return mu[:, None, :].copy()
    if K != 8:
        raise ValueError("K must be 1 or 8")
    q = np.asarray(quats, np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((mu.shape[0], 3, 3))
    R[:, 0] = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1)
    R[:, 1] = np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1)
    R[:, 2] = np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)
    half = 3.0 * np.asarray(scales, np.float64)
    out = np.empty((mu.shape[0], 8, 3))
    for k in range(8):
        sgn = np.array([1.0 if (k >> a) & 1 else -1.0 for a in range(3)])
        out[:, k] = mu + (R @ (sgn * half)[:, :, None])[:, :, 0]
    return out


def crossings(o, d, A, B, C):
    """Solve A + b (B - A) + g (C - A) = o + t d for (b, g, t) by Cramer's rule,
    broadcasting over leading axes.  det is the determinant of the columns
    (B - A, C - A, -d); where it is zero the line is parallel to the plane and
    (b, g, t) are NaN."""
    e1, e2, m3 = B - A, C - A, -d
    r = o - A
    det = np.einsum("...i,...i->...", e1, np.cross(e2, m3))
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = np.where(det != 0.0, 1.0 / det, np.nan)
        b = np.einsum("...i,...i->...", r, np.cross(e2, m3)) * inv
        g = np.einsum("...i,...i->...", e1, np.cross(r, m3)) * inv
        t = np.einsum("...i,...i->...", e1, np.cross(e2, r)) * inv
    return b, g, t


def candidates(P, cam_centers, V, F, chunk: int = 512):
    """Every (camera, face) crossing for each target point.

    Returns a dict of (M, Ccams, nF) arrays: t, u, v (binding layout), dist
    (distance from the crossing to the target) and margin = min(u, v, w), the
    barycentric distance to the nearest edge (>= 0 inside the face).  Rays
    parallel to a face get NaN."""
    P = np.asarray(P, np.float64).reshape(-1, 3)
    O = np.asarray(cam_centers, np.float64).reshape(-1, 3)
    V = np.asarray(V, np.float64)
    F = np.asarray(F, np.int64)
    A, B, Cv = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    M, nc, nf = P.shape[0], O.shape[0], F.shape[0]
    out = {k: np.empty((M, nc, nf)) for k in ("t", "u", "v", "dist", "margin")}
    for s in range(0, M, chunk):
        p = P[s:s + chunk]
        for c in range(nc):
            d = p - O[c]                                        # (m,3), target at t = 1
            b, g, t = crossings(O[c][None, None, :], d[:, None, :], A[None], B[None], Cv[None])
            u = 1.0 - b - g                                     # weight of V[f0]
            out["t"][s:s + chunk, c] = t
            out["u"][s:s + chunk, c] = u
            out["v"][s:s + chunk, c] = b                        # weight of V[f1]
            out["dist"][s:s + chunk, c] = np.abs(t - 1.0) * np.linalg.norm(d, axis=1)[:, None]
            out["margin"][s:s + chunk, c] = np.minimum(np.minimum(u, b), g)
    return out


def associate(P, cam_centers, V, F, cand=None):
    """Nearest candidate per target: (face (M,) int32, bary (M, 2), dist (M,),
    cam (M,) int32), with the tie and no-hit rules of the module doc."""
    if cand is None:
        cand = candidates(P, cam_centers, V, F)
    t, margin, dist = cand["t"], cand["margin"], cand["dist"]
    hit = (t > 0.0) & (margin >= 0.0)            # NaN compares false: parallel rays miss
    M, nc, nf = t.shape
    dd = np.where(hit, dist, np.inf).reshape(M, nc * nf)
    # lexicographic (dist, camera, face): argmin returns the first minimum,
    # and the flattened order is camera-major, face-minor
    best = np.argmin(dd, axis=1)
    r = np.arange(M)
    bd = dd[r, best]
    cam, face = best // nf, best % nf
    found = np.isfinite(bd)
    u = cand["u"].reshape(M, -1)[r, best]
    v = cand["v"].reshape(M, -1)[r, best]
    face_out = np.where(found, face, -1).astype(np.int32)
    bary = np.where(found[:, None], np.stack([u, v], -1), 0.0)
    return face_out, bary, np.where(found, bd, np.inf), np.where(found, cam, -1).astype(np.int32)


def bind_gaussians(means, scales, quats, K, cam_centers, V, F):
    """Section 3.3.1 for a set of Gaussians: (face (N, K), bary (N, K, 2),
    dist (N, K))."""
    P = target_points(means, scales, quats, K)
    N = P.shape[0]
    f, b, d, _ = associate(P.reshape(-1, 3), cam_centers, V, F)
    return f.reshape(N, K), b.reshape(N, K, 2), d.reshape(N, K)


def camera_center(R, t):
    """Centre of a world->camera transform x_c = R x + t: o = -R^T t."""
    return -np.asarray(R, np.float64).T @ np.asarray(t, np.float64)
