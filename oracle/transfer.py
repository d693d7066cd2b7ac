"""Deformation-transfer oracle (test infrastructure).

Follows the paper's Section 3.3.2 (Eq. 12-13) in FP64, plus the per-vertex
transform that the paper takes from ACAP:

Per proxy vertex v (rest positions V, deformed V'):
  * offset  Delta_v = V'_v - V_v;
  * deformation gradient D_v: the least-squares map of the vertex's rest
    1-ring edges onto the deformed ones with cotangent weights
    c_vu = (cot a + cot b) / 2 (rest angles opposite the edge), augmented by
    one normal pair (rest normal n_v -> deformed normal n'_v, each scaled by
    the mean 1-ring edge length of its mesh, weight = mean c_vu) so the
    normal direction of D is defined on flat or nearly flat 1-rings:
        D = (sum c e' e^T + w n' n^T) (sum c e e^T + w n n^T)^-1;
  * polar decomposition D = R S (R the nearest rotation, via SVD);
  * r_v = log R_v as an axis-angle vector (principal branch, angle in
    [0, pi]; see log_rot for its evaluation near pi).

Per Gaussian with K bindings (face f_i, barycentric (u, v, w = 1 - u - v) of
the bound point P_i, i = 1..K; K = 8 bounding-box corners or K = 1 centre):
  * Eq. 12: Delta_i, r_i, S_i interpolated from the face's vertices;
  * Eq. 13: R' = exp(mean r_i), S' = mean S_i, A = R' S',
    Sigma' = A Sigma A^T, mu' = mu + mean Delta_i.
The output quaternion is q' = quat(R') (x) q.

Unbound corners (the paper's Section 3.3.1 leaves them open: a ray that
crosses no face binds nothing): a corner whose face index lies outside
[0, nF) -- the ray-cast binding writes -1 there -- is left out of Eq. 13,
which then averages over the k_b bound corners only; a Gaussian with no
bound corner keeps its rest pose (mu' = mu, R' = I, S' = I, q' = q).

mu' is defined in float32 by a fixed operation order (one rounding per op):
Delta_v = V'_v - V_v; w = (1 - u) - v; Delta_i = (u Delta_a + v Delta_b)
+ w Delta_c; s = ((Delta_1 + Delta_2) + ...) + Delta_K over the bound
corners in corner order; mu' = mu + s * (1/k_b) with 1/k_b rounded to
float32 (mu' = mu when k_b = 0).
It is the mean that orders the deformed Gaussians, so it is pinned like the
rasterizer's other decision values.
"""
from __future__ import annotations

import math

import numpy as np

F32 = np.float32


def _rotate_faces(faces):
    """The three rotations (v, a, b) of every face, preserving orientation."""
    f = np.asarray(faces, np.int64)
    return np.concatenate([f, f[:, [1, 2, 0]], f[:, [2, 0, 1]]])


def cot_weights_per_corner(V, faces):
    """For each rotated face (v, a, b): cot of the angle at b (opposite edge
    v-a) and at a (opposite edge v-b)."""
    F = _rotate_faces(faces)
    v, a, b = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]

    def cot(p, q, r):           # angle at p between p->q and p->r
        u1, u2 = q - p, r - p
        return (u1 * u2).sum(-1) / np.linalg.norm(np.cross(u1, u2), axis=-1)
    return F, cot(b, v, a), cot(a, v, b)


def deformation_gradients(V_rest, faces, V_def):
    V = np.asarray(V_rest, np.float64)
    Vd = np.asarray(V_def, np.float64)
    nV = V.shape[0]
    F, cot_b, cot_a = cot_weights_per_corner(V, faces)
    iv, ia, ib = F[:, 0], F[:, 1], F[:, 2]
    ea, eb = V[ia] - V[iv], V[ib] - V[iv]
    fa, fb = Vd[ia] - Vd[iv], Vd[ib] - Vd[iv]
    P = np.zeros((nV, 3, 3))
    Q = np.zeros((nV, 3, 3))
    np.add.at(P, iv, 0.5 * cot_b[:, None, None] * np.einsum("ni,nj->nij", fa, ea)
              + 0.5 * cot_a[:, None, None] * np.einsum("ni,nj->nij", fb, eb))
    np.add.at(Q, iv, 0.5 * cot_b[:, None, None] * np.einsum("ni,nj->nij", ea, ea)
              + 0.5 * cot_a[:, None, None] * np.einsum("ni,nj->nij", eb, eb))
    wsum = np.bincount(iv, 0.5 * (cot_a + cot_b), nV)
    nf = np.bincount(iv, None, nV).astype(np.float64)
    nrm = np.zeros((nV, 3))
    nrmd = np.zeros((nV, 3))
    np.add.at(nrm, iv, np.cross(ea, eb))
    np.add.at(nrmd, iv, np.cross(fa, fb))
    ell = np.bincount(iv, np.linalg.norm(ea, axis=1) + np.linalg.norm(eb, axis=1), nV) / (2 * nf)
    elld = np.bincount(iv, np.linalg.norm(fa, axis=1) + np.linalg.norm(fb, axis=1), nV) / (2 * nf)
    n = nrm / np.linalg.norm(nrm, axis=1, keepdims=True) * ell[:, None]
    nd = nrmd / np.linalg.norm(nrmd, axis=1, keepdims=True) * elld[:, None]
    w = wsum / nf
    P += w[:, None, None] * np.einsum("ni,nj->nij", nd, n)
    Q += w[:, None, None] * np.einsum("ni,nj->nij", n, n)
    return P @ np.linalg.inv(Q)


def polar(D):
    """D = R S with R the proper rotation nearest to D: R = U diag(1,1,det(U V^T)) V^T."""
    U, s, Vt = np.linalg.svd(D)
    d = np.sign(np.linalg.det(U @ Vt))
    E = np.tile(np.eye(3), (D.shape[0], 1, 1))
    E[:, 2, 2] = d
    Rm = U @ E @ Vt
    S = np.transpose(Rm, (0, 2, 1)) @ D
    return Rm, 0.5 * (S + np.transpose(S, (0, 2, 1)))


def log_rot(Rm):
    """Principal axis-angle vector r = theta a of rotation matrices (theta in
    [0, pi]).  With vee = (R32 - R23, R13 - R31, R21 - R12) = 2 sin(theta) a
    and cos(theta) = (tr R - 1) / 2, theta = atan2(|vee| / 2, cos theta)
    (accurate at both ends, unlike arccos near pi).  Up to pi/2,
    r = theta / (2 sin theta) vee (its series near 0); beyond, where sin theta
    no longer carries the axis accurately, the axis comes from the symmetric
    part (R + R^T) / 2 - cos(theta) I = (1 - cos theta) a a^T: its column with
    the largest diagonal entry, normalised and signed to agree with vee
    (at theta = pi exactly, where -a is as good as a, that column's own
    sign)."""
    Rm = np.asarray(Rm, np.float64)
    n = Rm.shape[0]
    c = (np.trace(Rm, axis1=1, axis2=2) - 1.0) / 2.0
    vee = np.stack([Rm[:, 2, 1] - Rm[:, 1, 2], Rm[:, 0, 2] - Rm[:, 2, 0],
                    Rm[:, 1, 0] - Rm[:, 0, 1]], -1)
    sn = 0.5 * np.linalg.norm(vee, axis=1)
    th = np.arctan2(sn, c)
    small = th < 1e-4
    # th / (2 sin th) with its series 1/2 (1 + th^2/6) near 0
    f = np.where(small, 0.5 * (1.0 + th * th / 6.0), th / (2.0 * np.where(small, 1.0, sn)))
    r = f[:, None] * vee
    big = c < 0.0
    if np.any(big):
        B = 0.5 * (Rm[big] + np.transpose(Rm[big], (0, 2, 1))) - c[big, None, None] * np.eye(3)
        k = np.argmax(np.diagonal(B, axis1=1, axis2=2), axis=1)
        col = B[np.arange(B.shape[0]), :, k]
        a = col / np.sqrt(B[np.arange(B.shape[0]), k, k] * (1.0 - c[big]))[:, None]
        sg = np.sign((a * vee[big]).sum(1))
        sg[sg == 0] = 1.0
        r[big] = (th[big] * sg)[:, None] * a
    return r


def exp_rot(r):
    """Rodrigues: exp of axis-angle vectors (n,3) -> (n,3,3)."""
    th = np.linalg.norm(r, axis=1)
    small = th < 1e-4
    ths = np.where(small, 1.0, th)
    a = np.where(small, 1.0 - th ** 2 / 6.0, np.sin(ths) / ths)
    b = np.where(small, 0.5 - th ** 2 / 24.0, (1.0 - np.cos(ths)) / ths ** 2)
    K = np.zeros((r.shape[0], 3, 3))
    K[:, 0, 1], K[:, 0, 2] = -r[:, 2], r[:, 1]
    K[:, 1, 0], K[:, 1, 2] = r[:, 2], -r[:, 0]
    K[:, 2, 0], K[:, 2, 1] = -r[:, 1], r[:, 0]
    I = np.eye(3)[None]
    return I + a[:, None, None] * K + b[:, None, None] * (K @ K)


def quat_of_axis_angle(r):
    th = np.linalg.norm(r, axis=1)
    half = 0.5 * th
    s = np.where(th < 1e-12, 0.5, np.sin(half) / np.where(th < 1e-12, 1.0, th))
    return np.concatenate([np.cos(half)[:, None], s[:, None] * r], 1)


def quat_mul(p, q):
    pw, px, py, pz = p.T
    qw, qx, qy, qz = q.T
    return np.stack([pw * qw - px * qx - py * qy - pz * qz,
                     pw * qx + px * qw + py * qz - pz * qy,
                     pw * qy - px * qz + py * qw + pz * qx,
                     pw * qz + px * qy - py * qx + pz * qw], 1)


def vertex_transforms(V_rest, faces, V_def):
    """Per-vertex (Delta_v float32, r_v, S_v) of the deformed proxy."""
    D = deformation_gradients(V_rest, faces, V_def)
    Rm, S = polar(D)
    r = log_rot(Rm)
    delta32 = np.asarray(V_def, F32) - np.asarray(V_rest, F32)
    return dict(delta32=delta32, D=D, R=Rm, S=S, r=r)


def _cov3d(scales, quats):
    q = np.asarray(quats, np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    Rq = np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)
    return np.einsum("nij,nj,nkj->nik", Rq, np.asarray(scales, np.float64) ** 2, Rq)


def bound_mask(bind_face, nF):
    """True where a corner is bound to a face of the proxy (index in [0, nF))."""
    f = np.asarray(bind_face)
    return (f >= 0) & (f < nF)


def pinned_mean(means, delta32, faces, bind_face, bind_bary):
    """mu' in float32 with the fixed operation order stated in the module doc."""
    K = bind_face.shape[1]
    faces = np.asarray(faces, np.int64)
    bound = bound_mask(bind_face, faces.shape[0])
    fv = faces[np.where(bound, bind_face, 0)]               # (N,K,3)
    u = bind_bary[:, :, 0].astype(F32)
    v = bind_bary[:, :, 1].astype(F32)
    w = (F32(1.0) - u) - v
    N = fv.shape[0]
    s = np.zeros((N, 3), F32)
    started = np.zeros(N, bool)
    for i in range(K):
        da, db, dc = delta32[fv[:, i, 0]], delta32[fv[:, i, 1]], delta32[fv[:, i, 2]]
        di = (u[:, i, None] * da + v[:, i, None] * db) + w[:, i, None] * dc
        b = bound[:, i]
        s = np.where((b & started)[:, None], s + di, np.where((b & ~started)[:, None], di, s))
        started |= b
    kb = bound.sum(1)
    inv = np.where(kb > 0, F32(1.0) / np.maximum(kb, 1).astype(F32), F32(0.0)).astype(F32)
    m = np.asarray(means, F32)
    return np.where((kb > 0)[:, None], m + s * inv[:, None], m)


def gaussians_from_frames(frames, faces, means, quats, scales, bind_face, bind_bary,
                          chunk=1 << 17):
    """Eq. 12 at every bound corner, then Eq. 13, from the per-vertex frames
    ``frames`` = dict(delta32 (nV,3) float32, r (nV,3) axis-angle, S (nV,3,3)).

    Returns means' (float32, pinned), cov3d' packed (xx,xy,xz,yy,yz,zz),
    quats' (w,x,y,z) and A = R'S' (N,3,3), all but means' in FP64."""
    faces = np.asarray(faces, np.int64)
    bind_face = np.asarray(bind_face)
    means32 = pinned_mean(means, frames["delta32"], faces, bind_face, bind_bary)
    N = means.shape[0]
    cov = np.empty((N, 6))
    A_all = np.empty((N, 3, 3))
    q_all = np.empty((N, 4))
    for s0 in range(0, N, chunk):
        sl = slice(s0, min(N, s0 + chunk))
        bound = bound_mask(bind_face[sl], faces.shape[0])            # (n,K)
        fv = faces[np.where(bound, bind_face[sl], 0)]                # (n,K,3)
        u = bind_bary[sl, :, 0].astype(np.float64)
        v = bind_bary[sl, :, 1].astype(np.float64)
        w = 1.0 - u - v
        bw = np.stack([u, v, w], -1)                                 # (n,K,3)
        r_i = np.einsum("nkj,nkjc->nkc", bw, frames["r"][fv])        # Eq. 12
        S_i = np.einsum("nkj,nkjab->nkab", bw, frames["S"][fv])
        kb = bound.sum(1).astype(np.float64)
        ks = np.maximum(kb, 1.0)
        # Eq. 13: the mean over the bound corners; none bound: rest pose
        r_bar = (r_i * bound[:, :, None]).sum(1) / ks[:, None]
        S_bar = (S_i * bound[:, :, None, None]).sum(1) / ks[:, None, None]
        S_bar[kb == 0] = np.eye(3)
        Rp = exp_rot(r_bar)
        A = Rp @ S_bar
        Sig = _cov3d(scales[sl], quats[sl])
        Sp = A @ Sig @ np.transpose(A, (0, 2, 1))
        cov[sl] = np.stack([Sp[:, 0, 0], Sp[:, 0, 1], Sp[:, 0, 2], Sp[:, 1, 1], Sp[:, 1, 2],
                            Sp[:, 2, 2]], 1)
        A_all[sl] = A
        q = np.asarray(quats[sl], np.float64)
        q = q / np.linalg.norm(q, axis=1, keepdims=True)
        q_all[sl] = quat_mul(quat_of_axis_angle(r_bar), q)
    return dict(means=means32, cov3d=cov, quats=q_all, A=A_all)


def transfer(V_rest, faces, V_def, means, quats, scales, bind_face, bind_bary, chunk=1 << 17):
    """Deformed Gaussians: means' (float32, pinned), cov3d' packed (xx,xy,xz,yy,yz,zz),
    quats' (w,x,y,z) and A = R'S' (N,3,3), all but means' in FP64; ``vertex``
    holds the per-vertex frames."""
    vt = vertex_transforms(V_rest, faces, V_def)
    out = gaussians_from_frames(vt, faces, means, quats, scales, bind_face, bind_bary, chunk)
    out["vertex"] = vt
    return out
