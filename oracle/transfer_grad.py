"""Gradient oracle of the deformation transfer (test infrastructure).

The transfer of oracle/transfer.py (Section 3.3.2, Eq. 12-13, with the
per-vertex ACAP transform) rewritten with PyTorch CPU FP64 operations, so
that autograd gives the gradient of a loss with respect to the deformed
proxy vertices V' from its gradients with respect to the transfer's outputs,
the deformed means mu' and the per-Gaussian linear maps A = R'S' (whose
gradient the Gaussian backward gives through Sigma' = A Sigma A^T):

    L = sum_n dL/dmu'_n . mu'_n + sum_n <dL/dA_n, A_n>.

Two steps are written for differentiation rather than copied from the
forward oracle: the polar factor R of D is the limit of Newton's iteration
X <- (X + X^-T) / 2 from X = D (Higham's method; it reaches the nearest
rotation of oracle/transfer.py's SVD when det D > 0, and unlike the SVD its
derivative stays finite when singular values coincide, e.g. under uniform
scaling), and the rotation log takes theta = atan2(|w|/2, cos theta) with
the series of theta / (2 sin theta) near 0.  Angles stay below 0.9 pi here
(the log's derivative is singular at pi).  mu' is taken in FP64 (the
forward oracle pins its FP32 rounding; the gradient of a rounding is the
identity).
"""
from __future__ import annotations

import numpy as np
import torch

from . import transfer as OT

DT = torch.float64


def _rotated_faces(faces):
    f = torch.as_tensor(np.asarray(faces, np.int64))
    return torch.cat([f, f[:, [1, 2, 0]], f[:, [2, 0, 1]]])


def _cot(p, q, r):
    u1, u2 = q - p, r - p
    return (u1 * u2).sum(-1) / torch.linalg.norm(torch.cross(u1, u2, dim=-1), dim=-1)


def deformation_gradients(V_rest, faces, Vd):
    """D_v = (sum c e' e^T + w n' n^T)(sum c e e^T + w n n^T)^-1 as a torch
    function of the deformed vertices Vd (nV,3)."""
    V = torch.as_tensor(np.asarray(V_rest, np.float64))
    nV = V.shape[0]
    F = _rotated_faces(faces)
    iv, ia, ib = F[:, 0], F[:, 1], F[:, 2]
    cot_b = _cot(V[ib], V[iv], V[ia])
    cot_a = _cot(V[ia], V[iv], V[ib])
    ea, eb = V[ia] - V[iv], V[ib] - V[iv]
    fa, fb = Vd[ia] - Vd[iv], Vd[ib] - Vd[iv]
    outer = lambda x, y: x[:, :, None] * y[:, None, :]
    P = torch.zeros((nV, 3, 3), dtype=DT).index_add(
        0, iv, 0.5 * cot_b[:, None, None] * outer(fa, ea) + 0.5 * cot_a[:, None, None] * outer(fb, eb))
    Q = torch.zeros((nV, 3, 3), dtype=DT).index_add(
        0, iv, 0.5 * cot_b[:, None, None] * outer(ea, ea) + 0.5 * cot_a[:, None, None] * outer(eb, eb))
    nf = torch.zeros(nV, dtype=DT).index_add(0, iv, torch.ones(iv.shape[0], dtype=DT))
    w = torch.zeros(nV, dtype=DT).index_add(0, iv, 0.5 * (cot_a + cot_b)) / nf
    nrm = torch.zeros((nV, 3), dtype=DT).index_add(0, iv, torch.cross(ea, eb, dim=-1))
    nrmd = torch.zeros((nV, 3), dtype=DT).index_add(0, iv, torch.cross(fa, fb, dim=-1))
    ell = torch.zeros(nV, dtype=DT).index_add(
        0, iv, torch.linalg.norm(ea, dim=1) + torch.linalg.norm(eb, dim=1)) / (2 * nf)
    elld = torch.zeros(nV, dtype=DT).index_add(
        0, iv, torch.linalg.norm(fa, dim=1) + torch.linalg.norm(fb, dim=1)) / (2 * nf)
    n = nrm / torch.linalg.norm(nrm, dim=1, keepdim=True) * ell[:, None]
    nd = nrmd / torch.linalg.norm(nrmd, dim=1, keepdim=True) * elld[:, None]
    P = P + w[:, None, None] * outer(nd, n)
    Q = Q + w[:, None, None] * outer(n, n)
    return P @ torch.linalg.inv(Q)


def polar(D, iters=40):
    """D = R S: R by Newton's iteration X <- (X + X^-T)/2, S = sym(R^T D)."""
    if not bool((torch.linalg.det(D) > 0).all()):
        raise ValueError("a deformation gradient with det <= 0 (a reflection)")
    X = D
    for _ in range(iters):
        X = 0.5 * (X + torch.linalg.inv(X).transpose(1, 2))
    S = X.transpose(1, 2) @ D
    return X, 0.5 * (S + S.transpose(1, 2))


def log_rot(R):
    w = torch.stack([R[:, 2, 1] - R[:, 1, 2], R[:, 0, 2] - R[:, 2, 0], R[:, 1, 0] - R[:, 0, 1]], -1)
    c = (R[:, 0, 0] + R[:, 1, 1] + R[:, 2, 2] - 1.0) / 2.0
    s2 = 0.25 * (w * w).sum(1)
    small = s2 < 1e-16
    sn = torch.sqrt(torch.where(small, torch.ones_like(s2), s2))
    th = torch.atan2(sn, c)
    if bool((th > 0.9 * np.pi).any()):
        raise ValueError("a per-vertex rotation beyond 0.9 pi")
    f = torch.where(small, 0.5 * (1.0 + s2 / 6.0), th / (2.0 * sn))
    return f[:, None] * w


def exp_rot(r):
    t2 = (r * r).sum(1)
    small = t2 < 1e-16
    th = torch.sqrt(torch.where(small, torch.ones_like(t2), t2))
    a = torch.where(small, 1.0 - t2 / 6.0, torch.sin(th) / th)
    b = torch.where(small, 0.5 - t2 / 24.0, (1.0 - torch.cos(th)) / (th * th))
    K = torch.zeros((r.shape[0], 3, 3), dtype=DT)
    K[:, 0, 1], K[:, 0, 2] = -r[:, 2], r[:, 1]
    K[:, 1, 0], K[:, 1, 2] = r[:, 2], -r[:, 0]
    K[:, 2, 0], K[:, 2, 1] = -r[:, 1], r[:, 0]
    return torch.eye(3, dtype=DT)[None] + a[:, None, None] * K + b[:, None, None] * (K @ K)


def transfer_torch(V_rest, faces, Vd, means, bind_face, bind_bary):
    """mu' (FP64) and A = R'S' of every Gaussian as torch functions of Vd."""
    faces_np = np.asarray(faces, np.int64)
    D = deformation_gradients(V_rest, faces_np, Vd)
    R, S = polar(D)
    r = log_rot(R)
    delta = Vd - torch.as_tensor(np.asarray(V_rest, np.float64))
    bind_face = np.asarray(bind_face)
    bound = torch.as_tensor(OT.bound_mask(bind_face, faces_np.shape[0]))            # (N,K)
    fv = torch.as_tensor(faces_np[np.where(bound.numpy(), bind_face, 0)])           # (N,K,3)
    bb = np.asarray(bind_bary, np.float64)
    u, v = torch.as_tensor(bb[..., 0]), torch.as_tensor(bb[..., 1])
    bw = torch.stack([u, v, 1.0 - u - v], -1) * bound[..., None]                     # (N,K,3)
    kb = bound.sum(1).to(DT)
    inv = torch.where(kb > 0, 1.0 / torch.clamp(kb, min=1.0), torch.zeros_like(kb))
    r_bar = torch.einsum("nkj,nkjc->nc", bw, r[fv]) * inv[:, None]                  # Eq. 12-13
    S_bar = torch.einsum("nkj,nkjab->nab", bw, S[fv]) * inv[:, None, None]
    S_bar = torch.where((kb > 0)[:, None, None], S_bar, torch.eye(3, dtype=DT)[None])
    A = exp_rot(r_bar) @ S_bar
    mu = torch.as_tensor(np.asarray(means, np.float64)) + \
        torch.einsum("nkj,nkjc->nc", bw, delta[fv]) * inv[:, None]
    return mu, A


def proxy_gradient(V_rest, faces, V_def, means, bind_face, bind_bary, dL_dmeans, dL_dA):
    """dL/dV' (nV,3) for L = sum dL_dmeans . mu' + sum <dL_dA, A>."""
    Vd = torch.tensor(np.asarray(V_def, np.float64), dtype=DT, requires_grad=True)
    mu, A = transfer_torch(V_rest, faces, Vd, means, bind_face, bind_bary)
    L = (mu * torch.as_tensor(np.asarray(dL_dmeans, np.float64))).sum() + \
        (A * torch.as_tensor(np.asarray(dL_dA, np.float64).reshape(-1, 3, 3))).sum()
    L.backward()
    return Vd.grad.numpy()
