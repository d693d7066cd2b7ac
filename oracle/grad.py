"""Gradient oracle (test infrastructure).

Re-evaluates the forward of ``oracle.render`` with PyTorch on the CPU in
FP64, with every discrete decision frozen at the values the NumPy oracle
takes (which fragments each pixel blends, in which order, where it stops,
which sub-samples each triangle covers), and differentiates it with
autograd.  Gradients are with respect to the Gaussian parameters: means,
linear scales, raw (unnormalised) quaternions, opacities in (0, 1) and SH
coefficients.  Triangles are constants.  A deformed scene is handled with
the transfer's A = R'S' and mean offset held constant:
Sigma' = A Sigma(s, q) A^T, mu' = mu + offset.

Per pixel the forward is, with decisions frozen (Section 3.2):
  Gaussian:  C += T a c,  T *= 1 - a,          a = min(0.99, o exp(power));
  triangle entity (Eq. 7-9): T_in = T at its first triangle, t^j = 1;
             C += T_in O a c,  O = mean_j o^j t^j;  t^j *= 1 - o^j a;
             T = T_in mean_j t^j;
  background: C += T C_bg.
Only the UniMGS rule and the direct-blend ablation are differentiated.
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np
import torch

from . import render as OR
from . import sh as SH

DT = torch.float64


def _basis(d: torch.Tensor, degree: int) -> torch.Tensor:
    """Real SH basis of oracle.sh, evaluated with torch ops (same closed-form
    normalisation constants)."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    k = SH._k
    s2 = math.sqrt(2.0)
    out = [torch.full_like(x, k(0, 0))]
    if degree >= 1:
        out += [-s2 * k(1, 1) * y, k(1, 0) * z, -s2 * k(1, 1) * x]
    if degree >= 2:
        xx, yy, zz = x * x, y * y, z * z
        out += [s2 * k(2, 2) * 3.0 * (2.0 * x * y), -s2 * k(2, 1) * 3.0 * y * z,
                k(2, 0) * 0.5 * (2.0 * zz - xx - yy), -s2 * k(2, 1) * 3.0 * x * z,
                s2 * k(2, 2) * 3.0 * (xx - yy)]
    if degree >= 3:
        xx, yy, zz = x * x, y * y, z * z
        out += [-s2 * k(3, 3) * 15.0 * y * (3.0 * xx - yy), s2 * k(3, 2) * 15.0 * (2.0 * x * y * z),
                -s2 * k(3, 1) * 1.5 * y * (4.0 * zz - xx - yy),
                k(3, 0) * 0.5 * z * (2.0 * zz - 3.0 * xx - 3.0 * yy),
                -s2 * k(3, 1) * 1.5 * x * (4.0 * zz - xx - yy), s2 * k(3, 2) * 15.0 * z * (xx - yy),
                -s2 * k(3, 3) * 15.0 * x * (xx - 3.0 * yy)]
    return torch.stack(out, 1)


def _rot(q: torch.Tensor) -> torch.Tensor:
    q = q / q.norm(dim=1, keepdim=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def project_torch(cam, means, scales, quats, opacity, sh, degree, xform=None, mean_offset=None):
    """EWA projection of oracle.render.project_gaussians, differentiable."""
    W = torch.tensor(np.asarray(cam.R, np.float32).astype(np.float64), dtype=DT)
    t = torch.tensor(np.asarray(cam.t, np.float32).astype(np.float64), dtype=DT)
    fx, fy = float(np.float32(cam.fx)), float(np.float32(cam.fy))
    cx, cy = float(np.float32(cam.cx)), float(np.float32(cam.cy))
    mu = means if mean_offset is None else means + mean_offset
    p = mu @ W.T + t
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    Rq = _rot(quats)
    Sig = Rq @ torch.diag_embed(scales * scales) @ Rq.transpose(1, 2)
    if xform is not None:
        Sig = xform @ Sig @ xform.transpose(1, 2)
    tanx, tany = cam.width / (2.0 * fx), cam.height / (2.0 * fy)
    limx, limy = OR.FRUSTUM_CLAMP * tanx, OR.FRUSTUM_CLAMP * tany
    txc = torch.clamp(x / z, -limx, limx) * z
    tyc = torch.clamp(y / z, -limy, limy) * z
    zero = torch.zeros_like(z)
    J = torch.stack([torch.stack([fx / z, zero, -fx * txc / (z * z)], -1),
                     torch.stack([zero, fy / z, -fy * tyc / (z * z)], -1)], -2)
    M = J @ W
    S2 = M @ Sig @ M.transpose(1, 2)
    a = S2[:, 0, 0] + OR.DILATION
    b = S2[:, 0, 1]
    c = S2[:, 1, 1] + OR.DILATION
    det = a * c - b * b
    conic = torch.stack([c / det, -b / det, a / det], -1)
    mean2d = torch.stack([fx * x / z + cx, fy * y / z + cy], -1)
    cam_c = -(W.T @ t)
    d = mu - cam_c
    d = d / d.norm(dim=1, keepdim=True)
    B = _basis(d, degree)
    nc = (degree + 1) ** 2
    rgb = torch.clamp(torch.einsum("nk,nkc->nc", B, sh[:, :nc, :]) + 0.5, min=0.0)
    return mean2d, conic, rgb


def render_pixels(frame: OR.Frame, pixels, means, scales, quats, opacity, sh, degree,
                  xform=None, mean_offset=None, results=None, tri_rgb=None, tri_alpha=None):
    """C (P,3) and T (P,) of the listed pixels as torch functions of the
    Gaussian parameters -- and of the triangles' per-vertex colours tri_rgb
    (T,3,3) and opacity attributes tri_alpha (T,) when those are given as
    tensors -- decisions frozen from ``frame`` (an oracle Frame built at the
    same parameter values).  A triangle's colour at a pixel is
    sum_k w_k rgb_k (times the texel RGB) with its perspective-correct
    weights w_k, its opacity alpha (times the texel alpha); coverage is a
    constant of the geometry."""
    if results is None:
        results = [frame.pixel(int(px), int(py)) for px, py in pixels]
    N = frame.N
    mode = frame.mode
    assert mode in (OR.MODE_UNIMGS, OR.MODE_DIRECT)
    P = len(pixels)
    L = max([len(r.order) for r in results] + [1])
    ids = np.full((P, L), -1, np.int64)
    for i, r in enumerate(results):
        ids[i, :len(r.order)] = r.order
    valid = ids >= 0
    isg = valid & (ids < N)
    ist = valid & (ids >= N)
    # triangle constants: coverage, interpolation weights of the input
    # vertices and texel factors at each (pixel, position)
    tcov = np.zeros((P, L, 4))
    tw = np.zeros((P, L, 3))
    tvid = np.zeros((P, L, 3), np.int64)
    tfac = np.ones((P, L, 4))
    ttid = np.zeros((P, L), np.int64)
    ts = frame.t
    for i, (px, py) in enumerate(pixels):
        cols = np.flatnonzero(ist[i])
        if cols.size == 0:
            continue
        tid = ids[i, cols] - N
        if mode == OR.MODE_DIRECT:
            cov = np.ones((cols.size, 4))
        else:
            cov = OR.sample_coverage(ts, tid, int(px), int(py)).astype(np.float64)
        tcov[i, cols] = cov
        lam = OR._perspective_weights(ts, tid, int(px), int(py))
        tw[i, cols] = lam
        tvid[i, cols] = ts.order[tid]
        ttid[i, cols] = tid
        if frame.tex is not None and ts.uv is not None:
            uvs = np.einsum("nk,nkc->nc", lam, ts.uv[tid])
            tfac[i, cols] = OR.texture_sample(frame.tex, uvs)
    if tri_rgb is None:
        tri_rgb = torch.tensor(np.asarray(ts.rgb, np.float64)[np.arange(ts.rgb.shape[0])[:, None],
                                                              np.argsort(ts.order, 1)], dtype=DT) \
            if ts.rgb.shape[0] else torch.zeros((0, 3, 3), dtype=DT)
    if tri_alpha is None:
        tri_alpha = torch.tensor(ts.alpha, dtype=DT)
    tt = torch.tensor(ttid)
    vrgb = tri_rgb[tt[..., None], torch.tensor(tvid)] if tri_rgb.shape[0] else \
        torch.zeros((P, L, 3, 3), dtype=DT)                          # (P,L,3 vertices,3)
    fac = torch.tensor(tfac, dtype=DT)
    tcol_t = (torch.tensor(tw, dtype=DT)[..., None] * vrgb).sum(2) * fac[..., :3]
    tal_t = (tri_alpha[tt] if tri_alpha.shape[0] else torch.zeros((P, L), dtype=DT)) * fac[..., 3]

    mean2d, conic, rgb = project_torch(frame.cam, means, scales, quats, opacity, sh, degree,
                                       xform, mean_offset)
    gi = torch.tensor(np.where(isg, ids, 0))
    pc = torch.tensor(np.asarray(pixels, np.float64) + 0.5, dtype=DT)
    dx = mean2d[gi, 0] - pc[:, None, 0]
    dy = mean2d[gi, 1] - pc[:, None, 1]
    con = conic[gi]
    power = -0.5 * (con[..., 0] * dx * dx + con[..., 2] * dy * dy) - con[..., 1] * dx * dy
    ga = torch.clamp(opacity[gi] * torch.exp(torch.clamp(power, max=0.0)), max=OR.ALPHA_MAX)
    gcol = rgb[gi]
    isg_t = torch.tensor(isg)
    ist_t = torch.tensor(ist)
    tcov_t = torch.tensor(tcov, dtype=DT)

    C = torch.zeros((P, 3), dtype=DT)
    T = torch.ones(P, dtype=DT)
    T_in = torch.ones(P, dtype=DT)
    tsub = torch.ones((P, 4), dtype=DT)
    in_ent = torch.zeros(P, dtype=torch.bool)
    for l in range(L):
        g = isg_t[:, l]
        tr = ist_t[:, l]
        a = ga[:, l]
        C = C + torch.where(g[:, None], T[:, None] * a[:, None] * gcol[:, l], torch.zeros_like(C))
        Tg = T * (1.0 - a)
        if mode == OR.MODE_DIRECT:
            at = tal_t[:, l]
            C = C + torch.where(tr[:, None], T[:, None] * at[:, None] * tcol_t[:, l], torch.zeros_like(C))
            T = torch.where(g, Tg, torch.where(tr, T * (1.0 - at), T))
            continue
        T = torch.where(g, Tg, T)
        in_ent = in_ent & ~g
        opening = tr & ~in_ent
        T_in = torch.where(opening, T, T_in)
        tsub = torch.where(opening[:, None], torch.ones_like(tsub), tsub)
        o = tcov_t[:, l]
        at = tal_t[:, l]
        O = (o * tsub).mean(1)
        C = C + torch.where(tr[:, None], (T_in * O * at)[:, None] * tcol_t[:, l], torch.zeros_like(C))
        tsub = torch.where(tr[:, None], tsub * (1.0 - o * at[:, None]), tsub)
        T = torch.where(tr, T_in * tsub.mean(1), T)
        in_ent = in_ent | tr
    bg = torch.tensor(frame.bg, dtype=DT)
    return C + T[:, None] * bg[None, :], T


def gradients(cam, pixels, dL_dC, means, scales, quats, opacity, sh, degree, tri_xyz, tri_rgb,
              tri_alpha, bg=(0.0, 0.0, 0.0), mode=OR.MODE_UNIMGS, xform=None,
              mean_offset=None, tri_uv=None, tex=None) -> Dict[str, np.ndarray]:
    """dL/d(means, scales, quats, opacity, sh) and dL/d(tri_rgb, tri_alpha)
    (and dL/dA as "xform" for a deformed scene) for L = sum_p dL_dC[p] . C[p]
    over the listed pixels.  Inputs are NumPy
    arrays; xform (N,3,3) and mean_offset (N,3) describe a deformed scene
    (then ``means`` are the rest means and the frame is built from means +
    mean_offset and A Sigma A^T)."""
    def t64(a):
        return torch.tensor(np.asarray(a, np.float64), dtype=DT, requires_grad=True)
    if xform is not None:
        Sig = OR.cov3d_from_scale_rot(scales, quats)
        A = np.asarray(xform, np.float64)
        Sp = A @ Sig @ np.transpose(A, (0, 2, 1))
        cov = np.stack([Sp[:, 0, 0], Sp[:, 0, 1], Sp[:, 0, 2], Sp[:, 1, 1], Sp[:, 1, 2], Sp[:, 2, 2]], 1)
        mu = np.asarray(means, np.float64) + np.asarray(mean_offset, np.float64)
        frame = OR.Frame(cam, mu, opacity, sh, degree, tri_xyz, tri_rgb, tri_alpha, cov3d=cov,
                         bg=bg, mode=mode, tri_uv=tri_uv, tex=tex)
    else:
        frame = OR.Frame(cam, means, opacity, sh, degree, tri_xyz, tri_rgb, tri_alpha,
                         scales=scales, quats=quats, bg=bg, mode=mode, tri_uv=tri_uv, tex=tex)
    P = [t64(means), t64(scales), t64(quats), t64(opacity), t64(sh), t64(tri_rgb), t64(tri_alpha)]
    A_t = None if xform is None else torch.tensor(np.asarray(xform, np.float64), dtype=DT,
                                                  requires_grad=True)
    off_t = None if mean_offset is None else torch.tensor(np.asarray(mean_offset, np.float64), dtype=DT)
    C, T = render_pixels(frame, pixels, *P[:5], degree, A_t, off_t, tri_rgb=P[5], tri_alpha=P[6])
    L = (C * torch.tensor(np.asarray(dL_dC, np.float64), dtype=DT)).sum()
    L.backward()
    names = ["means", "scales", "quats", "opacity", "sh", "tri_rgb", "tri_alpha"]
    out = ({n: (p.grad.numpy() if p.grad is not None else np.zeros(p.shape)) for n, p in zip(names, P)}
           | {"C": C.detach().numpy(), "T": T.detach().numpy()})
    if A_t is not None:
        out["xform"] = A_t.grad.numpy() if A_t.grad is not None else np.zeros(A_t.shape)
    return out
