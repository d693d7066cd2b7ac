"""GPU backward (umgs_backward through the C ABI) vs the FP64 gradient oracle
and vs central finite differences of the FP64 forward oracle.

Tolerance: 1e-3 relative per element, with an absolute floor of 1e-5 times
the largest gradient magnitude of the same array (FP32 sums over many
pixels against FP64).  Pixels holding a decision within 1e-4 (relative) of
its threshold get zero loss weight on both sides, so both sides blend the
same fragments wherever the loss looks.
"""
import math
import sys

import numpy as np
import pytest

from oracle import grad as OG
from oracle import render as OR
from oracle import transfer as OT
from paper_2601_19233_amd import scenes
from tests.test_oracle_grad import mixed_scene

pytestmark = pytest.mark.gpu
NAMES = ["means", "scales", "quats", "opacity", "sh"]


def note(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def assert_close(gpu, ref, name, rtol=1e-3, floor=1e-5):
    gpu = np.asarray(gpu, np.float64).reshape(ref.shape)
    scale = np.abs(ref).max()
    err = np.abs(gpu - ref)
    bad = err > rtol * np.abs(ref) + floor * scale
    assert not bad.any(), (f"{name}: {bad.sum()} of {bad.size} elements off; worst rel "
                           f"{(err / (np.abs(ref) + 1e-30)).max():.3g}, max|ref| {scale:.3g}")


def gpu_grads(cam, means, scales, quats, opac, sh, deg, xyz, rgb, al, dL, mode=0, bg=(0.1, 0.2, 0.3)):
    import torch
    from paper_2601_19233_amd.render import Rasterizer
    r = Rasterizer("cuda:0", sh_degree=deg, mode=mode, bg=bg)
    T = xyz.shape[0]
    out = r.render([cam], means=means, scales=scales, quats=quats, opacity=opac,
                   sh=sh.reshape(sh.shape[0], -1), tri_xyz=xyz.reshape(T, 9), tri_rgb=rgb.reshape(T, 9),
                   tri_alpha=al)
    dLt = torch.from_numpy(np.ascontiguousarray(dL.T.reshape(-1), np.float32)).cuda()
    g = r.backward(dLt, out, means, scales, quats, sh.reshape(sh.shape[0], -1))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}, out


def mask_ambiguous(fr, px, dL):
    """Zero the loss weight of pixels with a near-threshold decision."""
    amb = np.array([fr.pixel(x, y).margin <= 1e-4 for x, y in px])
    assert amb.mean() < 0.05
    dL = dL.copy()
    dL[amb] = 0.0
    return dL


@pytest.mark.parametrize("mode,deg,seed", [(0, 0, 2), (1, 0, 2), (0, 3, 3)])
def test_backward_matches_oracle_gradient(gpu, mode, deg, seed):
    cam, means, scales, quats, opac, sh, xyz, rgb, al = mixed_scene(seed, degree=deg, W=24, H=20)
    note(f"backward mode={mode} deg={deg}")
    f32 = lambda a: np.asarray(a, np.float32)
    means, scales, quats, opac, sh = (f32(a) for a in (means, scales, quats, opac, sh))
    px = [(x, y) for y in range(cam.height) for x in range(cam.width)]
    fr = OR.Frame(cam, means, opac, sh, deg, xyz, rgb, al, scales=scales, quats=quats,
                  bg=(0.1, 0.2, 0.3), mode=mode)
    rng = np.random.default_rng(11)
    W, H = cam.width, cam.height
    dL = mask_ambiguous(fr, px, rng.normal(size=(W * H, 3)))   # per pixel (row-major), per channel
    dL_img = dL.reshape(H, W, 3).transpose(2, 0, 1)      # (3,H,W)
    ref = OG.gradients(cam, px, dL, means, scales, quats, opac, sh, deg, xyz, rgb, al,
                       bg=(0.1, 0.2, 0.3), mode=mode)
    g, _ = gpu_grads(cam, means, scales, quats, opac, sh, deg, xyz, rgb, al,
                     dL_img.reshape(3, -1).T, mode)
    for n in NAMES:
        assert_close(g[n], ref[n], n)


def test_backward_matches_finite_differences(gpu):
    """GPU gradients against central differences of the FP64 forward oracle
    (h = 1e-6 max(1, |theta|)) for every parameter of two Gaussians."""
    cam, means, scales, quats, opac, sh, xyz, rgb, al = mixed_scene(2, W=24, H=20)
    f32 = lambda a: np.asarray(a, np.float32)
    means, scales, quats, opac, sh = (f32(a) for a in (means, scales, quats, opac, sh))
    note("backward vs finite differences")
    px = [(x, y) for y in range(cam.height) for x in range(cam.width)]
    rng = np.random.default_rng(12)
    dL = rng.normal(size=(len(px), 3))
    W, H = cam.width, cam.height
    g, _ = gpu_grads(cam, means, scales, quats, opac, sh, 0, xyz, rgb, al, dL)
    params = [means.astype(np.float64), scales.astype(np.float64), quats.astype(np.float64),
              opac.astype(np.float64), sh.astype(np.float64)]

    def L(pp):
        fr = OR.Frame(cam, pp[0], pp[3], pp[4], 0, xyz, rgb, al, scales=pp[1], quats=pp[2],
                      bg=(0.1, 0.2, 0.3))
        res = [fr.pixel(x, y) for x, y in px]
        return float((np.stack([r.C for r in res]) * dL).sum()), [tuple(r.order) for r in res]

    _, sig0 = L(params)
    checked = 0
    gmax = {n: np.abs(g[n]).max() for n in NAMES}
    for gi in (0, 3):
        for pi, n in enumerate(NAMES):
            arr = params[pi]
            for comp in np.ndindex(arr.shape[1:]):
                idx = (gi,) + comp
                h = 1e-6 * max(1.0, abs(arr[idx]))
                vals, ok = [], True
                for sgn in (1, -1):
                    pp = [p.copy() for p in params]
                    pp[pi][idx] += sgn * h
                    v, sig = L(pp)
                    ok &= sig == sig0
                    vals.append(v)
                if not ok:
                    continue
                fd = (vals[0] - vals[1]) / (2 * h)
                an = g[n].reshape(arr.shape)[idx]
                assert abs(an - fd) <= 1e-3 * abs(fd) + 1e-5 * gmax[n], (n, idx, an, fd)
                checked += 1
    assert checked >= 20


def test_deformed_backward_matches_oracle(gpu):
    """Deformed scene: GPU transfer + forward + backward (rest parameters)
    against the oracle gradient with the oracle transfer's A and mean offset."""
    import torch
    from paper_2601_19233_amd.render import Rasterizer, render_differentiable
    s = scenes.make_config(1, scale=0.0008, res_scale=0.02)
    cam = s.cams[0]
    note(f"deformed backward N={s.N} T={s.T} {cam.width}x{cam.height}")
    ot = OT.transfer(s.proxy.V_rest, s.proxy.faces, s.proxy.V_def, s.means, s.quats, s.scales,
                     s.bind_face, s.bind_bary)
    off = ot["means"].astype(np.float64) - s.means.astype(np.float64)
    px = [(x, y) for y in range(cam.height) for x in range(cam.width)]
    fr = OR.Frame(cam, ot["means"], s.opacity, s.sh, 0, s.tri_xyz, s.tri_rgb, s.tri_alpha, cov3d=ot["cov3d"])
    rng = np.random.default_rng(13)
    dL = mask_ambiguous(fr, px, rng.normal(size=(len(px), 3)))
    ref = OG.gradients(cam, px, dL, s.means, s.scales, s.quats, s.opacity, s.sh, 0, s.tri_xyz,
                       s.tri_rgb, s.tri_alpha, xform=ot["A"], mean_offset=off)
    r = Rasterizer("cuda:0")
    r.set_proxy(s.proxy.V_rest, s.proxy.faces)
    dev = torch.device("cuda:0")
    t = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev, requires_grad=True)
    P = [t(s.means), t(s.scales), t(s.quats), t(s.opacity), t(s.sh)]
    img = render_differentiable(r, [cam], *P, tri_xyz=s.tri_xyz, tri_rgb=s.tri_rgb,
                                tri_alpha=s.tri_alpha,
                                deform=dict(V_def=s.proxy.V_def, bind_face=s.bind_face,
                                            bind_bary=s.bind_bary))
    W, H = cam.width, cam.height
    w = torch.tensor(dL.reshape(H, W, 3).transpose(2, 0, 1).reshape(-1), dtype=torch.float32, device=dev)
    (img * w).sum().backward()
    for n, p in zip(NAMES, P):
        assert_close(p.grad.cpu().numpy(), ref[n], n)


def test_backward_requires_a_blended_frame(gpu):
    import torch
    from paper_2601_19233_amd import _lib as L
    from paper_2601_19233_amd.render import Rasterizer
    r = Rasterizer("cuda:0")
    z = torch.zeros(12, device="cuda:0")
    with pytest.raises(L.UmgsError) as e:
        r.backward(z, dict(image=z, T_final=z, n_contrib=z.int(), T_entity_in=z), z, z, z, z)
    assert e.value.status == -4
    r2 = Rasterizer("cuda:0", mode=2)
    cam = scenes.look_at((0, 0, 3), 4, 3)
    out = r2.render([cam])
    with pytest.raises(L.UmgsError) as e:
        r2.backward(torch.zeros(36, device="cuda:0"), out, z, z, z, z)
    assert e.value.status == -5
