"""Gradients with respect to the deformed proxy (umgs_backward_transfer, and
dL/dA from umgs_backward) on the GPU against the FP64 oracles.

* The transfer backward alone, from random dL/dmu' and dL/dA, against
  oracle/transfer_grad.py (K = 8 and K = 1, unbound corners, rotations up to
  about a radian and uneven stretches).
* The whole chain on a deformed scene through the autograd wrapper: the
  Gaussian backward's dL/dA against the gradient oracle's, and dL/dV' of
  the rendered loss against the transfer gradient oracle fed with the
  gradient oracle's dL/dmu and dL/dA; the triangles' colour and opacity
  gradients of the same loss against the gradient oracle's.

Tolerance: 1e-3 relative per element with an absolute floor of 1e-5 times
the largest magnitude of the same array, as for the other gradients.
"""
import sys

import numpy as np
import pytest

from oracle import grad as OG
from oracle import render as OR
from oracle import transfer as OT
from oracle import transfer_grad as TG
from paper_2601_19233_amd import scenes
from tests.test_gpu_backward import assert_close, mask_ambiguous
from tests.test_oracle_transfer_grad import deformed_proxy

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("K,seed", [(8, 2), (1, 3), (8, 9)])
def test_transfer_backward_matches_oracle(gpu, K, seed):
    import torch
    from paper_2601_19233_amd.render import Rasterizer
    V, F, Vd, mu, q, sc, bf, bb = deformed_proxy(seed, n=300, K=K)
    rng = np.random.default_rng(seed + 100)
    N = mu.shape[0]
    gm = rng.normal(size=(N, 3)).astype(np.float32)
    gA = rng.normal(size=(N, 3, 3)).astype(np.float32)
    note(f"transfer backward K={K} N={N} nV={V.shape[0]}")
    ref = TG.proxy_gradient(V, F, Vd, mu, bf, bb, gm.astype(np.float64), gA.astype(np.float64))
    r = Rasterizer("cuda:0", k_bind=K)
    r.set_proxy(V, F)
    dev = torch.device("cuda:0")
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    face = torch.from_numpy(np.ascontiguousarray(bf, np.int32)).to(dev)
    g = r.backward_transfer(f(Vd), face, f(bb), f(gm), f(gA.reshape(N, 9)))
    # accumulate adds, NULL gradients count as zero
    g2 = r.backward_transfer(f(Vd), face, f(bb), None, None, out=g.clone(), accumulate=True)
    torch.cuda.synchronize()
    gn = g.cpu().numpy().astype(np.float64)
    assert np.abs(ref).max() > 0
    assert_close(gn, ref, "dL/dV_def")
    assert torch.equal(g2, g)
    # the mean gradient alone: the vertices' gradients sum to the bound means'
    gm_only = r.backward_transfer(f(Vd), face, f(bb), f(gm), None).cpu().numpy().astype(np.float64)
    anyb = OT.bound_mask(bf, F.shape[0]).any(1)
    np.testing.assert_allclose(gm_only.sum(0), gm[anyb].astype(np.float64).sum(0), rtol=1e-4, atol=1e-3)
    r.close()


def test_transfer_backward_requires_a_proxy(gpu):
    import torch
    from paper_2601_19233_amd import _lib as L
    from paper_2601_19233_amd.render import Rasterizer
    r = Rasterizer("cuda:0")
    z = torch.zeros(9, device="cuda:0")
    with pytest.raises(L.UmgsError) as e:
        r.backward_transfer(z, torch.zeros((1, 8), dtype=torch.int32, device="cuda:0"),
                            torch.zeros((1, 8, 2), device="cuda:0"))
    assert "proxy" in str(e.value)
    r.close()


def test_deformed_chain_gradients_match_oracle(gpu):
    """Deformed scene rendered through the autograd wrapper with V', the
    triangles' colours and their opacities requiring gradients."""
    import torch
    from paper_2601_19233_amd.render import Rasterizer, render_differentiable
    s = scenes.make_config(1, scale=0.003, res_scale=0.025)
    cam = s.cams[0]
    note(f"deformed chain N={s.N} T={s.T} nV={s.proxy.V_rest.shape[0]} {cam.width}x{cam.height}")
    ot = OT.transfer(s.proxy.V_rest, s.proxy.faces, s.proxy.V_def, s.means, s.quats, s.scales,
                     s.bind_face, s.bind_bary)
    off = ot["means"].astype(np.float64) - s.means.astype(np.float64)
    px = [(x, y) for y in range(cam.height) for x in range(cam.width)]
    fr = OR.Frame(cam, ot["means"], s.opacity, s.sh, 0, s.tri_xyz, s.tri_rgb, s.tri_alpha,
                  cov3d=ot["cov3d"])
    dL = mask_ambiguous(fr, px, np.random.default_rng(17).normal(size=(len(px), 3)))
    ref = OG.gradients(cam, px, dL, s.means, s.scales, s.quats, s.opacity, s.sh, 0, s.tri_xyz,
                       s.tri_rgb, s.tri_alpha, xform=ot["A"], mean_offset=off)
    refV = TG.proxy_gradient(s.proxy.V_rest, s.proxy.faces, s.proxy.V_def, s.means, s.bind_face,
                             s.bind_bary, ref["means"], ref["xform"])
    r = Rasterizer("cuda:0")
    r.set_proxy(s.proxy.V_rest, s.proxy.faces)
    dev = torch.device("cuda:0")
    t = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev, requires_grad=True)
    P = [t(s.means), t(s.scales), t(s.quats), t(s.opacity), t(s.sh)]
    Vd = t(s.proxy.V_def)
    trgb, tal = t(s.tri_rgb), t(s.tri_alpha)
    img = render_differentiable(r, [cam], *P, tri_xyz=s.tri_xyz, tri_rgb=trgb, tri_alpha=tal,
                                deform=dict(V_def=Vd, bind_face=s.bind_face, bind_bary=s.bind_bary))
    W, H = cam.width, cam.height
    w = torch.tensor(dL.reshape(H, W, 3).transpose(2, 0, 1).reshape(-1), dtype=torch.float32, device=dev)
    (img * w).sum().backward()
    assert np.abs(refV).max() > 0
    assert_close(Vd.grad.cpu().numpy(), refV, "dL/dV_def")
    assert_close(trgb.grad.cpu().numpy(), ref["tri_rgb"], "tri_rgb")
    assert_close(tal.grad.cpu().numpy(), ref["tri_alpha"], "tri_alpha")
    for n, p in zip(("means", "scales", "quats", "opacity", "sh"), P):
        assert_close(p.grad.cpu().numpy(), ref[n], n)
    r.close()


def test_backward_writes_the_transfer_map_gradient(gpu):
    """umgs_backward's dL/dA on a deformed scaled workload against the
    gradient oracle's."""
    import torch
    from paper_2601_19233_amd.render import Rasterizer
    s = scenes.make_config(1, scale=0.0008, res_scale=0.02)
    cam = s.cams[0]
    ot = OT.transfer(s.proxy.V_rest, s.proxy.faces, s.proxy.V_def, s.means, s.quats, s.scales,
                     s.bind_face, s.bind_bary)
    off = ot["means"].astype(np.float64) - s.means.astype(np.float64)
    px = [(x, y) for y in range(cam.height) for x in range(cam.width)]
    fr = OR.Frame(cam, ot["means"], s.opacity, s.sh, 0, s.tri_xyz, s.tri_rgb, s.tri_alpha,
                  cov3d=ot["cov3d"])
    dL = mask_ambiguous(fr, px, np.random.default_rng(18).normal(size=(len(px), 3)))
    ref = OG.gradients(cam, px, dL, s.means, s.scales, s.quats, s.opacity, s.sh, 0, s.tri_xyz,
                       s.tri_rgb, s.tri_alpha, xform=ot["A"], mean_offset=off)
    note(f"backward dL/dA N={s.N}")
    r = Rasterizer("cuda:0")
    r.set_proxy(s.proxy.V_rest, s.proxy.faces)
    dev = torch.device("cuda:0")
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    dt = r.bind_transfer(f(s.proxy.V_def), torch.from_numpy(s.bind_face.astype(np.int32)).to(dev),
                         f(s.bind_bary), f(s.means), f(s.quats), f(s.scales))
    out = r.render([cam], means=dt["means"], cov3d=dt["cov3d"], opacity=f(s.opacity),
                   sh=f(s.sh.reshape(s.N, -1)), tri_xyz=f(s.tri_xyz.reshape(s.T, 9)),
                   tri_rgb=f(s.tri_rgb.reshape(s.T, 9)), tri_alpha=f(s.tri_alpha))
    W, H = cam.width, cam.height
    w = torch.tensor(dL.reshape(H, W, 3).transpose(2, 0, 1).reshape(-1), dtype=torch.float32, device=dev)
    g = r.backward(w, out, dt["means"], f(s.scales), f(s.quats), f(s.sh.reshape(s.N, -1)), dt["xform"])
    torch.cuda.synchronize()
    assert_close(g["xform"].cpu().numpy().reshape(-1, 3, 3), ref["xform"], "dL/dA")
    assert_close(g["means"].cpu().numpy(), ref["means"], "means")
    r.close()
