"""Textured triangles on the GPU (umgs_set_texture) against the oracle's
textured shading: per-vertex texture coordinates interpolated perspective-
correctly at the pixel centre, a bilinear RGBA fetch clamped to the edge,
colour x texel RGB and opacity x texel alpha.  Every pixel of a small view
within 1e-4 (the last blended fragment's id exact); a white texture changes
no bit of the untextured frame; batched views equal single views; Gaussian
gradients with textured occluders against the oracle gradient."""
import sys

import numpy as np
import pytest

from oracle import grad as OG
from oracle import render as OR
from paper_2601_19233_amd import scenes
from tests import _parity as PT

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def textured(seed, T, w=37, h=23):
    rng = np.random.default_rng(seed)
    tex = rng.uniform(0, 1, size=(h, w, 4)).astype(np.float32)
    tex[..., 3] = rng.uniform(0.3, 1.0, size=(h, w))
    tex[: h // 3, :, 3] = 1.0                      # an opaque band (stops inside the texture)
    uv = rng.uniform(-0.2, 1.2, size=(T, 3, 2)).astype(np.float32)
    return tex, uv


def oracle_frame(s, cam, uv, tex, bg=(0.0, 0.0, 0.0)):
    return OR.Frame(cam, s.means, s.opacity, s.sh, s.sh_degree, s.tri_xyz, s.tri_rgb, s.tri_alpha,
                    scales=s.scales, quats=s.quats, bg=bg, tri_uv=uv, tex=tex)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_textured_frame_parity(gpu, tile):
    import torch
    from paper_2601_19233_amd.render import Rasterizer, scene_inputs
    from tests.test_gpu_forward import last_gids, view_arrays
    s = scenes.make_config(0)
    tex, uv = textured(1, s.T)
    cam = s.cams[0]
    note(f"textured frame tile={tile} T={s.T} tex={tex.shape}")
    r = Rasterizer("cuda:0", tile=tile, bg=(0.2, 0.1, 0.3))
    r.set_texture(tex, uv)
    out = r.render([cam], **scene_inputs(s))
    torch.cuda.synchronize()
    img, Tf, nc = view_arrays(r, out)
    fr = oracle_frame(s, cam, uv, tex, bg=(0.2, 0.1, 0.3))
    px = [(x, y) for y in range(cam.height) for x in range(cam.width)]
    res = PT.compare_pixels(fr, img, Tf, last_gids(r, nc), px)
    note(f"textured tile={tile}: {res}")
    r.close()


def test_white_texture_changes_no_bit(gpu):
    import torch
    from paper_2601_19233_amd.render import Rasterizer, scene_inputs
    s = scenes.make_config(0)
    _, uv = textured(2, s.T)
    r = Rasterizer("cuda:0")
    plain = {k: v.clone() for k, v in r.render(s.cams, **scene_inputs(s)).items()}
    r.set_texture(np.ones((5, 9, 4), np.float32), uv)
    tx = r.render(s.cams, **scene_inputs(s))
    torch.cuda.synchronize()
    for k in ("image", "T_final", "n_contrib", "T_entity_in"):
        assert torch.equal(plain[k], tx[k]), k
    # removing the texture returns to untextured shading; a count mismatch is refused
    r.set_texture(None)
    again = r.render(s.cams, **scene_inputs(s))
    assert torch.equal(plain["image"], again["image"])
    from paper_2601_19233_amd import _lib as L
    r.set_texture(np.ones((2, 2, 4), np.float32), uv[:-1])
    with pytest.raises(L.UmgsError) as e:
        r.render(s.cams, **scene_inputs(s))
    assert e.value.status == -1
    r.close()


def test_textured_batched_views_match_single_views(gpu):
    import torch
    from paper_2601_19233_amd.render import Rasterizer, scene_inputs
    s = scenes.make_config(3, scale=0.004, res_scale=0.08, n_views=4)
    tex, uv = textured(3, s.T, 64, 40)
    note(f"textured batched {[(c.width, c.height) for c in s.cams]}")
    r = Rasterizer("cuda:0", schedule=1)
    r.set_texture(tex, uv)
    allv = r.render(s.cams, **scene_inputs(s))
    imgs = [t.clone() for t in r.split_views(allv["image"], 3)]
    r1 = Rasterizer("cuda:0")
    r1.set_texture(tex, uv)
    for v, c in enumerate(s.cams):
        one = r1.render([c], **scene_inputs(s))
        assert torch.equal(one["image"].view_as(imgs[v]), imgs[v]), v
    cam = s.cams[1]
    fr = oracle_frame(s, cam, uv, tex)
    img = imgs[1].cpu().numpy()
    Tf = r.split_views(allv["T_final"], 1)[1].cpu().numpy()
    rng = np.random.default_rng(5)
    px = list(zip(rng.integers(0, cam.width, 60).tolist(), rng.integers(0, cam.height, 60).tolist()))
    note(f"textured batched view 1: {PT.compare_pixels(fr, img, Tf, None, px)}")
    r.close()
    r1.close()


def test_textured_backward_matches_oracle_gradient(gpu):
    """Gaussian gradients through textured semi-transparent occluders."""
    import torch
    from paper_2601_19233_amd.render import Rasterizer
    from tests.test_gpu_backward import assert_close, mask_ambiguous
    from tests.test_oracle_grad import mixed_scene
    cam, means, scales, quats, opac, sh, xyz, rgb, al = mixed_scene(2, W=24, H=20)
    f32 = lambda a: np.asarray(a, np.float32)
    means, scales, quats, opac, sh = (f32(a) for a in (means, scales, quats, opac, sh))
    tex, uv = textured(4, xyz.shape[0], 6, 5)
    bg = (0.1, 0.2, 0.3)
    px = [(x, y) for y in range(cam.height) for x in range(cam.width)]
    fr = OR.Frame(cam, means, opac, sh, 0, xyz, rgb, al, scales=scales, quats=quats, bg=bg,
                  tri_uv=uv, tex=tex)
    rng = np.random.default_rng(11)
    W, H = cam.width, cam.height
    dL = mask_ambiguous(fr, px, rng.normal(size=(W * H, 3)))
    ref = OG.gradients(cam, px, dL, means, scales, quats, opac, sh, 0, xyz, rgb, al, bg=bg,
                       tri_uv=uv, tex=tex)
    note("textured backward")
    r = Rasterizer("cuda:0", bg=bg)
    r.set_texture(tex, uv)
    T = xyz.shape[0]
    out = r.render([cam], means=means, scales=scales, quats=quats, opacity=opac,
                   sh=sh.reshape(sh.shape[0], -1), tri_xyz=xyz.reshape(T, 9),
                   tri_rgb=rgb.reshape(T, 9), tri_alpha=al)
    dLt = torch.from_numpy(np.ascontiguousarray(dL.reshape(H, W, 3).transpose(2, 0, 1).reshape(-1),
                                                np.float32)).cuda()
    g = r.backward(dLt, out, means, scales, quats, sh.reshape(sh.shape[0], -1))
    torch.cuda.synchronize()
    for n in ("means", "scales", "quats", "opacity", "sh"):
        assert_close(g[n].cpu().numpy(), ref[n], n)
    r.close()
