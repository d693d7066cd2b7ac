"""Triangle appearance gradients on the GPU (umgs_backward_triangles through
the C ABI) against the FP64 gradient oracle: per-vertex colours and opacity
attributes, through the sub-sample entity blend and the direct blend.

Tolerance: 1e-3 relative per element with an absolute floor of 1e-5 times
the largest magnitude of the same array (FP32 sums over many pixels against
FP64).  Pixels holding a near-threshold decision get zero loss weight on
both sides (coverage decisions are exact integers on both sides)."""
import sys

import numpy as np
import pytest

from oracle import grad as OG
from oracle import render as OR
from paper_2601_19233_amd import scenes
from tests.test_gpu_backward import assert_close, mask_ambiguous
from tests.test_oracle_grad import mixed_scene

pytestmark = pytest.mark.gpu
BG = (0.1, 0.2, 0.3)


def note(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def f32(a):
    return np.ascontiguousarray(a, np.float32)


def gpu_tri_grads(cams, scene, dLs, mode=0, tile=(16, 16), uv=None, tex=None, twice=False,
                  inspect=None):
    """Render the views in one frame, run the triangle backward with the
    per-view loss weights dLs[v] ((H*W, 3) row-major pixels), return numpy
    gradients; inspect(r, out) sees the rasterizer and the frame first."""
    import torch
    from paper_2601_19233_amd.render import Rasterizer
    means, scales, quats, opac, sh, deg, xyz, rgb, al = scene
    T = xyz.shape[0]
    r = Rasterizer("cuda:0", sh_degree=deg, mode=mode, bg=BG, tile=tile)
    if tex is not None:
        r.set_texture(tex, uv)
    out = r.render(list(cams), means=f32(means), scales=f32(scales), quats=f32(quats),
                   opacity=f32(opac), sh=f32(sh).reshape(sh.shape[0], -1), tri_xyz=f32(xyz).reshape(T, 9),
                   tri_rgb=f32(rgb).reshape(T, 9), tri_alpha=f32(al))
    flat = np.concatenate([np.ascontiguousarray(d.T).reshape(-1) for d in dLs]).astype(np.float32)
    dLt = torch.from_numpy(flat).cuda()
    if inspect is not None:
        inspect(r, out)
    g = r.backward_triangles(dLt, out)
    if twice:
        g = r.backward_triangles(dLt, out, out=g, accumulate=True)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}
    r.close()
    return res


def oracle_tri_grads(cam, scene, dL, mode=0, uv=None, tex=None):
    means, scales, quats, opac, sh, deg, xyz, rgb, al = scene
    px = [(x, y) for y in range(cam.height) for x in range(cam.width)]
    return OG.gradients(cam, px, dL, means, scales, quats, opac, sh, deg, xyz, rgb, al, bg=BG,
                        mode=mode, tri_uv=uv, tex=tex)


def masked_loss(cam, scene, seed, mode=0, uv=None, tex=None):
    means, scales, quats, opac, sh, deg, xyz, rgb, al = scene
    fr = OR.Frame(cam, means, opac, sh, deg, xyz, rgb, al, scales=scales, quats=quats, bg=BG,
                  mode=mode, tri_uv=uv, tex=tex)
    px = [(x, y) for y in range(cam.height) for x in range(cam.width)]
    return mask_ambiguous(fr, px, np.random.default_rng(seed).normal(size=(len(px), 3)))


def f32_scene(seed, W=24, H=20, deg=0):
    cam, means, scales, quats, opac, sh, xyz, rgb, al = mixed_scene(seed, W=W, H=H, degree=deg)
    return cam, [f32(means), f32(scales), f32(quats), f32(opac), f32(sh), deg, f32(xyz), f32(rgb), f32(al)]


def check(g, ref):
    assert np.abs(ref["tri_rgb"]).max() > 0 and np.abs(ref["tri_alpha"]).max() > 0
    assert_close(g["tri_rgb"], ref["tri_rgb"], "tri_rgb")
    assert_close(g["tri_alpha"], ref["tri_alpha"], "tri_alpha")


@pytest.mark.parametrize("mode,seed,tile", [(0, 2, (16, 16)), (1, 2, (16, 16)), (0, 3, (8, 8)),
                                            (0, 5, (32, 8))])
def test_triangle_gradients_match_oracle(gpu, mode, seed, tile):
    cam, sc = f32_scene(seed)
    note(f"triangle backward mode={mode} seed={seed} tile={tile}")
    dL = masked_loss(cam, sc, 20 + seed, mode)
    ref = oracle_tri_grads(cam, sc, dL, mode)
    g = gpu_tri_grads([cam], sc, [dL], mode, tile)
    check(g, ref)


@pytest.mark.parametrize("hi", [1.0, 0.97])
def test_opaque_and_stacked_triangles(gpu, hi):
    """Opaque triangles (a sub-sample's transmittance drops to exactly zero)
    in front of and behind translucent ones: the linear re-walk counts the
    zero factors.  With alpha 0.97 instead, factors of 0.03 send those
    entities to the quadratic re-walk."""
    cam, sc = f32_scene(6)
    al = sc[8].copy()
    al[:2] = hi
    al[2::3] = 0.6
    sc[8] = al
    note(f"triangle backward opaque/stacked hi={hi}")
    dL = masked_loss(cam, sc, 31)
    ref = oracle_tri_grads(cam, sc, dL)
    g = gpu_tri_grads([cam], sc, [dL])
    check(g, ref)


def test_textured_triangle_gradients(gpu):
    cam, sc = f32_scene(7)
    rng = np.random.default_rng(9)
    tex = rng.uniform(0.1, 1.0, size=(5, 7, 4)).astype(np.float32)
    uv = rng.uniform(-0.1, 1.1, size=(sc[6].shape[0], 3, 2)).astype(np.float32)
    note("triangle backward textured")
    dL = masked_loss(cam, sc, 32, uv=uv, tex=tex)
    ref = oracle_tri_grads(cam, sc, dL, uv=uv, tex=tex)
    g = gpu_tri_grads([cam], sc, [dL], uv=uv, tex=tex)
    check(g, ref)


def test_two_views_sum_and_accumulate(gpu):
    """Gradients of a two-view frame are the sums of the views' gradients;
    accumulate=1 adds to the outputs."""
    cam, sc = f32_scene(2)
    cam2 = scenes.look_at((-0.3, 0.2, 2.0), 20, 16)
    note("triangle backward two views")
    dL1 = masked_loss(cam, sc, 40)
    dL2 = masked_loss(cam2, sc, 41)
    r1 = oracle_tri_grads(cam, sc, dL1)
    r2 = oracle_tri_grads(cam2, sc, dL2)
    ref = {k: r1[k] + r2[k] for k in ("tri_rgb", "tri_alpha")}
    g = gpu_tri_grads([cam, cam2], sc, [dL1, dL2])
    check(g, ref)
    g2 = gpu_tri_grads([cam, cam2], sc, [dL1, dL2], twice=True)
    check(g2, {k: 2 * v for k, v in ref.items()})


def test_dense_mesh_overflows_the_tile_table(gpu):
    """More than 512 triangle fragments in one tile's list (a fine, faint
    sphere seen small, so no pixel stops early): the triangles past the LDS
    table add straight to global memory, and entities of many triangles
    spread over long list spans.  16x16 pixels, 8x8 tiles."""
    rng = np.random.default_rng(3)
    V, F = scenes.icosphere(16, 0.5)                # 5,120 faces
    xyz = V[F].astype(np.float32)
    T = xyz.shape[0]
    rgb = rng.uniform(0, 1, size=(T, 3, 3)).astype(np.float32)
    al = rng.uniform(0.05, 0.3, size=T).astype(np.float32)
    n = 40
    means = rng.uniform(-0.6, 0.6, size=(n, 3)).astype(np.float32)
    s, q, o, sh = scenes._gaussian_stats(rng, n, 0)
    sc = [means, f32(s), f32(q), f32(o), f32(sh), 0, xyz, rgb, al]
    cam = scenes.look_at((0.0, 0.0, 3.0), 16, 16)
    note(f"triangle backward dense mesh T={T}")
    dL = masked_loss(cam, sc, 50)
    ref = oracle_tri_grads(cam, sc, dL)
    seen = {}

    def count(r, out):
        # triangle fragments each tile's walk covers (positions below its
        # largest last-blended position)
        from paper_2601_19233_amd import _lib as L
        rg = r.copy_state(L.STATE_RANGES).long().view(-1, 2).cpu().numpy()
        vals = (r.copy_state(L.STATE_SORTED_VALS).long() & 0xFFFFFFFF).cpu().numpy()
        nc = out["n_contrib"].cpu().numpy().reshape(16, 16)
        best = 0
        for t in range(rg.shape[0]):
            ty, tx = divmod(t, 2)
            m = int(nc[8 * ty:8 * ty + 8, 8 * tx:8 * tx + 8].max())
            best = max(best, int(((vals[rg[t, 0]:rg[t, 0] + m] % (n + T)) >= n).sum()))
        seen["max"] = best

    g = gpu_tri_grads([cam], sc, [dL], tile=(8, 8), inspect=count)
    note(f"dense mesh: up to {seen['max']} triangle fragments in one tile's walk")
    assert seen["max"] > 512
    check(g, ref)
