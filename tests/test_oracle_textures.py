"""Pins of the oracle's textured triangles (the paper's Section 1: an opacity
attribute on textured meshes; colour = vertex colour x texel RGB, opacity =
attribute x texel alpha, texture coordinates interpolated perspective-
correctly like the colour and sampled bilinearly, clamped to the edge).

Each test checks the oracle against something it does not compute itself:
a constant texture reduces to the untextured renderer; a pixel centre that
maps to a texel centre returns that texel; a linear ramp texture returns
the texture coordinate of the ray-plane hit computed from the geometry
(perspective correctness, the half-texel convention and the bilinear
weights at once); the clamp; and the closed form of two stacked textured
triangles with per-texel opacity.
"""
import numpy as np
import pytest

from oracle import render as R
from paper_2601_19233_amd import scenes
from tests.test_oracle_pins import single_gaussian

F32 = np.float32


def tri_at_pixels(cam, pix, depth):
    """World vertices of a triangle whose vertices project to the pixel
    coordinates pix (3, 2) at camera depth ``depth`` (constant depth)."""
    R_ = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)
    pts = []
    for u, v in pix:
        pc = np.array([(u - cam.cx) * depth / cam.fx, (v - cam.cy) * depth / cam.fy, depth])
        pts.append(R_.T @ (pc - t))
    return np.array(pts)


def textured_frame(cam, xyz, rgb, alpha, uv, tex, **kw):
    """Oracle frame of textured triangles only."""
    return R.Frame(cam, np.zeros((0, 3), F32), np.zeros((0,), F32), np.zeros((0, 1, 3), F32), 0,
                   np.asarray(xyz, F32).reshape(-1, 3, 3), np.asarray(rgb, F32).reshape(-1, 3, 3),
                   np.asarray(alpha, F32).reshape(-1), scales=np.zeros((0, 3), F32),
                   quats=np.zeros((0, 4), F32), tri_uv=np.asarray(uv, F32), tex=tex, **kw)


def mixed_textured_scene(seed):
    s = scenes.make_config(0, scale=0.1, res_scale=0.4, seed=seed)
    rng = np.random.default_rng(seed)
    uv = rng.uniform(-0.2, 1.2, size=(s.T, 3, 2)).astype(F32)
    return s, uv


def test_constant_texture_reduces_to_untextured():
    """A texture whose texels are all (1, 1, 1, 1) changes nothing, exactly:
    every pixel of a mixed scene (Gaussians, an icosphere, the
    semi-transparent quad) equals the untextured render bit for bit."""
    s, uv = mixed_textured_scene(3)
    cam = s.cams[0]
    tex = np.ones((5, 7, 4), F32)
    kw = dict(scales=s.scales, quats=s.quats, bg=(0.2, 0.3, 0.4))
    a = R.Frame(cam, s.means, s.opacity, s.sh, 0, s.tri_xyz, s.tri_rgb, s.tri_alpha, **kw)
    b = R.Frame(cam, s.means, s.opacity, s.sh, 0, s.tri_xyz, s.tri_rgb, s.tri_alpha, **kw,
                tri_uv=uv, tex=tex)
    n_tri = 0
    for y in range(cam.height):
        for x in range(cam.width):
            ra, rb = a.pixel(x, y), b.pixel(x, y)
            assert np.array_equal(ra.C, rb.C) and ra.T == rb.T and ra.order == rb.order
            n_tri += any(g >= s.N for g in ra.order)
    assert n_tri > 30


def test_texel_centre_returns_the_texel():
    """A fronto-parallel opaque triangle with white vertex colours whose
    texture coordinates are u = x / 8, v = y / 8 in pixel units: the centre
    of pixel (x, y) maps to the centre of texel (x, y) of an 8 x 8 texture,
    so the pixel shows that texel's colour, blended with its alpha."""
    cam = scenes.look_at((0.0, 0.0, 3.0), 8, 8)
    rng = np.random.default_rng(4)
    tex = rng.uniform(0, 1, size=(8, 8, 4)).astype(F32)
    tex[..., 3] = np.where(rng.uniform(size=(8, 8)) < 0.5, 1.0, tex[..., 3])
    pix = np.array([[-64.0, -64.0], [192.0, -64.0], [-64.0, 192.0]])
    xyz = tri_at_pixels(cam, pix, 2.0)
    uv = pix / 8.0
    bg = np.array([0.1, 0.7, 0.3])
    fr = textured_frame(cam, xyz, np.ones((3, 3)), [1.0], uv[None], tex, bg=tuple(bg))
    for y in range(8):
        for x in range(8):
            r = fr.pixel(x, y)
            t = tex[y, x].astype(np.float64)
            np.testing.assert_allclose(r.C, t[3] * t[:3] + (1 - t[3]) * bg, rtol=0, atol=1e-12)
            assert abs(r.T - (1 - t[3])) < 1e-12


def test_ramp_texture_returns_the_ray_plane_hit_coordinates():
    """An oblique triangle textured with a linear ramp (texel (i, j) holds
    ((i + 1/2) / W, (j + 1/2) / H)): bilinear sampling reproduces a linear
    function, so the colour at each covered pixel centre is the texture
    coordinate of the point where the pixel's ray hits the triangle's plane
    (barycentrics of that 3D point, computed here from the geometry), up to
    the clamp at the edge texels."""
    cam = scenes.look_at((0.3, -0.2, 3.0), 24, 20)
    W, H = 16, 12
    ii, jj = np.meshgrid(np.arange(W), np.arange(H))
    tex = np.stack([(ii + 0.5) / W, (jj + 0.5) / H, np.zeros_like(ii, float), np.ones_like(ii, float)],
                   -1).astype(F32)
    xyz = np.array([[-1.3, -1.1, 0.4], [1.4, -0.9, -0.6], [0.1, 1.5, 0.2]])
    uv = np.array([[0.05, 0.1], [0.97, 0.2], [0.4, 0.93]], F32)
    fr = textured_frame(cam, xyz, np.ones((3, 3)), [1.0], uv[None], tex)
    P = xyz.astype(F32).astype(np.float64)
    n = np.cross(P[1] - P[0], P[2] - P[0])
    o = -(cam.R.astype(F32).astype(np.float64).T @ cam.t.astype(F32).astype(np.float64))
    checked = 0
    for y in range(cam.height):
        for x in range(cam.width):
            r = fr.pixel(x, y)
            if r.order != [0] or r.T != 0.0:
                continue          # not covered, or not all four sub-samples (opaque: T = 1 - O)
            d = cam.R.astype(F32).astype(np.float64).T @ np.array(
                [(x + 0.5 - float(F32(cam.cx))) / float(F32(cam.fx)),
                 (y + 0.5 - float(F32(cam.cy))) / float(F32(cam.fy)), 1.0])
            X = o + d * np.dot(P[0] - o, n) / np.dot(d, n)
            a0 = np.dot(np.cross(P[1] - X, P[2] - X), n) / np.dot(n, n)
            a1 = np.dot(np.cross(P[2] - X, P[0] - X), n) / np.dot(n, n)
            if min(a0, a1, 1 - a0 - a1) < 0.02:
                continue          # the oracle clamps barycentrics of edge pixels
            want = a0 * uv[0] + a1 * uv[1] + (1 - a0 - a1) * uv[2]
            want = np.clip(want, [0.5 / W, 0.5 / H], [1 - 0.5 / W, 1 - 0.5 / H])
            np.testing.assert_allclose(r.C[:2], want, rtol=0, atol=2e-3)
            checked += 1
    assert checked > 60


def test_bilinear_weights_and_edge_clamp():
    """texture_sample against a hand evaluation: the four texels around the
    sample point weighted by the distances to their centres; outside [0, 1]
    the edge texels are repeated."""
    rng = np.random.default_rng(9)
    tex = rng.uniform(0, 1, size=(3, 4, 4)).astype(F32)
    t64 = tex.astype(np.float64)
    # between texel centres (1, 0), (2, 0), (1, 1), (2, 1): x = 1.25, y = 0.75
    uv = np.array([[(1.25 + 0.5) / 4, (0.75 + 0.5) / 3]])
    want = (0.75 * 0.25 * t64[0, 1] + 0.25 * 0.25 * t64[0, 2] + 0.75 * 0.75 * t64[1, 1]
            + 0.25 * 0.75 * t64[1, 2])
    np.testing.assert_allclose(R.texture_sample(tex, uv)[0], want, rtol=0, atol=1e-15)
    # clamped: far left / far below repeat column 0 / row 2
    np.testing.assert_allclose(R.texture_sample(tex, np.array([[-3.0, (1 + 0.5) / 3]]))[0], t64[1, 0],
                               atol=1e-15)
    np.testing.assert_allclose(R.texture_sample(tex, np.array([[(3 + 0.5) / 4, 5.0]]))[0], t64[2, 3],
                               atol=1e-15)


def test_per_texel_opacity_in_an_entity_closed_form():
    """Two full-coverage textured triangles, one texel each (textures of a
    single colour), attributes a1, a2 and texel alphas b1, b2, a Gaussian
    behind both: the entity blends C = A1 c1 + (1 - A1) A2 c2 +
    (1 - A1)(1 - A2) aG cG with A = a b, texel colours multiplying the
    white vertex colours."""
    W = H = 33
    cam = scenes.look_at((0.0, 0.0, 3.0), W, H)
    cam.cx = cam.cy = 16.5
    big = np.array([[-10.0, -10.0], [10.0, -10.0], [0.0, 10.0]])
    x1 = np.array([[-10.0, -10.0, 1.0], [10.0, -10.0, 1.0], [0.0, 10.0, 1.0]])
    x2 = x1.copy()
    x2[:, 2] = 0.5
    tex = np.zeros((1, 2, 4), F32)
    tex[0, 0] = [0.9, 0.2, 0.1, 0.6]
    tex[0, 1] = [0.1, 0.3, 0.8, 0.5]
    # texture coordinates fixed at each texel's centre (one texel per triangle)
    uv = np.array([[[0.25, 0.5]] * 3, [[0.75, 0.5]] * 3], F32)
    a1, a2 = 0.8, 0.7
    g = single_gaussian(-1.0, 0.6, [0.2, 0.9, 0.4], 0.05, cam)
    fr = R.Frame(cam, g["means"], g["opac"], g["sh"], 0, np.stack([x1, x2]).astype(F32),
                 np.ones((2, 3, 3), F32), np.array([a1, a2], F32), scales=g["scales"],
                 quats=g["quats"], tri_uv=uv, tex=tex)
    r = fr.pixel(16, 16)
    assert r.order == [1, 2, 0]
    t = tex.astype(np.float64)[0]
    A1, A2 = float(F32(a1)) * t[0, 3], float(F32(a2)) * t[1, 3]
    gp = R.project_gaussians(cam, g["means"], g["opac"], g["sh"], 0, g["scales"], g["quats"])
    aG = min(0.99, float(g["opac"][0]))
    want = A1 * t[0, :3] + (1 - A1) * A2 * t[1, :3] + (1 - A1) * (1 - A2) * aG * gp.rgb[0]
    np.testing.assert_allclose(r.C, want, rtol=0, atol=1e-9)
    assert abs(r.T - (1 - A1) * (1 - A2) * (1 - aG)) < 1e-9


def test_gradient_oracle_with_textured_occluders_matches_finite_differences():
    """The gradient oracle shades triangles exactly as the forward oracle
    (texel colour and opacity): its Gaussian gradients in a scene with a
    textured semi-transparent quad and sphere match central differences of
    the textured forward oracle."""
    from oracle import grad as OG
    from tests.test_oracle_grad import mixed_scene
    cam, means, scales, quats, opac, sh, xyz, rgb, al = mixed_scene(2)
    rng = np.random.default_rng(17)
    uv = rng.uniform(0, 1, size=(xyz.shape[0], 3, 2)).astype(F32)
    tex = rng.uniform(0.2, 1, size=(6, 5, 4)).astype(F32)
    px = [(x, y) for y in range(cam.height) for x in range(cam.width)]
    w = rng.normal(size=(len(px), 3))
    bg = (0.1, 0.2, 0.3)

    def loss(m, sc, q, o, s_):
        fr = R.Frame(cam, m, o, s_, 0, xyz, rgb, al, scales=sc, quats=q, bg=bg, tri_uv=uv, tex=tex)
        res = [fr.pixel(x, y) for x, y in px]
        return float((np.stack([r.C for r in res]) * w).sum()), [tuple(r.order) for r in res]

    g = OG.gradients(cam, px, w, means, scales, quats, opac, sh, 0, xyz, rgb, al, bg=bg,
                     tri_uv=uv, tex=tex)
    params = [means, scales, quats, opac, sh]
    names = ["means", "scales", "quats", "opacity", "sh"]
    _, sig0 = loss(*params)
    gmax = max(np.abs(g[n]).max() for n in names)
    checked = 0
    for gi in (0, 3, 5):
        for pi, name in enumerate(names):
            for comp in np.ndindex(params[pi].shape[1:]):
                idx = (gi,) + comp
                h = 1e-6 * max(1.0, abs(params[pi][idx]))
                vals, ok = [], True
                for sgn in (1, -1):
                    pp = [p.copy() for p in params]
                    pp[pi][idx] += sgn * h
                    v, sig = loss(*pp)
                    ok &= sig == sig0
                    vals.append(v)
                if not ok:
                    continue
                fd = (vals[0] - vals[1]) / (2 * h)
                assert abs(fd - g[name][idx]) <= 2e-5 * abs(fd) + 1e-7 * gmax, (name, idx)
                checked += 1
    assert checked >= 30
    # the textures matter here: without them the gradient differs
    g0 = OG.gradients(cam, px, w, means, scales, quats, opac, sh, 0, xyz, rgb, al, bg=bg)
    assert np.abs(g0["opacity"] - g["opacity"]).max() > 1e-3 * np.abs(g["opacity"]).max()
