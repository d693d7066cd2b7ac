"""Pins of the forward oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: a library
routine (scipy's spherical harmonics and rotations), a numerical derivative,
a closed-form case of Section 3.2, an invariant, or an independently written
brute-force compositor.  A dropped term, wrong sign or swapped index in the
oracle fails at least one of them.
"""
import math
import struct
from types import SimpleNamespace

import numpy as np
import pytest

from oracle import render as R
from oracle import sh as SH
from paper_2601_19233_amd import scenes

F32 = np.float32


def cam_at(W=32, H=32, eye=(0.0, 0.0, 3.0)):
    return scenes.look_at(eye, W, H)


def empty_tris():
    return np.zeros((0, 3, 3), F32), np.zeros((0, 3, 3), F32), np.zeros((0,), F32)


def no_gauss():
    return (np.zeros((0, 3), F32), np.zeros((0,), F32), np.zeros((0, 1, 3), F32),
            np.zeros((0, 3), F32), np.tile(F32([1, 0, 0, 0]), (0, 1)))


def frame(cam, means=None, opac=None, sh=None, deg=0, scales=None, quats=None,
          tris=None, bg=(0, 0, 0), mode=R.MODE_UNIMGS):
    if means is None:
        means, opac, sh, scales, quats = no_gauss()
    xyz, rgb, al = tris if tris is not None else empty_tris()
    return R.Frame(cam, means, opac, sh, deg, xyz, rgb, al, scales=scales, quats=quats,
                   bg=bg, mode=mode)


def dc_of(rgb):
    """SH DC coefficient giving colour rgb (Y_00 = 1 / (2 sqrt(pi)))."""
    return (np.asarray(rgb, np.float64) - 0.5) * 2.0 * math.sqrt(math.pi)


def pixel_ray_world(cam, px, py):
    """Unit direction in world space of the ray through a pixel centre."""
    u, v = px + 0.5, py + 0.5
    d_cam = np.array([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy, 1.0])
    return cam.R.astype(np.float64).T @ d_cam


# ---------------------------------------------------------------- library pins

def test_sh_basis_matches_scipy():
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(1)
    d = rng.normal(size=(50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(d[:, 2])
    phi = np.arctan2(d[:, 1], d[:, 0])
    B = SH.basis(d, 3)
    k = 0
    for l in range(4):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), theta, phi)
            if m < 0:
                ref = math.sqrt(2) * Y.imag
            elif m == 0:
                ref = Y.real
            else:
                ref = math.sqrt(2) * Y.real
            np.testing.assert_allclose(B[:, k], ref, atol=1e-12, err_msg=f"l={l} m={m}")
            k += 1


def test_sh_basis_orthonormal():
    # Monte Carlo-free check: exact quadrature by a dense Fibonacci sphere
    n = 200000
    i = np.arange(n) + 0.5
    z = 1 - 2 * i / n
    phi = math.pi * (1 + 5 ** 0.5) * i
    r = np.sqrt(1 - z * z)
    d = np.stack([r * np.cos(phi), r * np.sin(phi), z], 1)
    B = SH.basis(d, 3)
    G = B.T @ B * (4 * math.pi / n)
    np.testing.assert_allclose(G, np.eye(16), atol=2e-3)


def test_quat_to_rot_matches_scipy():
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(2)
    q = rng.normal(size=(20, 4))
    Rm = R.quat_to_rot(q)
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    np.testing.assert_allclose(Rm, ref, atol=1e-12)


# ---------------------------------------------------------------- EWA pins

def test_ewa_cov2d_matches_numerical_jacobian():
    rng = np.random.default_rng(3)
    cam = scenes.look_at((0.3, -0.2, 3.0), 64, 48)
    n = 10
    means = rng.uniform(-0.4, 0.4, size=(n, 3)).astype(F32)
    scales = np.exp(rng.normal(-2.5, 0.3, size=(n, 3))).astype(F32)
    q = rng.normal(size=(n, 4)).astype(F32)
    gp = R.project_gaussians(cam, means, np.full(n, 0.5), np.zeros((n, 1, 3)), 0, scales, q)
    W = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)

    def proj(X):
        p = W @ X + t
        return np.array([cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy])

    Sig = R.cov3d_from_scale_rot(scales, q)
    for i in range(n):
        X0 = means[i].astype(np.float64)
        h = 1e-6
        Jw = np.stack([(proj(X0 + h * e) - proj(X0 - h * e)) / (2 * h) for e in np.eye(3)], 1)
        ref = Jw @ Sig[i] @ Jw.T + 0.3 * np.eye(2)
        got = np.array([[gp.cov2d[i, 0], gp.cov2d[i, 1]], [gp.cov2d[i, 1], gp.cov2d[i, 2]]])
        np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(gp.mean2d[i], proj(X0), atol=1e-9)
        inv = np.linalg.inv(ref)
        np.testing.assert_allclose(gp.conic[i], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-5)


def test_pinned_f32_view_depth_matches_exact_rounding():
    """The pinned depth is ((r0 x + r1 y) + r2 z) + t with one float32 rounding
    per operation; re-evaluate it with exact rational arithmetic rounded to
    float32 after each step (binary64 holds every such product exactly and a
    single rounding of a binary64 quotient/sum to binary32 is correct)."""
    rng = np.random.default_rng(4)
    cam = scenes.look_at(rng.normal(size=3) * 3, 40, 30)
    P = rng.uniform(-1, 1, size=(200, 3)).astype(F32)

    def r32(x):
        return struct.unpack("f", struct.pack("f", x))[0]

    Rm, t = cam.R, cam.t
    got = R.view_row_f32(Rm.astype(F32), t.astype(F32), P, 2)
    for i in range(P.shape[0]):
        a = r32(float(Rm[2, 0]) * float(P[i, 0]))
        b = r32(float(Rm[2, 1]) * float(P[i, 1]))
        c = r32(float(Rm[2, 2]) * float(P[i, 2]))
        ref = r32(r32(r32(a + b) + c) + float(t[2]))
        assert float(got[i]) == ref


# ---------------------------------------------------------------- closed cases

def single_gaussian(z_world, o, rgb, s, cam):
    means = np.array([[0.0, 0.0, z_world]], F32)
    return dict(means=means, opac=np.array([o], F32), sh=dc_of(rgb)[None, None, :].astype(F32),
                scales=np.full((1, 3), s, F32), quats=np.array([[1, 0, 0, 0]], F32))


def test_isotropic_gaussian_closed_form():
    """A Gaussian on the optical axis whose mean projects to a pixel centre:
    Sigma_2D = (f s / z)^2 I + 0.3 I, alpha = min(0.99, o exp(-d^2 / (2 sigma^2)))."""
    W = H = 33       # odd size: the optical axis hits the centre of pixel 16
    cam = scenes.look_at((0.0, 0.0, 3.0), W, H)
    cam.cx = cam.cy = 16.5
    s, o, rgb, bg = 0.02, 0.7, np.array([0.9, 0.2, 0.4]), np.array([0.1, 0.3, 0.5])
    fr = frame(cam, **single_gaussian(0.0, o, rgb, s, cam), bg=bg)
    # the inputs are float32: use their exact values
    o = float(F32(o))
    rgb = dc_of(rgb).astype(F32).astype(np.float64) / (2 * math.sqrt(math.pi)) + 0.5
    s = float(F32(s))
    sig2 = (cam.fx * s / 3.0) ** 2 + 0.3
    for (px, py) in [(16, 16), (17, 16), (16, 18), (19, 14)]:
        d2 = (px - 16) ** 2 + (py - 16) ** 2
        a = min(0.99, o * math.exp(-0.5 * d2 / sig2))
        r = fr.pixel(px, py)
        if a >= 1 / 255:
            np.testing.assert_allclose(r.C, a * rgb + (1 - a) * bg, rtol=0, atol=1e-12)
            assert abs(r.T - (1 - a)) < 1e-12
        else:
            np.testing.assert_allclose(r.C, bg, rtol=0, atol=1e-12)


def test_alpha_clamp_and_threshold():
    cam = scenes.look_at((0.0, 0.0, 3.0), 33, 33)
    cam.cx = cam.cy = 16.5
    fr = frame(cam, **single_gaussian(0.0, 0.999, [1, 1, 1], 0.02, cam))
    assert fr.pixel(16, 16).T == 1.0 - 0.99           # clamped at 0.99
    far = frame(cam, **single_gaussian(0.0, 0.9, [1, 1, 1], 0.001, cam))
    # sigma^2 ~ 0.3 + tiny: at distance 3 px alpha = 0.9 e^-15 < 1/255 -> not blended
    r = far.pixel(19, 16)
    assert r.n_blended == 0 and r.T == 1.0


def test_gaussian_early_termination_closed_form():
    """k identical Gaussians at one pixel with alpha 0.95: T runs 0.05,
    0.0025, 1.25e-4; the 4th would leave 6.25e-6 < 1e-4, so it is skipped and
    the pixel stops with C = c (1 - 1.25e-4)."""
    cam = scenes.look_at((0.0, 0.0, 3.0), 33, 33)
    cam.cx = cam.cy = 16.5
    n = 6
    means = np.stack([np.zeros(n), np.zeros(n), -np.arange(n) * 0.01], 1).astype(F32)
    fr = frame(cam, means, np.full(n, 0.95, F32), np.tile(dc_of([0.3, 0.6, 0.9]), (n, 1, 1)).astype(F32),
               0, np.full((n, 3), 0.02, F32), np.tile(F32([1, 0, 0, 0]), (n, 1)))
    r = fr.pixel(16, 16)
    assert r.n_blended == 3
    assert r.order == [0, 1, 2]
    a = float(F32(0.95))
    assert abs(r.T - (1 - a) ** 3) < 1e-15
    col = dc_of([0.3, 0.6, 0.9]).astype(F32).astype(np.float64) / (2 * math.sqrt(math.pi)) + 0.5
    np.testing.assert_allclose(r.C, col * (1 - (1 - a) ** 3), rtol=0, atol=1e-12)


def big_tri(z_cam, alpha, rgb, cam, flip=False):
    """Triangle in the plane at camera depth z that covers the whole image."""
    zc = 3.0 - z_cam
    v = np.array([[-10.0, -10.0, zc], [10.0, -10.0, zc], [0.0, 10.0, zc]])
    if flip:
        v = v[[0, 2, 1]]
    return v[None].astype(F32), np.tile(np.asarray(rgb, F32), (1, 3, 1)), np.array([alpha], F32)


def cat_tris(*ts):
    return (np.concatenate([t[0] for t in ts]).astype(F32), np.concatenate([t[1] for t in ts]).astype(F32),
            np.concatenate([t[2] for t in ts]).astype(F32))


def test_opaque_triangle_returns_its_colour_exactly():
    cam = cam_at(16, 16)
    c = [0.25, 0.5, 0.75]
    for flip in (False, True):
        fr = frame(cam, tris=big_tri(2.0, 1.0, c, cam, flip), bg=(1, 1, 1))
        for px, py in [(0, 0), (7, 9), (15, 15)]:
            r = fr.pixel(px, py)
            assert r.T == 0.0
            # exact up to the rounding of the interpolation weights (sum 1)
            np.testing.assert_allclose(r.C, np.array(c, F32).astype(np.float64), rtol=0, atol=4e-16)


def test_front_gaussian_back_entities_closed_form():
    """Front triangle (full coverage, alpha_A), a Gaussian (alpha_G) and a back
    triangle (alpha_B): the Gaussian separates the two triangles into two
    entities (Section 3.2, Fig. 3d), so
    C = a_A c_A + (1-a_A) a_G c_G + (1-a_A)(1-a_G) a_B c_B."""
    W = H = 33
    cam = scenes.look_at((0.0, 0.0, 3.0), W, H)
    cam.cx = cam.cy = 16.5
    aA, aB = 0.4, 0.7
    cA, cG, cB = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0])
    g = single_gaussian(0.0, 0.6, cG, 0.05, cam)        # camera depth 3.0
    tris = cat_tris(big_tri(2.0, aA, cA, cam), big_tri(4.0, aB, cB, cam))
    fr = frame(cam, **g, tris=tris)
    r = fr.pixel(16, 16)
    aG = 0.6
    ref = aA * cA + (1 - aA) * aG * cG + (1 - aA) * (1 - aG) * aB * cB
    np.testing.assert_allclose(r.C, ref, rtol=0, atol=1e-7)   # colours pass through float32
    aA, aG, aB = (float(F32(x)) for x in (aA, aG, aB))
    np.testing.assert_allclose(r.T, (1 - aA) * (1 - aG) * (1 - aB), rtol=0, atol=1e-12)
    assert r.order == [1, 0, 2]
    # all triangles as one entity (Fig. 3b/c) overshoots: colour overflow
    ov = frame(cam, **g, tris=tris, mode=R.MODE_ONE_ENTITY).pixel(16, 16)
    assert ov.C.sum() > r.C.sum() + 1e-3
    assert ov.C[2] > ref[2] + 1e-3


def two_halves(alpha, cam, split_px):
    """Two triangles sharing the vertical line u = split_px (in pixels) at
    camera depth 2; together they cover the whole image."""
    zc = 1.0
    f = cam.fx
    xs = (split_px - cam.cx) * 2.0 / f          # world x of the split at depth 2
    L = np.array([[-10, -10, zc], [xs, -10, zc], [xs, 10, zc]], F32)
    L2 = np.array([[-10, -10, zc], [xs, 10, zc], [-10, 10, zc]], F32)
    Rr = np.array([[xs, -10, zc], [10, -10, zc], [10, 10, zc]], F32)
    R2 = np.array([[xs, -10, zc], [10, 10, zc], [xs, 10, zc]], F32)
    xyz = np.stack([L, L2, Rr, R2])
    rgb = np.ones((4, 3, 3), F32)
    return xyz, rgb, np.full(4, alpha, F32)


def test_abutting_triangles_entity_transmittance():
    """A shared edge through a pixel splits its 4 samples between two
    triangles.  Opaque: T_final = 0 (the literal Eq. 6 update would leave
    0.25).  alpha = 0.5: T = 0.5 (literal: 0.5625)."""
    cam = cam_at(16, 16)
    # split at pixel 8's centre x = 8.5: samples at -1/8 and -3/8 go left
    for alpha, t_ent, t_lit in [(1.0, 0.0, 0.25), (0.5, 0.5, 0.5625)]:
        tris = two_halves(alpha, cam, 8.5)
        fr = frame(cam, tris=tris)
        r = fr.pixel(8, 5)
        assert sorted(r.order) == r.order and len(r.order) == 2
        assert abs(r.T - t_ent) < 1e-12
        lit = frame(cam, tris=tris, mode=R.MODE_LITERAL_T).pixel(8, 5)
        assert abs(lit.T - t_lit) < 1e-12
        # interior pixels are covered by one triangle on all samples
        assert abs(fr.pixel(3, 5).T - (1 - alpha)) < 1e-12


def test_shared_edges_cover_each_sample_once():
    """Triangulated grid planes: every sample in the interior is covered by
    exactly one triangle (tie rule for samples on shared edges/vertices)."""
    cam = cam_at(24, 24)
    for n in (3, 7):
        V, F = scenes.grid_plane(n, 2.0, (0.0, 0.0, 0.5), (0.2, -0.1, 1.0))
        ts = R.setup_triangles(cam, V[F].astype(F32), np.ones((F.shape[0], 3, 3), F32),
                               np.ones(F.shape[0], F32))
        idx = np.flatnonzero(ts.valid)
        for px in range(8, 16):
            for py in range(8, 16):
                cov = R.sample_coverage(ts, idx, px, py)
                assert np.all(cov.sum(0) == 1), (n, px, py)
    # vertices landing exactly on sample positions: 8 triangles fanned around
    # a vertex at a sample point (1/256-px grid)
    ts = fan_around_sample(cam)
    idx = np.flatnonzero(ts.valid)
    cov = R.sample_coverage(ts, idx, 10, 10)
    assert np.all(cov.sum(0) == 1)


def fan_around_sample(cam):
    """Direct TriSetup of a triangle fan whose centre sits on a sample of
    pixel (10, 10) and whose spokes pass through the other samples."""
    c = (10 * 256 + 128 - 32, 10 * 256 + 128 - 96)        # sample 0 of pixel (10,10)
    ang = np.linspace(0, 2 * math.pi, 9)[:-1]
    ring = [(c[0] + int(round(900 * math.cos(a))), c[1] + int(round(900 * math.sin(a)))) for a in ang]
    X, Y = [], []
    for i in range(8):
        a, b = ring[i], ring[(i + 1) % 8]
        X.append([c[0], a[0], b[0]])
        Y.append([c[1], a[1], b[1]])
    X = np.array(X, np.int64)
    Y = np.array(Y, np.int64)
    area = (X[:, 1] - X[:, 0]) * (Y[:, 2] - Y[:, 0]) - (Y[:, 1] - Y[:, 0]) * (X[:, 2] - X[:, 0])
    sw = area < 0
    X[sw] = X[sw][:, [0, 2, 1]]
    Y[sw] = Y[sw][:, [0, 2, 1]]
    n = 8
    return R.TriSetup(valid=np.ones(n, bool), key=np.ones(n, F32), X=X, Y=Y, area2=np.abs(area),
                      z=np.ones((n, 3)), rgb=np.ones((n, 3, 3)), alpha=np.ones(n))


def test_perspective_correct_colour_matches_ray_plane_hit():
    """Colour of a slanted triangle at a pixel centre equals the barycentric
    interpolation at the 3D point where the pixel's ray meets the triangle."""
    cam = scenes.look_at((0.0, 0.0, 3.0), 400, 400)
    v = np.array([[-0.8, -0.6, 0.9], [0.9, -0.5, -0.7], [-0.1, 0.9, 0.2]])
    rgb = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    ts = R.setup_triangles(cam, v[None].astype(F32), rgb[None].astype(F32), np.ones(1, F32))
    eye = cam.center
    n = np.cross(v[1] - v[0], v[2] - v[0])
    for px, py in [(200, 200), (150, 230), (230, 180), (190, 120)]:
        d = pixel_ray_world(cam, px, py)
        t = (n @ (v[0] - eye)) / (n @ d)
        P = eye + t * d
        # 3D barycentrics
        A = np.stack([v[0] - v[2], v[1] - v[2]], 1)
        lam01 = np.linalg.lstsq(A, P - v[2], rcond=None)[0]
        lam = np.array([lam01[0], lam01[1], 1 - lam01.sum()])
        assert np.all(lam > 0.02)
        got = R.triangle_colour(ts, np.array([0]), px, py)[0]
        np.testing.assert_allclose(got, lam @ rgb, atol=2e-4)


def test_quad_tie_breaks_by_id():
    s = scenes.make_config(0)
    ts = R.setup_triangles(s.cams[0], s.tri_xyz, s.tri_rgb, s.tri_alpha)
    assert ts.key[-1] == ts.key[-2]
    fr = R.Frame(s.cams[0], s.means, s.opacity, s.sh, 0, s.tri_xyz, s.tri_rgb, s.tri_alpha,
                 scales=s.scales, quats=s.quats)
    N = s.N
    hits = 0
    for px in range(20, 44):
        r = fr.pixel(px, 63 - px)      # the quad's diagonal runs along u + v = 64
        q = [g for g in r.contributors if g >= N + s.T - 2]
        if len(q) == 2:
            hits += 1
            assert q == [N + s.T - 2, N + s.T - 1]
    assert hits > 0


# ---------------------------------------------------------------- invariants

def test_transmittance_monotone_and_bounded():
    s = scenes.make_config(0, scale=0.5, res_scale=0.5)
    fr = R.Frame(s.cams[0], s.means, s.opacity, s.sh, 0, s.tri_xyz, s.tri_rgb, s.tri_alpha,
                 scales=s.scales, quats=s.quats)
    for py in range(0, 32, 3):
        for px in range(0, 32, 3):
            r = fr.pixel(px, py)
            tr = [1.0] + r.T_trace
            assert all(0.0 <= t <= 1.0 for t in tr)
            assert all(b <= a + 1e-15 for a, b in zip(tr, tr[1:]))


def white_scene(mode):
    s = scenes.make_config(0, scale=0.5, res_scale=0.5)
    sh = np.zeros_like(s.sh)
    sh[:, 0, :] = dc_of([1, 1, 1])
    return R.Frame(s.cams[0], s.means, s.opacity, sh, 0, s.tri_xyz, np.ones_like(s.tri_rgb),
                   s.tri_alpha, scales=s.scales, quats=s.quats, mode=mode)


def test_white_scene_energy():
    """All colours 1 and a black background: C = 1 - T_final at every pixel
    (energy is conserved by the sub-sample transmittance update).  The
    Gaussians' white comes from a float32 SH coefficient, so it is 1 only to
    ~3e-8."""
    fr = white_scene(R.MODE_UNIMGS)
    worst = 0.0
    for py in range(32):
        for px in range(32):
            r = fr.pixel(px, py)
            worst = max(worst, np.max(np.abs(r.C - (1 - r.T))))
    assert worst < 1e-7
    # the literal pixel-level update breaks it wherever entities hold partial coverage
    lit = white_scene(R.MODE_LITERAL_T)
    worst = 0.0
    for py in range(32):
        for px in range(32):
            r = lit.pixel(px, py)
            worst = max(worst, np.max(np.abs(r.C - (1 - r.T))))
    assert worst > 1e-3


# ---------------------------------------------------------------- reductions

def random_tri_scene(rng, cam, n, alpha_range):
    """Random triangles in front of the camera; vertices avoid landing on the
    sub-pixel sample grid only by chance (coverage ties are rare)."""
    v = rng.uniform(-0.7, 0.7, size=(n, 3, 3))
    v[:, :, 2] = rng.uniform(-0.5, 0.5, size=(n, 1)) + rng.uniform(-0.2, 0.2, size=(n, 3))
    rgb = rng.uniform(0, 1, size=(n, 3, 3))
    al = rng.uniform(*alpha_range, size=n)
    return v.astype(F32), rgb.astype(F32), al.astype(F32)


def inside_by_areas(ts, i, Sx, Sy):
    """Independent point-in-triangle test: the three sub-triangle areas of
    the sample sum to the triangle's area and none is negative."""
    X, Y = ts.X[i].tolist(), ts.Y[i].tolist()

    def cross(ax, ay, bx, by, cx, cy):
        return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)
    a0 = cross(X[1], Y[1], X[2], Y[2], Sx, Sy)
    a1 = cross(X[2], Y[2], X[0], Y[0], Sx, Sy)
    a2 = cross(X[0], Y[0], X[1], Y[1], Sx, Sy)
    tot = cross(X[0], Y[0], X[1], Y[1], X[2], Y[2])
    if min(a0, a1, a2) == 0:
        return None           # on an edge: tie, handled elsewhere
    return a0 > 0 and a1 > 0 and a2 > 0 and a0 + a1 + a2 == tot


def test_triangle_only_equals_supersampled_compositing():
    """With triangles only, every pixel holds one entity, and Eq. 7-9 reduce
    to ordinary alpha compositing run separately at each of the 4 samples
    (shading once per pixel) and averaged."""
    rng = np.random.default_rng(5)
    cam = cam_at(20, 20)
    checked = 0
    for trial in range(3):
        xyz, rgb, al = random_tri_scene(rng, cam, 12, (0.2, 0.7))
        fr = frame(cam, tris=(xyz, rgb, al))
        ts = fr.t
        for py in range(0, 20, 2):
            for px in range(0, 20, 2):
                r = fr.pixel(px, py)
                live = np.flatnonzero(ts.valid)
                cols = R.triangle_colour(ts, live, px, py) if live.size else None
                Cs, Ts, tie = [], [], False
                for ox, oy in R.SAMPLE_OFFSETS:
                    Sx, Sy = px * 256 + 128 + ox, py * 256 + 128 + oy
                    hit = []
                    for j, i in enumerate(live):
                        ins = inside_by_areas(ts, i, Sx, Sy)
                        if ins is None:
                            tie = True
                        elif ins:
                            hit.append((float(ts.key[i]), int(i), j))
                    hit.sort()
                    c, t = np.zeros(3), 1.0
                    for _, i, j in hit:
                        c += t * ts.alpha[i] * cols[j]
                        t *= 1 - ts.alpha[i]
                    Cs.append(c)
                    Ts.append(t)
                if tie or np.mean(Ts) < 2e-4:
                    continue
                np.testing.assert_allclose(r.C, np.mean(Cs, 0), rtol=0, atol=1e-12)
                assert abs(r.T - np.mean(Ts)) < 1e-12
                checked += 1
    assert checked > 200


def test_opaque_entity_equals_msaa_resolve():
    """All triangles opaque: Eq. 8 reduces to the depth-tested coverage of
    Eq. 3-4, i.e. a 4x MSAA resolve of the nearest triangle per sample."""
    rng = np.random.default_rng(6)
    cam = cam_at(20, 20)
    bg = np.array([0.2, 0.1, 0.05])
    for trial in range(3):
        xyz, rgb, _ = random_tri_scene(rng, cam, 10, (1, 1))
        al = np.ones(10, F32)
        fr = frame(cam, tris=(xyz, rgb, al), bg=bg)
        ts = fr.t
        live = np.flatnonzero(ts.valid)
        for py in range(0, 20, 2):
            for px in range(0, 20, 2):
                cols = R.triangle_colour(ts, live, px, py)
                acc = np.zeros(3)
                tie = False
                for ox, oy in R.SAMPLE_OFFSETS:
                    Sx, Sy = px * 256 + 128 + ox, py * 256 + 128 + oy
                    best = None
                    for j, i in enumerate(live):
                        ins = inside_by_areas(ts, i, Sx, Sy)
                        tie |= ins is None
                        if ins and (best is None or (ts.key[i], i) < best[0]):
                            best = ((ts.key[i], i), j)
                    acc += bg if best is None else cols[best[1]]
                if tie:
                    continue
                np.testing.assert_allclose(fr.pixel(px, py).C, acc / 4, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- brute force

def brute_force_pixel(cam, scene, px, py):
    """Independent per-pixel renderer for tiny scenes, written as a sample-state
    machine: the pixel keeps four absolute sub-sample transmittances u_j.  A
    Gaussian uses their mean and then makes them uniform again; a triangle
    shades with alpha c mean_j(o_j u_j) and attenuates the covered u_j."""
    means, opac, sh, scales, quats, xyz, rgb, al = scene
    N = means.shape[0]
    W = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)
    cen = cam.center
    frags = []
    for i in range(N):
        X = means[i].astype(np.float64)
        p = W @ X + t
        if not np.float32(p[2]) > 0.2:
            continue

        def proj(Y):
            q = W @ Y + t
            return np.array([cam.fx * q[0] / q[2] + cam.cx, cam.fy * q[1] / q[2] + cam.cy])
        h = 1e-6
        Jw = np.stack([(proj(X + h * e) - proj(X - h * e)) / (2 * h) for e in np.eye(3)], 1)
        from scipy.spatial.transform import Rotation
        Rq = Rotation.from_quat(np.r_[quats[i, 1:], quats[i, 0]]).as_matrix()
        Sig = Rq @ np.diag(scales[i].astype(np.float64) ** 2) @ Rq.T
        S2 = Jw @ Sig @ Jw.T + 0.3 * np.eye(2)
        d = proj(X) - np.array([px + 0.5, py + 0.5])
        a = min(0.99, float(opac[i]) * math.exp(-0.5 * d @ np.linalg.solve(S2, d)))
        if a < 1 / 255:
            continue
        col = np.maximum(sh[i, 0].astype(np.float64) / (2 * math.sqrt(math.pi)) + 0.5, 0)
        key = R.view_row_f32(cam.R.astype(F32), cam.t.astype(F32), means[i:i + 1], 2)[0]
        frags.append((float(key), i, "g", a, col, None))
    fr = frame(cam, tris=(xyz, rgb, al))
    ts = fr.t
    live = np.flatnonzero(ts.valid)
    if live.size:
        cols = R.triangle_colour(ts, live, px, py)
    for j, i in enumerate(live):
        o = []
        for ox, oy in R.SAMPLE_OFFSETS:
            ins = inside_by_areas(ts, i, px * 256 + 128 + ox, py * 256 + 128 + oy)
            if ins is None:
                return None
            o.append(1.0 if ins else 0.0)
        if any(o):
            frags.append((float(ts.key[i]), N + int(i), "t", float(ts.alpha[i]), cols[j], np.array(o)))
    frags.sort(key=lambda f: (f[0], f[1]))
    u = np.ones(4)
    C = np.zeros(3)
    for key, gid, kind, a, col, o in frags:
        T = u.mean()
        if kind == "g":
            if T * (1 - a) < 1e-4:
                break
            C += T * a * col
            u[:] = T * (1 - a)
        else:
            C += a * col * np.mean(o * u)
            u = u * (1 - o * a)
            if u.mean() < 1e-4:
                break
    return C, u.mean()


@pytest.mark.parametrize("seed", [10, 11, 12, 13])
def test_brute_force_tiny_scenes(seed):
    rng = np.random.default_rng(seed)
    cam = cam_at(8, 8, eye=(0.0, 0.0, 2.0))
    ng, nt = 3, 3
    means = rng.uniform(-0.25, 0.25, size=(ng, 3)).astype(F32)
    opac = rng.uniform(0.3, 0.95, size=ng).astype(F32)
    sh = dc_of(rng.uniform(0, 1, size=(ng, 3)))[:, None, :].astype(F32)
    scales = np.exp(rng.normal(-2.5, 0.3, size=(ng, 3))).astype(F32)
    quats = rng.normal(size=(ng, 4)).astype(F32)
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    xyz, rgb, al = random_tri_scene(rng, cam, nt, (0.3, 1.0))
    xyz *= 0.5
    fr = frame(cam, means, opac, sh, 0, scales, quats, tris=(xyz, rgb, al))
    n = 0
    for py in range(8):
        for px in range(8):
            bf = brute_force_pixel(cam, (means, opac, sh, scales, quats, xyz, rgb, al), px, py)
            if bf is None:
                continue
            r = fr.pixel(px, py)
            if r.margin < 1e-6:
                continue
            np.testing.assert_allclose(r.C, bf[0], rtol=0, atol=1e-9)
            assert abs(r.T - bf[1]) < 1e-9
            n += 1
    assert n > 40


# ---------------------------------------------------------------- ablation modes

def tri_at_pixels(cam, uv, depth, alpha, rgb):
    """One triangle whose vertices project to the pixel coordinates uv (3,2)
    at camera depth ``depth`` (inverse of the pinhole map), constant colour."""
    R = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)
    pts = []
    for u, v in uv:
        pc = np.array([(u - cam.cx) * depth / cam.fx, (v - cam.cy) * depth / cam.fy, depth])
        pts.append(R.T @ (pc - t))
    return (np.array(pts, F32)[None], np.tile(np.asarray(rgb, F32), (1, 3, 1)),
            np.array([alpha], F32))


def upper_tri(cam, py, edge_off, depth, alpha, rgb):
    """Large triangle covering everything above the horizontal line
    v = py + 0.5 + edge_off/256 (edge_off in 1/256 px from the centre row of
    pixel row py)."""
    ve = py + 0.5 + edge_off / 256.0
    return tri_at_pixels(cam, [(-300.0, ve), (300.0, ve), (0.0, ve - 600.0)], depth, alpha, rgb)


def test_direct_mode_uses_the_pixel_centre_only():
    """Direct alpha-blending (Fig. 3a) treats a triangle like a Gaussian with
    coverage decided at the pixel centre: a triangle over the centre gives
    C = alpha c + (1 - alpha) C_bg exactly (C = c when opaque) whatever part
    of the pixel it covers; one that covers two of the four sub-samples but
    not the centre gives nothing.  The UniMGS entity rule weighs both by the
    covered fraction of the sub-samples (1/2 here)."""
    cam = cam_at(16, 16)
    c = np.array([0.2, 0.6, 0.9])
    bg = np.array([0.3, 0.1, 0.5])
    c32 = c.astype(F32).astype(np.float64)
    for alpha in (1.0, 0.6):
        a = float(F32(alpha))
        # edge 16/256 px above the centre: samples at -96 and -32 covered, centre not
        off = frame(cam, tris=upper_tri(cam, 7, -16, 2.0, alpha, c), bg=bg, mode=R.MODE_DIRECT).pixel(5, 7)
        assert off.n_blended == 0 and off.T == 1.0
        np.testing.assert_allclose(off.C, bg, rtol=0, atol=0)
        # edge 16/256 px below the centre: the centre and the same two samples covered
        on = frame(cam, tris=upper_tri(cam, 7, 16, 2.0, alpha, c), bg=bg, mode=R.MODE_DIRECT).pixel(5, 7)
        assert on.n_blended == 1
        assert abs(on.T - (1 - a)) < 1e-15
        np.testing.assert_allclose(on.C, a * c32 + (1 - a) * bg, rtol=0, atol=4e-16)
        for edge in (-16, 16):
            uni = frame(cam, tris=upper_tri(cam, 7, edge, 2.0, alpha, c), bg=bg).pixel(5, 7)
            assert abs(uni.T - (1 - a / 2)) < 1e-15
            np.testing.assert_allclose(uni.C, 0.5 * a * c32 + (1 - a / 2) * bg, rtol=0, atol=4e-16)


def test_direct_mode_blends_triangles_in_depth_order_and_stops_after_opaque():
    """Direct mode: two full-coverage triangles (alpha_A in front, alpha_B
    behind) give C = a_A c_A + (1-a_A) a_B c_B; an opaque front triangle ends
    the pixel with its exact colour and nothing behind it is blended."""
    cam = cam_at(16, 16)
    cA, cB = np.array([1.0, 0.5, 0.0]), np.array([0.0, 0.25, 1.0])
    for aA, aB in ((0.3, 0.8), (1.0, 0.8)):
        tris = cat_tris(big_tri(2.0, aA, cA, cam), big_tri(3.0, aB, cB, cam))
        r = frame(cam, tris=tris, mode=R.MODE_DIRECT).pixel(6, 9)
        a1, a2 = float(F32(aA)), float(F32(aB))
        if aA == 1.0:
            assert r.order == [0] and r.T == 0.0
            np.testing.assert_allclose(r.C, cA, rtol=0, atol=4e-16)
        else:
            assert r.order == [0, 1]
            np.testing.assert_allclose(r.C, a1 * cA + (1 - a1) * a2 * cB, rtol=0, atol=1e-15)
            assert abs(r.T - (1 - a1) * (1 - a2)) < 1e-15


def test_one_entity_mode_closed_form():
    """All triangles of a pixel as one entity (Fig. 3b/c): a Gaussian between
    the front (alpha_A) and back (alpha_B) triangles does not close the
    entity, so the back triangle is weighted by the sub-sample transmittance
    of the front one only: C = a_A c_A + (1-a_A) a_G c_G + (1-a_A) a_B c_B
    (the Gaussian's share is counted twice: colour overflow), and the pixel
    transmittance after the entity is (1-a_A)(1-a_B)."""
    W = H = 33
    cam = scenes.look_at((0.0, 0.0, 3.0), W, H)
    cam.cx = cam.cy = 16.5
    aA, aB, aG = 0.4, 0.7, 0.6
    cA, cG, cB = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0])
    g = single_gaussian(0.0, aG, cG, 0.05, cam)
    tris = cat_tris(big_tri(2.0, aA, cA, cam), big_tri(4.0, aB, cB, cam))
    r = frame(cam, **g, tris=tris, mode=R.MODE_ONE_ENTITY).pixel(16, 16)
    assert r.order == [1, 0, 2]
    ref = aA * cA + (1 - aA) * aG * cG + (1 - aA) * aB * cB
    np.testing.assert_allclose(r.C, ref, rtol=0, atol=1e-7)   # colours pass through float32
    a1, a2 = float(F32(aA)), float(F32(aB))
    assert abs(r.T - (1 - a1) * (1 - a2)) < 1e-15


# ---------------------------------------------------------------- EWA frustum clamp

def test_ewa_jacobian_frustum_clamp_matches_numerical_jacobian():
    """Outside 1.3 tan(fov/2) the EWA Jacobian is the derivative of the
    pinhole map taken at the point moved onto the clamp boundary (same depth);
    inside, at the mean itself.  The 2D mean is never clamped.  Reference:
    central differences of the pinhole map at that point."""
    cam = scenes.look_at((0.0, 0.0, 3.0), 64, 48)
    tanx, tany = cam.width / (2 * cam.fx), cam.height / (2 * cam.fy)
    W = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)
    z = 2.5
    # camera-space directions: x/z, y/z in units of tan(fov/2)
    dirs = [(1.5, 0.2), (-2.0, 0.5), (0.3, -1.8), (1.7, 1.4), (1.2, -1.25), (0.9, 0.1), (-2.6, -2.2)]
    pc = np.array([[ax * tanx * z, ay * tany * z, z] for ax, ay in dirs])
    means = ((pc - t) @ W).astype(F32)                 # world = R^T (p - t)
    n = len(dirs)
    rng = np.random.default_rng(11)
    scales = np.exp(rng.normal(-1.5, 0.3, size=(n, 3))).astype(F32)
    q = rng.normal(size=(n, 4)).astype(F32)
    gp = R.project_gaussians(cam, means, np.full(n, 0.5), np.zeros((n, 1, 3)), 0, scales, q)
    Sig = R.cov3d_from_scale_rot(scales, q)

    def pinhole(p):
        return np.array([cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy])

    clamped = 0
    for i in range(n):
        p = W @ means[i].astype(np.float64) + t
        lx, ly = 1.3 * tanx, 1.3 * tany
        pcl = np.array([np.clip(p[0] / p[2], -lx, lx) * p[2], np.clip(p[1] / p[2], -ly, ly) * p[2], p[2]])
        h = 1e-6
        Jc = np.stack([(pinhole(pcl + h * e) - pinhole(pcl - h * e)) / (2 * h) for e in np.eye(3)], 1)
        ref = Jc @ W @ Sig[i] @ W.T @ Jc.T + 0.3 * np.eye(2)
        got = np.array([[gp.cov2d[i, 0], gp.cov2d[i, 1]], [gp.cov2d[i, 1], gp.cov2d[i, 2]]])
        np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(gp.mean2d[i], pinhole(p), atol=1e-9)
        if not np.allclose(pcl, p):
            clamped += 1
            Ju = np.stack([(pinhole(p + h * e) - pinhole(p - h * e)) / (2 * h) for e in np.eye(3)], 1)
            unc = Ju @ W @ Sig[i] @ W.T @ Ju.T + 0.3 * np.eye(2)
            assert np.abs(unc - ref).max() > 1e-3 * np.abs(ref).max()
    assert clamped == 5                # (1.2, -1.25) and (0.9, 0.1) lie inside the clamp
