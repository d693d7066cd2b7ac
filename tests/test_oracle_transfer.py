"""Pins of the deformation-transfer oracle (Section 3.3.2, Eq. 12-13).

Closed forms for identity, rigid and similarity deformations of the proxy;
library routines for the polar decomposition and the rotation log/exp; the
least-squares optimality of the per-vertex gradient; and the cotangent
weights of a regular fan.
"""
import math

import numpy as np
import pytest
from scipy.linalg import polar as scipy_polar
from scipy.spatial.transform import Rotation

from oracle import transfer as TR
from paper_2601_19233_amd import scenes

F32 = np.float32


def small_scene(K, seed=0, n=300, freq=6):
    rng = np.random.default_rng(seed)
    V, F = scenes.icosphere(freq, 1.0)
    means = scenes._sample_on_mesh(rng, V, F, n, 0.02).astype(F32)
    log_s = rng.normal(-3.0, 0.5, size=(n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    s = np.exp(log_s).astype(F32)
    q = q.astype(F32)
    bf, bb = scenes.make_binding(means, s, q, V, F, K)
    return V, F, means, s, q, bf, bb


def cov_of(c6):
    c = c6
    return np.stack([np.stack([c[:, 0], c[:, 1], c[:, 2]], -1),
                     np.stack([c[:, 1], c[:, 3], c[:, 4]], -1),
                     np.stack([c[:, 2], c[:, 4], c[:, 5]], -1)], -2)


def bound_points(V, F, bf, bb):
    fv = F[bf]
    u, v = bb[..., 0].astype(np.float64), bb[..., 1].astype(np.float64)
    w = 1 - u - v
    return (u[..., None] * V[fv[..., 0]] + v[..., None] * V[fv[..., 1]] + w[..., None] * V[fv[..., 2]])


@pytest.mark.parametrize("K", [1, 8])
def test_identity_deformation(K):
    V, F, mu, s, q, bf, bb = small_scene(K)
    out = TR.transfer(V, F, V.copy(), mu, q, s, bf, bb)
    assert np.array_equal(out["means"], mu)
    Sig = TR._cov3d(s, q)
    np.testing.assert_allclose(cov_of(out["cov3d"]), Sig, rtol=0, atol=1e-14)
    qn = q.astype(np.float64) / np.linalg.norm(q.astype(np.float64), axis=1, keepdims=True)
    np.testing.assert_allclose(out["quats"], qn, atol=1e-12)


@pytest.mark.parametrize("K", [1, 8])
@pytest.mark.parametrize("scale", [1.0, 1.7])
def test_similarity_deformation_closed_form(K, scale):
    """V' = s Q V + t: every vertex gets D = s Q, so R' = Q, S' = s I,
    Sigma' = s^2 Q Sigma Q^T, mu' = mu + mean_i((sQ - I) P_i + t) and
    q' = q_Q (x) q."""
    V, F, mu, s, q, bf, bb = small_scene(K, seed=1)
    Qr = Rotation.from_rotvec([0.3, -0.5, 0.2])
    Q = Qr.as_matrix()
    t = np.array([0.1, -0.2, 0.3])
    Vd = scale * V @ Q.T + t
    out = TR.transfer(V, F, Vd, mu, q, s, bf, bb)
    vt = out["vertex"]
    np.testing.assert_allclose(vt["D"], np.broadcast_to(scale * Q, vt["D"].shape), atol=1e-9)
    np.testing.assert_allclose(vt["S"], np.broadcast_to(scale * np.eye(3), vt["S"].shape), atol=1e-9)
    Sig = TR._cov3d(s, q)
    ref = scale ** 2 * np.einsum("ij,njk,lk->nil", Q, Sig, Q)
    np.testing.assert_allclose(cov_of(out["cov3d"]), ref, rtol=1e-8, atol=1e-14)
    P = bound_points(V, F, bf, bb)
    mu_ref = mu.astype(np.float64) + (P @ (scale * Q - np.eye(3)).T + t).mean(1)
    np.testing.assert_allclose(out["means"], mu_ref, atol=3e-6)
    qq = np.r_[Qr.as_quat()[3], Qr.as_quat()[:3]]
    qn = q.astype(np.float64) / np.linalg.norm(q.astype(np.float64), axis=1, keepdims=True)
    ref_q = TR.quat_mul(np.tile(qq, (qn.shape[0], 1)), qn)
    sgn = np.sign((out["quats"] * ref_q).sum(1))[:, None]
    np.testing.assert_allclose(out["quats"] * sgn, ref_q, atol=1e-9)


def test_pinned_mean_exact_rounding():
    """mu' float32 operation order: check against a per-element re-evaluation."""
    import struct

    def r32(x):
        return struct.unpack("f", struct.pack("f", x))[0]
    V, F, mu, s, q, bf, bb = small_scene(8, seed=2, n=20)
    rng = np.random.default_rng(3)
    Vd = V + rng.normal(0, 0.05, size=V.shape)
    d32 = np.asarray(Vd, F32) - np.asarray(V, F32)
    got = TR.pinned_mean(mu, d32, F, bf, bb)
    for n in range(20):
        for c in range(3):
            acc = None
            for i in range(8):
                a, b, cc = F[bf[n, i]]
                u, v = float(bb[n, i, 0]), float(bb[n, i, 1])
                w = r32(r32(1.0 - u) - v)
                di = r32(r32(r32(u * float(d32[a, c])) + r32(v * float(d32[b, c])))
                         + r32(w * float(d32[cc, c])))
                acc = di if acc is None else r32(acc + di)
            ref = r32(float(mu[n, c]) + r32(acc * 0.125))
            assert float(got[n, c]) == ref


def test_gradient_is_least_squares_minimiser():
    """Optimality of D_v: the objective's gradient
    sum c (e' - D e) e^T + w (n' - D n) n^T vanishes (checked by perturbation)."""
    V, F = scenes.icosphere(5, 1.0)
    rng = np.random.default_rng(4)
    L = np.eye(3) + rng.normal(0, 0.3, size=(3, 3))
    Vd = V @ L.T + np.sin(3 * V) * 0.05
    D = TR.deformation_gradients(V, F, Vd)
    Fr, cot_b, cot_a = TR.cot_weights_per_corner(V, F)

    def objective(v, Dm):
        m = Fr[:, 0] == v
        val = 0.0
        nrm, nrmd, ls, lsd, ws = np.zeros(3), np.zeros(3), 0.0, 0.0, 0.0
        for (vv, a, b), cb, ca in zip(Fr[m], cot_b[m], cot_a[m]):
            ea, eb = V[a] - V[v], V[b] - V[v]
            fa, fb = Vd[a] - Vd[v], Vd[b] - Vd[v]
            val += 0.5 * cb * np.sum((fa - Dm @ ea) ** 2) + 0.5 * ca * np.sum((fb - Dm @ eb) ** 2)
            nrm += np.cross(ea, eb)
            nrmd += np.cross(fa, fb)
            ls += np.linalg.norm(ea) + np.linalg.norm(eb)
            lsd += np.linalg.norm(fa) + np.linalg.norm(fb)
            ws += 0.5 * (ca + cb)
        k = m.sum()
        n = nrm / np.linalg.norm(nrm) * ls / (2 * k)
        nd = nrmd / np.linalg.norm(nrmd) * lsd / (2 * k)
        return val + ws / k * np.sum((nd - Dm @ n) ** 2)

    for v in [0, 17, 101]:
        f0 = objective(v, D[v])
        for _ in range(5):
            E = rng.normal(size=(3, 3)) * 1e-4
            # at a minimum, f(D + E) - f(D) is quadratic (no linear term)
            d1 = objective(v, D[v] + E) - f0
            d2 = objective(v, D[v] - E) - f0
            assert d1 > 0 and d2 > 0
            assert abs(d1 - d2) < 1e-6 * (abs(d1) + abs(d2))


def test_polar_matches_scipy_and_invariants():
    rng = np.random.default_rng(5)
    D = np.eye(3) + rng.normal(0, 0.3, size=(50, 3, 3))
    D = D[np.linalg.det(D) > 0.05]
    Rm, S = TR.polar(D)
    for i in range(D.shape[0]):
        U, P = scipy_polar(D[i])
        np.testing.assert_allclose(Rm[i], U, atol=1e-10)
        np.testing.assert_allclose(S[i], P, atol=1e-10)
    np.testing.assert_allclose(Rm @ S, D, atol=1e-12)
    np.testing.assert_allclose(np.transpose(Rm, (0, 2, 1)) @ Rm, np.broadcast_to(np.eye(3), Rm.shape), atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(Rm), 1.0, atol=1e-12)
    assert np.all(np.linalg.eigvalsh(S) > 0)


def test_log_exp_match_scipy():
    rng = np.random.default_rng(6)
    r = rng.normal(size=(100, 3))
    r *= (rng.uniform(0, 2.5, size=100) / np.linalg.norm(r, axis=1))[:, None]
    r[:5] *= 1e-7          # series branch
    Rm = TR.exp_rot(r)
    np.testing.assert_allclose(Rm, Rotation.from_rotvec(r).as_matrix(), atol=1e-13)
    np.testing.assert_allclose(TR.log_rot(Rm), r, atol=1e-9)
    np.testing.assert_allclose(TR.log_rot(Rm)[:5], Rotation.from_matrix(Rm[:5]).as_rotvec(), atol=1e-15)
    q = TR.quat_of_axis_angle(r)
    qs = Rotation.from_rotvec(r).as_quat()
    np.testing.assert_allclose(q, np.c_[qs[:, 3], qs[:, :3]] * np.sign(qs[:, 3:4]) * np.sign(q[:, :1]), atol=1e-13)


def test_log_near_pi_matches_scipy():
    """Angles from pi/2 to pi - 1e-9 (and pi itself): the log returns the
    rotation vector (scipy's independent conversion) to 1e-9; at pi, where
    +a and -a name the same rotation, exp(log R) = R."""
    rng = np.random.default_rng(16)
    a = rng.normal(size=(200, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    th = np.concatenate([rng.uniform(0.5 * np.pi, np.pi - 1e-3, 150),
                         np.pi - 10.0 ** -rng.uniform(3, 9, 50)])
    r = a * th[:, None]
    Rm = Rotation.from_rotvec(r).as_matrix()
    got = TR.log_rot(Rm)
    np.testing.assert_allclose(got, Rotation.from_matrix(Rm).as_rotvec(), atol=1e-9)
    np.testing.assert_allclose(got, r, atol=2e-8)
    Rpi = Rotation.from_rotvec(a[:20] * np.pi).as_matrix()
    lp = TR.log_rot(Rpi)
    np.testing.assert_allclose(np.linalg.norm(lp, axis=1), np.pi, atol=1e-12)
    np.testing.assert_allclose(TR.exp_rot(lp), Rpi, atol=1e-12)


def test_cot_weights_regular_fan():
    """Six equilateral triangles around a vertex: every interior angle is 60
    degrees, so each spoke's weight is (cot 60 + cot 60)/2 = 1/sqrt 3."""
    ang = np.arange(6) * math.pi / 3
    V = np.vstack([[0, 0, 0], np.stack([np.cos(ang), np.sin(ang), np.zeros(6)], 1)])
    F = np.array([[0, 1 + i, 1 + (i + 1) % 6] for i in range(6)])
    Fr, cot_b, cot_a = TR.cot_weights_per_corner(V, F)
    m = Fr[:, 0] == 0
    np.testing.assert_allclose(cot_b[m], 1 / math.sqrt(3), atol=1e-14)
    np.testing.assert_allclose(cot_a[m], 1 / math.sqrt(3), atol=1e-14)
    # planar 1-ring: the normal pair keeps D defined; a rigid motion is recovered
    Q = Rotation.from_rotvec([0.2, 0.4, -0.1]).as_matrix()
    D = TR.deformation_gradients(V, F, V @ Q.T)
    np.testing.assert_allclose(D[0], Q, atol=1e-12)


def test_interpolation_at_a_vertex_reproduces_the_vertex():
    """Eq. 12 with barycentric (1, 0, 0) returns vertex quantities; Eq. 13 with
    all K bindings at one vertex returns exp(r_v), S_v."""
    V, F = scenes.icosphere(4, 1.0)
    Vd = scenes.bend(V)
    vt = TR.vertex_transforms(V, F, Vd)
    n = 5
    bf = np.tile(np.arange(n)[:, None], (1, 8)).astype(np.int32)
    bb = np.zeros((n, 8, 2), F32)
    bb[:, :, 0] = 1.0                       # u = 1 -> vertex F[f, 0]
    mu = np.zeros((n, 3), F32)
    s = np.full((n, 3), 0.05, F32)
    q = np.tile(F32([1, 0, 0, 0]), (n, 1))
    out = TR.transfer(V, F, Vd, mu, q, s, bf, bb)
    v0 = F[np.arange(n), 0]
    A_ref = TR.exp_rot(vt["r"][v0]) @ vt["S"][v0]
    np.testing.assert_allclose(out["A"], A_ref, atol=1e-12)
    np.testing.assert_allclose(out["A"], vt["D"][v0], atol=1e-10)    # exp(log R) S = R S = D
    np.testing.assert_allclose(out["means"], vt["delta32"][v0], atol=0)


# ---------------------------------------------------------------- Eq. 13 averaging

def _frames(r, S, nV=None):
    """Hand-built per-vertex frames: axis-angle r (nV,3), stretch S (nV,3,3), no offset."""
    r = np.asarray(r, np.float64)
    nV = r.shape[0]
    return dict(delta32=np.zeros((nV, 3), F32), r=r, S=np.asarray(S, np.float64))


def _one_gaussian(n=1):
    mu = np.zeros((n, 3), F32)
    s = np.tile(F32([0.05, 0.02, 0.08]), (n, 1))
    q = np.tile(F32([0.9, 0.1, -0.3, 0.2]), (n, 1))
    return mu, s, q


def test_opposite_rotations_average_to_identity():
    """Eq. 13 averages the log-rotations of the corners, then exponentiates:
    four corners at a vertex turned by +theta about z and four at one turned
    by -theta give R' = I, so Sigma' = Sigma and q' = q.  Averaging the
    rotation matrices instead would give diag(cos theta, cos theta, 1)."""
    th = 0.7
    fr = _frames([[0, 0, th], [0, 0, -th], [0, 0, 0]], np.tile(np.eye(3), (3, 1, 1)))
    F = np.array([[0, 1, 2]])
    mu, s, q = _one_gaussian()
    bf = np.zeros((1, 8), np.int32)
    bb = np.zeros((1, 8, 2), F32)
    bb[0, :4, 0] = 1.0              # u = 1: vertex 0
    bb[0, 4:, 1] = 1.0              # v = 1: vertex 1
    out = TR.gaussians_from_frames(fr, F, mu, q, s, bf, bb)
    np.testing.assert_allclose(out["A"][0], np.eye(3), atol=1e-15)
    np.testing.assert_allclose(cov_of(out["cov3d"]), TR._cov3d(s, q), atol=1e-15)
    qn = q[0].astype(np.float64) / np.linalg.norm(q[0].astype(np.float64))
    np.testing.assert_allclose(out["quats"][0], qn, atol=1e-15)
    # Eq. 12 interpolates the log-rotation inside a face: the edge midpoint
    # between the two vertices carries r = 0 as well
    bb1 = np.array([[[0.5, 0.5]]], F32)
    out1 = TR.gaussians_from_frames(fr, F, mu, q, s, np.zeros((1, 1), np.int32), bb1)
    np.testing.assert_allclose(out1["A"][0], np.eye(3), atol=1e-15)


def test_distinct_rotations_log_average_closed_form():
    """Three corners at a vertex with r = a x, five at one with r = b y, and
    per-vertex stretches diag(1.2, 1, 1), diag(1, 0.8, 1): R' = exp((3a x +
    5b y)/8) (scipy's rotation-vector map), S' = diag(1.075, 0.875, 1),
    A = R'S', Sigma' = A Sigma A^T, and q' is the quaternion of R' R(q)."""
    a, b = 0.9, -0.6
    S0, S1 = np.diag([1.2, 1.0, 1.0]), np.diag([1.0, 0.8, 1.0])
    fr = _frames([[a, 0, 0], [0, b, 0], [0, 0, 0]], np.stack([S0, S1, np.eye(3)]))
    F = np.array([[0, 1, 2]])
    mu, s, q = _one_gaussian()
    bf = np.zeros((1, 8), np.int32)
    bb = np.zeros((1, 8, 2), F32)
    bb[0, [0, 3, 6], 0] = 1.0
    bb[0, [1, 2, 4, 5, 7], 1] = 1.0
    out = TR.gaussians_from_frames(fr, F, mu, q, s, bf, bb)
    Rp = Rotation.from_rotvec([3 * a / 8, 5 * b / 8, 0.0]).as_matrix()
    Sp = np.diag([1.075, 0.875, 1.0])
    A = Rp @ Sp
    np.testing.assert_allclose(out["A"][0], A, atol=1e-14)
    np.testing.assert_allclose(cov_of(out["cov3d"])[0], A @ TR._cov3d(s, q)[0] @ A.T, atol=1e-15)
    qs = out["quats"][0]
    got = Rotation.from_quat([qs[1], qs[2], qs[3], qs[0]]).as_matrix()
    qq = q[0].astype(np.float64)
    ref = Rp @ Rotation.from_quat([qq[1], qq[2], qq[3], qq[0]]).as_matrix()
    np.testing.assert_allclose(got, ref, atol=1e-14)
    # same axis: the angles simply average
    fz = _frames([[0, 0, 0.4], [0, 0, -0.2], [0, 0, 0]], np.tile(np.eye(3), (3, 1, 1)))
    outz = TR.gaussians_from_frames(fz, F, mu, q, s, bf, bb)
    ang = (3 * 0.4 + 5 * -0.2) / 8
    Rz = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0], [0, 0, 1]])
    np.testing.assert_allclose(outz["A"][0], Rz, atol=1e-15)


# ---------------------------------------------------------------- unbound corners

def test_gaussian_without_bound_corners_keeps_its_rest_pose():
    """Every corner unbound (face -1, or any index outside the proxy): mu' = mu
    bit for bit, A = I, Sigma' = Sigma(s, q), q' = q / |q|."""
    V, F, mu, s, q, bf, bb = small_scene(8, seed=4, n=40)
    Vd = scenes.bend(V)
    bf = bf.copy()
    bf[:20] = -1
    bf[20:, 3] = F.shape[0]            # one past the end counts as unbound too
    bf[30:] = F.shape[0] + 7
    out = TR.transfer(V, F, Vd, mu, q, s, bf, bb)
    rest = np.r_[0:20, 30:40]
    assert np.array_equal(out["means"][rest], mu[rest])
    np.testing.assert_allclose(out["A"][rest], np.broadcast_to(np.eye(3), (rest.size, 3, 3)), atol=0)
    np.testing.assert_allclose(cov_of(out["cov3d"])[rest], TR._cov3d(s[rest], q[rest]), atol=1e-15)
    qn = q[rest].astype(np.float64)
    qn /= np.linalg.norm(qn, axis=1, keepdims=True)
    np.testing.assert_allclose(out["quats"][rest], qn, atol=1e-15)


@pytest.mark.parametrize("K", [1, 8])
def test_unbound_corners_leave_the_similarity_closed_form(K):
    """V' = s Q V + t with a random subset of corners unbound: Eq. 13 averages
    over the bound corners only, so mu' = mu + mean over bound i of
    ((sQ - I) P_i + t) (dividing by K instead would shrink the offset) and
    Sigma' = s^2 Q Sigma Q^T wherever at least one corner is bound."""
    V, F, mu, s, q, bf, bb = small_scene(K, seed=5)
    rng = np.random.default_rng(6)
    bf = bf.copy()
    drop = rng.random(bf.shape) < 0.4
    bf[drop] = -1
    scale = 1.3
    Qr = Rotation.from_rotvec([-0.2, 0.6, 0.1])
    Q = Qr.as_matrix()
    t = np.array([0.05, 0.1, -0.3])
    Vd = scale * V @ Q.T + t
    out = TR.transfer(V, F, Vd, mu, q, s, bf, bb)
    bound = bf >= 0
    kb = bound.sum(1)
    some = kb > 0
    P = bound_points(V, F, np.where(bound, bf, 0), bb)
    off = ((P @ (scale * Q - np.eye(3)).T + t) * bound[..., None]).sum(1) / np.maximum(kb, 1)[:, None]
    mu_ref = mu.astype(np.float64) + off
    np.testing.assert_allclose(out["means"][some], mu_ref[some], atol=3e-6)
    assert np.array_equal(out["means"][~some], mu[~some])
    Sig = TR._cov3d(s, q)
    ref = scale ** 2 * np.einsum("ij,njk,lk->nil", Q, Sig, Q)
    np.testing.assert_allclose(cov_of(out["cov3d"])[some], ref[some], rtol=1e-8, atol=1e-14)
    np.testing.assert_allclose(cov_of(out["cov3d"])[~some], Sig[~some], atol=1e-15)
    if K == 8:
        assert some.all() and (kb < 8).any() and (kb < 6).any()


def test_pinned_mean_with_unbound_corners_exact_rounding():
    """The float32 mean over the bound corners only: sum in corner order,
    times 1/k_b rounded to float32; re-evaluated element by element."""
    import struct

    def r32(x):
        return struct.unpack("f", struct.pack("f", x))[0]
    V, F, mu, s, q, bf, bb = small_scene(8, seed=7, n=25)
    bf = bf.copy()
    rng = np.random.default_rng(8)
    bf[rng.random(bf.shape) < 0.5] = -1
    bf[0] = -1
    Vd = V + rng.normal(0, 0.05, size=V.shape)
    d32 = np.asarray(Vd, F32) - np.asarray(V, F32)
    got = TR.pinned_mean(mu, d32, F, bf, bb)
    for n in range(25):
        kb = int((bf[n] >= 0).sum())
        for c in range(3):
            acc = None
            for i in range(8):
                if bf[n, i] < 0:
                    continue
                a, b, cc = F[bf[n, i]]
                u, v = float(bb[n, i, 0]), float(bb[n, i, 1])
                w = r32(r32(1.0 - u) - v)
                di = r32(r32(r32(u * float(d32[a, c])) + r32(v * float(d32[b, c])))
                         + r32(w * float(d32[cc, c])))
                acc = di if acc is None else r32(acc + di)
            ref = float(mu[n, c]) if kb == 0 else r32(float(mu[n, c]) + r32(acc * r32(1.0 / kb)))
            assert float(got[n, c]) == ref
