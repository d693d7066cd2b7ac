"""Pins of the ray-cast binding oracle (Section 3.3.1) against facts that do
not come from the oracle itself: numpy's dense solver, closed-form
crossings, points on a face that must bind to it, a two-layer mesh that
separates "nearest to the target" from "first crossing", crossings behind
the camera, and the box corners of axis-aligned and rotated Gaussians."""
import numpy as np

from oracle import binding as B
from paper_2601_19233_amd import scenes


def test_cramer_solution_matches_dense_solver():
    rng = np.random.default_rng(0)
    o, d = rng.normal(size=(50, 3)), rng.normal(size=(50, 3))
    A, Bv, C = rng.normal(size=(50, 3)), rng.normal(size=(50, 3)), rng.normal(size=(50, 3))
    b, g, t = B.crossings(o, d, A, Bv, C)
    for i in range(50):
        M = np.stack([Bv[i] - A[i], C[i] - A[i], -d[i]], 1)
        ref = np.linalg.solve(M, o[i] - A[i])
        np.testing.assert_allclose([b[i], g[i], t[i]], ref, rtol=1e-9, atol=1e-12)


def test_closed_form_crossing_of_an_axis_aligned_triangle():
    # triangle in the plane z = 2 with corners (0,0), (1,0), (0,1); a ray
    # from the origin towards (0.2, 0.3, 4) crosses it at t = 1/2, (0.1, 0.15, 2)
    V = np.array([[0, 0, 2], [1, 0, 2], [0, 1, 2]], np.float64)
    F = np.array([[0, 1, 2]])
    face, bary, dist, cam = B.associate(np.array([[0.2, 0.3, 4.0]]), np.zeros((1, 3)), V, F)
    assert face[0] == 0 and cam[0] == 0
    # crossing = u V0 + v V1 + (1-u-v) V2 with V1 = (1,0), V2 = (0,1)
    np.testing.assert_allclose(bary[0], [1 - 0.1 - 0.15, 0.1], atol=1e-12)
    np.testing.assert_allclose(dist[0], 0.5 * np.linalg.norm([0.2, 0.3, 4.0]), rtol=1e-12)


def test_crossings_behind_the_camera_and_parallel_rays_do_not_count():
    V = np.array([[0, 0, -2], [1, 0, -2], [0, 1, -2]], np.float64)
    F = np.array([[0, 1, 2]])
    # the face lies behind the camera at the origin looking towards +z
    face, _, dist, _ = B.associate(np.array([[0.1, 0.1, 1.0]]), np.zeros((1, 3)), V, F)
    assert face[0] == -1 and np.isinf(dist[0])
    # a ray in the face's plane never crosses it
    face, _, _, _ = B.associate(np.array([[0.3, 0.3, -2.0]]), np.array([[-1.0, 0.3, -2.0]]), V, F)
    assert face[0] == -1


def test_points_on_a_face_bind_to_that_face_with_their_barycentrics():
    V, F = scenes.icosphere(3, 1.0)
    rng = np.random.default_rng(1)
    f = rng.integers(0, F.shape[0], 40)
    w = rng.dirichlet([4, 4, 4], 40)
    P = (w[:, 0, None] * V[F[f, 0]] + w[:, 1, None] * V[F[f, 1]] + w[:, 2, None] * V[F[f, 2]])
    cams = np.array([[0, 0, 4.0], [4.0, 0, 0], [0, -4.0, 0], [-3, 2, 2.0]])
    face, bary, dist, cam = B.associate(P, cams, V, F)
    seen = face >= 0
    # a camera sees every point of the sphere from at least one of the four
    assert seen.all()
    assert (face == f).all()
    np.testing.assert_allclose(bary, w[:, :2], atol=1e-9)
    np.testing.assert_allclose(dist, 0.0, atol=1e-9)


def test_nearest_to_target_not_first_crossing():
    # two concentric spheres: targets just outside the inner one (r = 0.5)
    # are reached from outside through the outer sphere (r = 1.0) first, yet
    # bind to the inner sphere, a few hundredths from the target (the faces
    # of the inner sphere lie up to about 0.02 inside r = 0.5) where the outer
    # crossing is at least 0.4 away
    Vo, Fo = scenes.icosphere(3, 1.0)
    Vi, Fi = scenes.icosphere(3, 0.5)
    V = np.concatenate([Vo, Vi])
    F = np.concatenate([Fo, Fi + Vo.shape[0]])
    rng = np.random.default_rng(2)
    dirs = rng.normal(size=(30, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    P = dirs * 0.505
    cams = np.array([[0, 0, 3.0], [0, 0, -3.0], [3.0, 0, 0], [-3.0, 0, 0], [0, 3.0, 0], [0, -3.0, 0]])
    face, bary, dist, _ = B.associate(P, cams, V, F)
    assert (face >= Fo.shape[0]).all()
    assert (dist < 0.05).all()
    # the crossing it reports lies on that face and on a camera ray
    Vf = V[F[face]]
    X = bary[:, :1] * Vf[:, 0] + bary[:, 1:] * Vf[:, 1] + (1 - bary.sum(1, keepdims=True)) * Vf[:, 2]
    np.testing.assert_allclose(np.linalg.norm(X - P, axis=1), dist, rtol=1e-9, atol=1e-12)


def test_equal_distances_go_to_the_lower_camera_then_the_lower_face():
    # two coincident copies of one triangle: equal crossings, lower face wins;
    # two cameras at mirrored positions see the target at equal distance
    V = np.array([[-1, -1, 0], [1, -1, 0], [0, 1, 0]], np.float64)
    F = np.array([[0, 1, 2], [0, 1, 2]])
    P = np.array([[0.0, 0.0, 0.1]])
    cams = np.array([[0.0, 0.0, -2.0], [0.0, 0.0, -2.0]])
    face, _, _, cam = B.associate(P, cams, V, F)
    assert face[0] == 0 and cam[0] == 0


def test_box_corners_axis_aligned_and_rotated():
    mu = np.array([[1.0, 2.0, 3.0]])
    s = np.array([[0.1, 0.2, 0.3]])
    q = np.array([[2.0, 0.0, 0.0, 0.0]])                  # identity, unnormalised
    P = B.target_points(mu, s, q, 8)[0]
    for k in range(8):
        sgn = np.array([1 if (k >> a) & 1 else -1 for a in range(3)])
        np.testing.assert_allclose(P[k], mu[0] + 3 * s[0] * sgn, atol=1e-12)
    # 90 degrees about z maps the local x axis to world y, local y to -x
    qz = np.array([[np.cos(np.pi / 4), 0.0, 0.0, np.sin(np.pi / 4)]])
    P = B.target_points(np.zeros((1, 3)), s, qz, 8)[0]
    np.testing.assert_allclose(P[1] - P[0], [0.0, 0.6, 0.0], atol=1e-12)   # x sign flips
    np.testing.assert_allclose(P[2] - P[0], [-1.2, 0.0, 0.0], atol=1e-12)  # y sign flips
    np.testing.assert_allclose(B.target_points(mu, s, q, 1)[0, 0], mu[0])


def test_camera_center_inverts_the_view_transform():
    rng = np.random.default_rng(3)
    R, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    c = rng.normal(size=3)
    t = -R @ c
    np.testing.assert_allclose(B.camera_center(R, t), c, atol=1e-12)
