"""Pins of the transfer gradient oracle (oracle/transfer_grad.py): its
PyTorch forward reproduces the pinned NumPy transfer, its gradient with
respect to the deformed proxy vertices matches central differences of the
NumPy transfer (whose polar factor comes from an SVD, not Newton's
iteration), and it satisfies translation invariance exactly."""
import numpy as np
import pytest
import torch

from oracle import transfer as OT
from oracle import transfer_grad as TG
from paper_2601_19233_amd import scenes


def deformed_proxy(seed, n=60, K=8, unbound=0.15):
    """An icosphere bent, twisted and stretched unevenly (rotations up to
    about 1 rad, stretches of 0.7 to 1.4), Gaussians bound by their box
    corners, some corners unbound."""
    rng = np.random.default_rng(seed)
    V, F = scenes.icosphere(3, 1.0)
    V64 = V.astype(np.float64)
    ang = 0.9 * V64[:, 1]
    c, s = np.cos(ang), np.sin(ang)
    Vd = np.stack([c * V64[:, 0] + s * V64[:, 2], V64[:, 1], -s * V64[:, 0] + c * V64[:, 2]], 1)
    Vd *= np.array([1.3, 0.8, 1.1]) * (1 + 0.15 * V64[:, :1])
    Vd += 0.1 * np.sin(2.0 * V64[:, [2, 0, 1]])
    mu = scenes._sample_on_mesh(rng, V64, F, n, 0.03).astype(np.float32)
    sc, q, _, _ = scenes._gaussian_stats(rng, n, 0)
    sc = (np.asarray(sc) * 4.0).astype(np.float32)
    q = np.asarray(q, np.float32)
    bf, bb = scenes.make_binding(mu, sc, q, V.astype(np.float32), F.astype(np.int32), K)
    bf = bf.copy()
    bf[rng.random(bf.shape) < unbound] = -1
    bf[:2] = -1                                # two Gaussians keep their rest pose
    return V.astype(np.float32), F.astype(np.int32), Vd.astype(np.float32), mu, q, sc, bf, bb


def test_torch_transfer_reproduces_the_oracle():
    V, F, Vd, mu, q, sc, bf, bb = deformed_proxy(1)
    ot = OT.transfer(V, F, Vd, mu, q, sc, bf, bb)
    m, A = TG.transfer_torch(V, F, torch.tensor(Vd.astype(np.float64)), mu, bf, bb)
    np.testing.assert_allclose(A.numpy(), ot["A"], atol=1e-11)
    np.testing.assert_allclose(m.numpy(), ot["means"], atol=2e-6)       # FP32-pinned oracle mean
    assert np.abs(ot["vertex"]["r"]).max() > 0.5


@pytest.mark.parametrize("K", [8, 1])
def test_proxy_gradient_matches_finite_differences(K):
    """Central differences (h = 1e-6) of L = <dL_dA, A> + dL_dmu . mu' with
    A from the NumPy oracle (SVD polar) and mu' from its FP64 parts."""
    V, F, Vd, mu, q, sc, bf, bb = deformed_proxy(2, K=K)
    rng = np.random.default_rng(3)
    N = mu.shape[0]
    gA = rng.normal(size=(N, 3, 3))
    gm = rng.normal(size=(N, 3))
    g = TG.proxy_gradient(V, F, Vd, mu, bf, bb, gm, gA)
    bound = OT.bound_mask(bf, F.shape[0])
    fv = F[np.where(bound, bf, 0)]
    w = np.stack([bb[..., 0], bb[..., 1], 1 - bb[..., 0] - bb[..., 1]], -1).astype(np.float64) * bound[..., None]
    kb = np.maximum(bound.sum(1), 1)

    def L(Vd64):
        vt = OT.vertex_transforms(V, F, Vd64)
        A = OT.gaussians_from_frames(vt, F, mu, q, sc, bf, bb)["A"]
        off = np.einsum("nkj,nkjc->nc", w, (Vd64 - V.astype(np.float64))[fv]) / kb[:, None]
        return float((A * gA).sum() + (off * gm).sum())

    used = np.unique(fv[bound])
    pick = rng.choice(used, 12, replace=False)
    Vd64 = Vd.astype(np.float64)
    gmax = np.abs(g).max()
    checked = 0
    for vi in pick:
        for c in range(3):
            h = 1e-6
            Vp, Vm = Vd64.copy(), Vd64.copy()
            Vp[vi, c] += h
            Vm[vi, c] -= h
            fd = (L(Vp) - L(Vm)) / (2 * h)
            assert abs(fd - g[vi, c]) <= 1e-6 * abs(fd) + 1e-8 * gmax, (vi, c, fd, g[vi, c])
            checked += 1
    assert checked == 36 and np.abs(g[pick]).min() > 0


def test_translation_invariance():
    """A moves with the proxy's shape, not its position: translating V' by t
    leaves A unchanged and moves every bound mean by t, so the vertex
    gradients sum to the bound Gaussians' mean gradients, whatever dL/dA."""
    V, F, Vd, mu, q, sc, bf, bb = deformed_proxy(4)
    rng = np.random.default_rng(5)
    N = mu.shape[0]
    gm = rng.normal(size=(N, 3))
    g = TG.proxy_gradient(V, F, Vd, mu, bf, bb, gm, rng.normal(size=(N, 3, 3)))
    anyb = OT.bound_mask(bf, F.shape[0]).any(1)
    np.testing.assert_allclose(g.sum(0), gm[anyb].sum(0), atol=1e-9)
    g0 = TG.proxy_gradient(V, F, Vd, mu, bf, bb, np.zeros((N, 3)), rng.normal(size=(N, 3, 3)))
    np.testing.assert_allclose(g0.sum(0), 0.0, atol=1e-9)


def test_uniform_scaling_has_finite_gradients():
    """Under a uniform scaling every D = s R has equal singular values, where
    an SVD's derivative is undefined; the polar factor's is not, and the
    gradient matches the scaled-identity closed case: for A = s I at every
    vertex, d<G, A>/dV' along a further uniform scaling V' -> (1 + e) V'
    equals s sum tr(G)."""
    V, F, _, mu, q, sc, bf, bb = deformed_proxy(6)
    s = 1.7
    Vd = (s * V.astype(np.float64)).astype(np.float32)
    rng = np.random.default_rng(7)
    N = mu.shape[0]
    gA = rng.normal(size=(N, 3, 3))
    g = TG.proxy_gradient(V, F, Vd, mu, bf, bb, np.zeros((N, 3)), gA)
    assert np.isfinite(g).all()
    anyb = OT.bound_mask(bf, F.shape[0]).any(1)
    lhs = float((g * Vd.astype(np.float64)).sum())
    rhs = s * float(np.trace(gA[anyb], axis1=1, axis2=2).sum())
    assert abs(lhs - rhs) <= 1e-7 * abs(rhs)
