"""umgs_bind_transfer_noalloc (the allocation-free variant of the
deformation transfer, whose scratch is the library's static per-GPU array)
against umgs_bind_transfer through the C ABI: identical outputs on two calls
in a row, the second with a smaller proxy and fewer Gaussians, and the size
limit of the scratch enforced before any launch."""
import sys

import numpy as np
import pytest

from paper_2601_19233_amd import scenes

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def workload(freq, n, K, seed):
    rng = np.random.default_rng(seed)
    V, F = scenes.icosphere(freq, 1.0)
    V, F = V.astype(np.float32), F.astype(np.int32)
    mu = scenes._sample_on_mesh(rng, V.astype(np.float64), F, n, 0.02).astype(np.float32)
    s, q, _, _ = scenes._gaussian_stats(rng, n, 0)
    s, q = s.astype(np.float32), q.astype(np.float32)
    bf, bb = scenes.make_binding(mu, s, q, V, F, K)
    bf[rng.random(bf.shape) < 0.05] = -1          # a few unbound corners
    Vd = scenes.bend(V.astype(np.float64)).astype(np.float32)
    return V, F, Vd, bf, bb, mu, q, s


def outputs(r, args, noalloc, with_vertex=False):
    import torch
    V, F, Vd, bf, bb, mu, q, s = args
    out = r.bind_transfer(Vd, bf, bb, mu, q, s, with_vertex=with_vertex, noalloc=noalloc)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("K", [8, 1])
def test_noalloc_transfer_matches_the_allocating_entry_point(gpu, K):
    from paper_2601_19233_amd.render import Rasterizer
    from paper_2601_19233_amd import _lib as L
    # first call: 5,120-face proxy, 6,001 Gaussians; second: 1,280 faces, 777
    for freq, n, seed in ((16, 6001, 1), (8, 777, 2)):
        note(f"noalloc transfer K={K} freq={freq} N={n}")
        args = workload(freq, n, K, seed)
        r = Rasterizer("cuda:0", k_bind=K)
        r.set_proxy(args[0], args[1])
        for with_vertex in (False, True):
            a = outputs(r, args, False, with_vertex)
            b = outputs(r, args, True, with_vertex)
            assert a.keys() == b.keys()
            for k in a:
                assert np.array_equal(a[k], b[k]), (freq, k, with_vertex)
        r.close()
    # a proxy whose tables exceed the 16 MiB array: rejected before any
    # launch unless the caller takes the per-vertex table
    V, F = scenes.icosphere(72, 1.0)
    V, F = V.astype(np.float32), F.astype(np.int32)
    assert 144 * F.shape[0] <= 16 << 20 < 144 * F.shape[0] + 48 * V.shape[0]
    note(f"noalloc transfer over the limit faces={F.shape[0]}")
    r = Rasterizer("cuda:0", k_bind=K)
    r.set_proxy(V, F)
    mu = V[:10].copy()
    s = np.full((10, 3), 0.01, np.float32)
    q = np.tile(np.float32([1, 0, 0, 0]), (10, 1))
    bf = np.zeros((10, K), np.int32)
    bb = np.full((10, K, 2), 0.25, np.float32)
    with pytest.raises(L.UmgsError) as ei:
        r.bind_transfer(V, bf, bb, mu, q, s, noalloc=True)
    assert ei.value.status == -2          # UMGS_ERR_CAPACITY
    assert "16777216" in str(ei.value)
    a = outputs(r, (V, F, V, bf, bb, mu, q, s), False, True)
    b = outputs(r, (V, F, V, bf, bb, mu, q, s), True, True)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    r.close()
