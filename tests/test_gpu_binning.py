"""Binning on the GPU: the tile lists hold every (tile, Gaussian) pair that
the oracle finds contributing (alpha >= 1/255 at one of the tile's pixel
centres), including needle-shaped and barely visible Gaussians, and most
listed pairs do contribute (the lists are cut to each Gaussian's support, not
its bounding rectangle).
"""
import dataclasses
import sys

import numpy as np
import pytest

from paper_2601_19233_amd import scenes
from tests import _parity as PT

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def needed_pairs(fr, W, H, tw, th):
    """(tile, Gaussian) pairs with a pixel whose oracle alpha is clearly
    >= 1/255 (decisions within 1e-4 of the threshold are left out)."""
    ntx = (W + tw - 1) // tw
    need = set()
    seen = 0
    for py in range(H):
        for px in range(W):
            idx, alpha, contrib, amb, rel = fr._gauss_at(px, py, 1e-4)
            sel = idx[contrib & ~amb]
            seen += int(sel.size)
            t = (py // th) * ntx + px // tw
            need.update((t, int(g)) for g in sel)
    return need, seen


def gpu_pairs(r, N):
    from paper_2601_19233_amd import _lib as L
    k = r.copy_state(L.STATE_SORTED_KEYS).cpu().numpy().view(np.uint64)
    v = r.copy_state(L.STATE_SORTED_VALS).cpu().numpy().view(np.uint32).astype(np.int64)
    t = (k >> np.uint64(32)).astype(np.int64)
    g = v < N
    return set(zip(t[g].tolist(), v[g].tolist())), int(g.sum())


def stressed(s):
    """cfg0 with a third of the Gaussians stretched into needles (one axis
    x40) and a third barely visible (opacity just above 1/255)."""
    rng = np.random.default_rng(7)
    sc = s.scales.copy()
    op = s.opacity.copy()
    sel = rng.permutation(s.N)
    needles, faint = sel[: s.N // 3], sel[s.N // 3: 2 * (s.N // 3)]
    sc[needles, rng.integers(0, 3, needles.size)] *= 40.0
    op[faint] = (1.0 + rng.uniform(0.001, 0.2, faint.size)) / 255.0
    return dataclasses.replace(s, scales=sc.astype(np.float32), opacity=op.astype(np.float32))


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
@pytest.mark.parametrize("kind", ["cfg0", "stressed"])
def test_tile_lists_hold_every_contributing_pair(gpu, tile, kind):
    import torch
    from paper_2601_19233_amd.render import Rasterizer, scene_inputs
    s = scenes.make_config(0)
    if kind == "stressed":
        s = stressed(s)
    cam = s.cams[0]
    note(f"binning {kind} tile={tile}")
    r = Rasterizer("cuda:0", tile=tile, sh_degree=s.sh_degree)
    out = r.render([cam], **scene_inputs(s))
    torch.cuda.synchronize()
    fr = PT.oracle_frame(s, cam)
    need, seen = needed_pairs(fr, cam.width, cam.height, *tile)
    have, n_listed = gpu_pairs(r, s.N)
    missing = need - have
    assert not missing, sorted(missing)[:10]
    useful = len(have & need) / max(1, len(have))
    note(f"{kind} {tile}: listed {n_listed}, needed {len(need)}, useful fraction {useful:.3f}")
    # the image still matches the oracle
    img = r.split_views(out["image"], 3)[0].cpu().numpy()
    Tf = r.split_views(out["T_final"], 1)[0].cpu().numpy()
    px = [(x, y) for y in range(0, cam.height, 3) for x in range(0, cam.width, 3)]
    res = PT.compare_pixels(fr, img, Tf, None, px)
    assert res["ambiguous"] < 0.02 * len(px)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_per_pixel_order_is_oracle_contributor_order(gpu, tile):
    """Every pixel's front-to-back list on the GPU -- its tile's sorted list
    restricted to the fragments that contribute at the pixel -- is the
    oracle's contributor order, (FP32 key, global id), bit for bit; and the
    fragments the GPU blended are the oracle's blended prefix."""
    import torch
    from paper_2601_19233_amd import _lib as L
    from paper_2601_19233_amd.render import Rasterizer, scene_inputs
    s = scenes.make_config(0)
    cam = s.cams[0]
    note(f"per-pixel order tile={tile}")
    r = Rasterizer("cuda:0", tile=tile, sh_degree=s.sh_degree)
    out = r.render([cam], **scene_inputs(s))
    torch.cuda.synchronize()
    vals = r.copy_state(L.STATE_SORTED_VALS).cpu().numpy().view(np.uint32).astype(np.int64)
    rg = r.copy_state(L.STATE_RANGES).cpu().numpy().astype(np.int64)
    nc = r.split_views(out["n_contrib"], 1)[0].cpu().numpy()
    fr = PT.oracle_frame(s, cam)
    tw, th = tile
    ntx = (cam.width + tw - 1) // tw
    checked = 0
    for py in range(0, cam.height, 2):
        for px in range(0, cam.width, 2):
            p = fr.pixel(px, py)
            if p.ambiguous:
                continue
            t = (py // th) * ntx + px // tw
            lst = vals[rg[t, 0]:rg[t, 1]]
            want = set(p.contributors)
            got = [int(g) for g in lst if int(g) in want]
            assert got == list(p.contributors), (px, py)
            # the blended prefix ends at the GPU's last blended position
            blended_gpu = [int(g) for g in lst[: nc[py, px]] if int(g) in want]
            assert blended_gpu == list(p.order), (px, py)
            checked += 1
    assert checked > 800
    note(f"per-pixel order {tile}: {checked} pixels")
