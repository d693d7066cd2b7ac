"""Eager frames of changing size in one context: while the frame's counts
travel to the host, the first binning level goes ahead into the buffers of
earlier frames; a frame that does not fit them is binned again once they
have grown.  Every frame must come out bit-identical to the same frame in a
fresh context (image, final transmittance, n_contrib and the sorted tile
lists), whether it fitted (smaller than an earlier frame) or not (larger
than every earlier one, so the first level runs twice)."""
import sys

import numpy as np
import pytest

from paper_2601_19233_amd import scenes

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def frame(r, scene, cam):
    import torch
    from paper_2601_19233_amd import _lib as L
    from paper_2601_19233_amd.render import scene_inputs
    out = r.render([cam], **scene_inputs(scene))
    torch.cuda.synchronize()
    keys = r.copy_state(L.STATE_SORTED_KEYS).cpu().numpy()
    vals = r.copy_state(L.STATE_SORTED_VALS).cpu().numpy()
    return dict(image=out["image"].cpu().numpy(), T=out["T_final"].cpu().numpy(),
                nc=out["n_contrib"].cpu().numpy(), keys=keys, vals=vals)


def test_eager_frames_of_changing_size_match_fresh_contexts(gpu):
    from paper_2601_19233_amd.render import Rasterizer
    s = scenes.make_config(0)
    # distance sets the duplicates: near cameras give large footprints
    dists = [3.0, 4.5, 1.6, 4.0, 1.2, 3.0]
    cams = [scenes.look_at((0.3 * d, 0.2 * d, d), 160, 120) for d in dists]
    shared = Rasterizer("cuda:0", sh_degree=s.sh_degree)
    grew = []
    for d, cam in zip(dists, cams):
        note(f"eager frame at distance {d}")
        got = frame(shared, s, cam)
        fresh = Rasterizer("cuda:0", sh_degree=s.sh_degree)
        ref = frame(fresh, s, cam)
        fresh.close()
        grew.append(len(ref["vals"]))
        for k in ref:
            assert got[k].shape == ref[k].shape, (d, k)
            assert np.array_equal(got[k], ref[k]), (d, k)
        assert shared.query()[0] == len(ref["vals"]), d
        assert not shared.overflowed(), d
    shared.close()
    note(f"duplicates per frame: {grew}")
    # the sequence had frames that fit earlier buffers and frames that grew them
    fit = [i for i in range(1, len(grew)) if grew[i] <= max(grew[:i])]
    grow = [i for i in range(1, len(grew)) if grew[i] > max(grew[:i])]
    assert fit and grow, grew
