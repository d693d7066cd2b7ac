"""Batched multi-view path: graph capture and replay, persistent schedule,
capacity reservation and the autotuner, through the C ABI on the GPU.

Every graph replay is compared with the eager result of the same inputs,
replaying several times with eager work and synchronisations in between.
"""
import sys

import numpy as np
import pytest

from paper_2601_19233_amd import scenes

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def device_scene(s):
    import torch
    dev = torch.device("cuda:0")
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    return dict(means=f(s.means), scales=f(s.scales), quats=f(s.quats), opacity=f(s.opacity),
                sh=f(s.sh.reshape(s.N, -1)), tri_xyz=f(s.tri_xyz.reshape(s.T, 9)),
                tri_rgb=f(s.tri_rgb.reshape(s.T, 9)), tri_alpha=f(s.tri_alpha))


def eager(s, cams, sc, **opts):
    from paper_2601_19233_amd.render import Rasterizer
    r = Rasterizer("cuda:0", sh_degree=s.sh_degree, **opts)
    out = r.render(cams, **sc)
    return {k: v.clone() for k, v in out.items()}


def test_graph_replay_matches_eager(gpu):
    import torch
    from paper_2601_19233_amd.batched import BatchedStep
    from paper_2601_19233_amd.render import Rasterizer
    s = scenes.make_config(3, scale=0.01, res_scale=0.15, n_views=6)
    note(f"graph replay views={[(c.width, c.height) for c in s.cams]} N={s.N}")
    sc = device_scene(s)
    ref = eager(s, s.cams, sc)
    r = Rasterizer("cuda:0", sh_degree=0, own_stream=True)
    step = BatchedStep(r, s.cams, sc)
    for k in range(3):
        out = step()
        torch.cuda.synchronize()
        assert torch.equal(out["image"], ref["image"]), k
        assert torch.equal(out["n_contrib"], ref["n_contrib"]), k
        # eager work on the stream between replays
        torch.cuda.synchronize()
        _ = (sc["means"] * 2).sum().item()
    assert not r.overflowed()
    # change an input in place: the replay must follow
    sc["opacity"].mul_(0.5)
    ref2 = eager(s, s.cams, sc)
    out = step()
    torch.cuda.synchronize()
    assert torch.equal(out["image"], ref2["image"])
    assert not torch.equal(ref2["image"], ref["image"])


def test_update_views_between_replays(gpu):
    import torch
    from paper_2601_19233_amd.batched import BatchedStep
    from paper_2601_19233_amd.render import Rasterizer
    s = scenes.make_config(0, scale=0.5)
    sc = device_scene(s)
    camA = scenes.look_at((0.0, 0.0, 3.0), 40, 30)
    camB = scenes.look_at((0.4, -0.2, 2.8), 40, 30)
    note("update_views")
    r = Rasterizer("cuda:0", own_stream=True)
    step = BatchedStep(r, [camA], sc, headroom=3.0)
    outA = step()
    torch.cuda.synchronize()
    assert torch.equal(outA["image"], eager(s, [camA], sc)["image"])
    step.update_views([camB])
    outB = step()
    torch.cuda.synchronize()
    assert torch.equal(outB["image"], eager(s, [camB], sc)["image"])


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_persistent_schedule_matches_tile_grid(gpu, tile):
    import torch
    s = scenes.make_config(3, scale=0.01, res_scale=0.15, n_views=5)
    sc = device_scene(s)
    note(f"persistent tile={tile}")
    a = eager(s, s.cams, sc, tile=tile, schedule=0)
    b = eager(s, s.cams, sc, tile=tile, schedule=1)
    assert torch.equal(a["image"], b["image"])
    assert torch.equal(a["T_final"], b["T_final"])


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_render_batched_matches_separate_calls(gpu, tile):
    """umgs_render_batched (one call, persistent blend) gives the frame of
    project + bin + sort + blend bit for bit, packed or at the caller's
    view offsets, leaving the gaps between views untouched; a second frame
    at other cameras reuses the context."""
    import torch
    from paper_2601_19233_amd.render import Rasterizer
    s = scenes.make_config(3, scale=0.01, res_scale=0.15, n_views=5)
    sc = device_scene(s)
    cams = s.cams
    note(f"render_batched tile={tile} views={[(c.width, c.height) for c in cams]}")
    ref = eager(s, cams, sc, tile=tile, schedule=0)
    r = Rasterizer("cuda:0", sh_degree=s.sh_degree, tile=tile)
    packed = r.render_batched(cams, **sc)
    torch.cuda.synchronize()
    for k in ("image", "T_final", "n_contrib", "T_entity_in"):
        assert torch.equal(packed[k], ref[k]), k
    # caller-placed views with gaps, filled with a sentinel first
    sizes = [c.width * c.height for c in cams]
    offs, o = [], 7
    for n in sizes:
        offs.append(o)
        o += n + 13
    P = o
    offs.append(P)
    out = dict(image=torch.full((3 * P,), -7.0, device="cuda:0"),
               T_final=torch.full((P,), -7.0, device="cuda:0"),
               n_contrib=torch.full((P,), -7, device="cuda:0", dtype=torch.int32),
               T_entity_in=torch.full((P,), -7.0, device="cuda:0"))
    r.render_batched(cams, view_offsets=offs, out=out, **sc)
    torch.cuda.synchronize()
    ref_pos = np.cumsum([0] + sizes)
    covered = np.zeros(P, bool)
    for v, (off, n) in enumerate(zip(offs[:-1], sizes)):
        a = int(ref_pos[v])
        covered[off:off + n] = True
        for k in ("T_final", "n_contrib", "T_entity_in"):
            assert torch.equal(out[k][off:off + n], ref[k][a:a + n]), (v, k)
        assert torch.equal(out["image"][3 * off:3 * (off + n)], ref["image"][3 * a:3 * (a + n)]), v
    gap = torch.from_numpy(~covered).to("cuda:0")
    assert bool((out["T_final"][gap] == -7.0).all())
    assert bool((out["n_contrib"][gap] == -7).all())
    gap3 = gap.repeat_interleave(3)
    assert bool((out["image"][gap3] == -7.0).all())
    # overlapping offsets are refused before any launch
    with pytest.raises(Exception):
        r.render_batched(cams[:2], view_offsets=[0, sizes[0] - 1, P], **sc)
    with pytest.raises(Exception):
        r.render_batched(cams[:2], view_offsets=[0, sizes[0], sizes[0] + sizes[1] - 1], **sc)
    # next frame: other cameras, packed
    cams2 = list(reversed(cams))
    ref2 = eager(s, cams2, sc, tile=tile, schedule=0)
    again = r.render_batched(cams2, **sc)
    torch.cuda.synchronize()
    assert torch.equal(again["image"], ref2["image"])
    assert torch.equal(again["n_contrib"], ref2["n_contrib"])


def test_reservation_overflow_is_flagged(gpu):
    import torch
    from paper_2601_19233_amd.render import Rasterizer
    s = scenes.make_config(0, scale=0.5)
    sc = device_scene(s)
    note("overflow")
    r = Rasterizer("cuda:0")
    r.render(s.cams, **sc)
    n_dup, _, _ = r.query()
    assert not r.overflowed()
    r.reserve(max(1, n_dup // 3))
    r.render(s.cams, **sc)
    torch.cuda.synchronize()
    assert r.overflowed()
    assert not r.overflowed()          # reading clears it
    r.reserve(n_dup)
    ok = r.render(s.cams, **sc)
    torch.cuda.synchronize()
    assert not r.overflowed()
    assert torch.equal(ok["image"], eager(s, s.cams, sc)["image"])


def test_graph_forward_backward_matches_eager(gpu):
    import torch
    from paper_2601_19233_amd.batched import BatchedStep
    from paper_2601_19233_amd.render import Rasterizer
    s = scenes.make_config(1, scale=0.002, res_scale=0.05)
    note(f"graph fwd+bwd deformed N={s.N} views=3")
    dev = torch.device("cuda:0")
    sc = device_scene(s)
    cams = scenes.orbit_cameras(np.random.default_rng(4), 3, [(96, 54)] * 3)
    deform = dict(V_def=torch.from_numpy(s.proxy.V_def).to(dev),
                  bind_face=torch.from_numpy(s.bind_face.astype(np.int32)).to(dev),
                  bind_bary=torch.from_numpy(s.bind_bary).to(dev))
    # eager reference
    r0 = Rasterizer("cuda:0")
    r0.set_proxy(s.proxy.V_rest, s.proxy.faces)
    dt = r0.bind_transfer(deform["V_def"], deform["bind_face"], deform["bind_bary"], sc["means"],
                          sc["quats"], sc["scales"])
    ref = r0.render(cams, means=dt["means"], cov3d=dt["cov3d"], opacity=sc["opacity"], sh=sc["sh"],
                    tri_xyz=sc["tri_xyz"], tri_rgb=sc["tri_rgb"], tri_alpha=sc["tri_alpha"])
    g = torch.Generator(device="cpu").manual_seed(0)
    dL = torch.randn(ref["image"].shape, generator=g).to(dev)
    gref = r0.backward(dL, ref, dt["means"], sc["scales"], sc["quats"], sc["sh"], dt["xform"])
    # graph
    r = Rasterizer("cuda:0", own_stream=True)
    r.set_proxy(s.proxy.V_rest, s.proxy.faces)
    step = BatchedStep(r, cams, sc, deform=deform, backward=True)
    step.prepare()
    step.set_loss_gradient(dL)
    for k in range(3):
        out = step()
        torch.cuda.synchronize()
        assert torch.equal(out["image"], ref["image"]), k
        for n in ("means", "scales", "quats", "opacity", "sh"):
            torch.testing.assert_close(step.grads[n], gref[n], rtol=1e-4,
                                       atol=1e-6 * float(gref[n].abs().max()) + 1e-12)
        _ = dL.sum().item()


def test_loss_gradient_inside_the_graph(gpu):
    """A loss gradient computed inside the captured step (L2 against a target
    image, per view group) gives the gradients of the eager forward,
    dL = 2 (I - I*), backward; replays follow a changed target."""
    import torch
    from paper_2601_19233_amd.batched import BatchedStep
    from paper_2601_19233_amd.render import Rasterizer
    s = scenes.make_config(0, scale=0.5)
    sc = device_scene(s)
    cams = scenes.orbit_cameras(np.random.default_rng(11), 3, [(40, 30), (33, 21), (48, 40)])
    note("loss gradient in graph")
    r0 = Rasterizer("cuda:0")
    ref = r0.render(cams, **sc)
    g = torch.Generator(device="cpu").manual_seed(2)
    target = torch.rand(ref["image"].shape, generator=g).to("cuda:0")
    dL = 2.0 * (ref["image"] - target)
    gref = r0.backward(dL, ref, sc["means"], sc["scales"], sc["quats"], sc["sh"], None)

    def l2_grad(img, dl, p0, p1):
        torch.sub(img, target[3 * p0:3 * p1], out=dl)
        dl.mul_(2.0)

    r = Rasterizer("cuda:0", own_stream=True)
    step = BatchedStep(r, cams, sc, backward=True, group_budget=1, loss_grad=l2_grad)
    step.prepare()
    assert len(step.groups) == 3
    for k in range(3):
        out = step()
        torch.cuda.synchronize()
        assert torch.equal(out["image"], ref["image"]), k
        assert torch.equal(step.dL, dL), k
        for n in ("means", "scales", "quats", "opacity", "sh"):
            torch.testing.assert_close(step.grads[n], gref[n], rtol=1e-4,
                                       atol=1e-6 * float(gref[n].abs().max()) + 1e-12)
        _ = target.sum().item()
    target.mul_(0.5)
    out = step()
    torch.cuda.synchronize()
    assert torch.equal(step.dL, 2.0 * (ref["image"] - target))


def test_view_groups_replay_matches_eager(gpu):
    """A budget below one view's duplicates puts every view in a group of its
    own: the captured step runs project/bin/sort/blend once per group into
    slices of the packed outputs, and the backward sums over groups."""
    import torch
    from paper_2601_19233_amd.batched import BatchedStep
    from paper_2601_19233_amd.render import Rasterizer
    s = scenes.make_config(3, scale=0.01, res_scale=0.15, n_views=5)
    note(f"view groups views={[(c.width, c.height) for c in s.cams]} N={s.N}")
    sc = device_scene(s)
    ref = eager(s, s.cams, sc)
    r = Rasterizer("cuda:0", own_stream=True)
    step = BatchedStep(r, s.cams, sc, group_budget=1)
    step.prepare()
    assert step.groups == [(v, v + 1) for v in range(5)]
    for k in range(2):
        out = step()
        torch.cuda.synchronize()
        for n in ("image", "T_final", "n_contrib"):
            assert torch.equal(out[n], ref[n]), (k, n)
        _ = sc["means"].sum().item()
    # two views a group
    dups = step.view_dup_counts
    r2 = Rasterizer("cuda:0", own_stream=True)
    step2 = BatchedStep(r2, s.cams, sc, group_budget=max(dups[0] + dups[1], dups[2] + dups[3]))
    out2 = step2()
    torch.cuda.synchronize()
    assert len(step2.groups) >= 2
    assert torch.equal(out2["image"], ref["image"])


def test_view_groups_backward_sums_over_groups(gpu):
    import torch
    from paper_2601_19233_amd.batched import BatchedStep
    from paper_2601_19233_amd.render import Rasterizer
    s = scenes.make_config(0, scale=0.5)
    sc = device_scene(s)
    cams = scenes.orbit_cameras(np.random.default_rng(9), 3, [(40, 30), (33, 21), (48, 40)])
    note("view groups backward")
    dev = torch.device("cuda:0")
    r0 = Rasterizer("cuda:0")
    ref = r0.render(cams, **sc)
    g = torch.Generator(device="cpu").manual_seed(1)
    dL = torch.randn(ref["image"].shape, generator=g).to(dev)
    gref = r0.backward(dL, ref, sc["means"], sc["scales"], sc["quats"], sc["sh"], None)
    r = Rasterizer("cuda:0", own_stream=True)
    step = BatchedStep(r, cams, sc, backward=True, group_budget=1)
    step.prepare()
    assert len(step.groups) == 3
    step.set_loss_gradient(dL)
    for k in range(2):
        out = step()
        torch.cuda.synchronize()
        assert torch.equal(out["image"], ref["image"]), k
        for n in ("means", "scales", "quats", "opacity", "sh"):
            torch.testing.assert_close(step.grads[n], gref[n], rtol=1e-4,
                                       atol=1e-6 * float(gref[n].abs().max()) + 1e-12)


def test_autotuner_picks_and_caches(gpu, tmp_path, monkeypatch):
    from paper_2601_19233_amd import autotune
    monkeypatch.setenv("UMGS_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    s = scenes.make_config(3, scale=0.004, res_scale=0.1, n_views=4)
    sc = device_scene(s)
    note("autotune")
    best = autotune.tune(s.cams, sc, batches=(64, 128), reps=2)
    assert best["tile"] in [tuple(t) for t in autotune.TILES]
    assert best["frag_batch"] in (64, 128) and best["schedule"] in (0, 1)
    assert len(best["results"]) == 3 * 2 * 2
    again = autotune.tune(s.cams, sc, batches=(64, 128), reps=2)
    assert again["cached"] and again["tile"] == best["tile"]


def test_graph_triangle_and_proxy_gradients_match_eager(gpu):
    """The captured training step with the triangles' colour and opacity
    gradients and the deformed proxy's vertex gradient: every replay equals
    the eager calls on the same inputs (replays separated by eager work)."""
    import torch
    from paper_2601_19233_amd.batched import BatchedStep
    from paper_2601_19233_amd.render import Rasterizer
    s = scenes.make_config(1, scale=0.002, res_scale=0.05)
    note(f"graph fwd+bwd with triangle and proxy gradients N={s.N} T={s.T} views=3")
    dev = torch.device("cuda:0")
    sc = device_scene(s)
    cams = scenes.orbit_cameras(np.random.default_rng(4), 3, [(96, 54)] * 3)
    deform = dict(V_def=torch.from_numpy(s.proxy.V_def).to(dev),
                  bind_face=torch.from_numpy(s.bind_face.astype(np.int32)).to(dev),
                  bind_bary=torch.from_numpy(s.bind_bary).to(dev))
    r0 = Rasterizer("cuda:0")
    r0.set_proxy(s.proxy.V_rest, s.proxy.faces)
    dt = r0.bind_transfer(deform["V_def"], deform["bind_face"], deform["bind_bary"], sc["means"],
                          sc["quats"], sc["scales"])
    ref = r0.render(cams, means=dt["means"], cov3d=dt["cov3d"], opacity=sc["opacity"], sh=sc["sh"],
                    tri_xyz=sc["tri_xyz"], tri_rgb=sc["tri_rgb"], tri_alpha=sc["tri_alpha"])
    g = torch.Generator(device="cpu").manual_seed(0)
    dL = torch.randn(ref["image"].shape, generator=g).to(dev)
    gref = r0.backward(dL, ref, dt["means"], sc["scales"], sc["quats"], sc["sh"], dt["xform"])
    tref = r0.backward_triangles(dL, ref)
    vref = r0.backward_transfer(deform["V_def"], deform["bind_face"], deform["bind_bary"],
                                gref["means"], gref["xform"])
    torch.cuda.synchronize()
    assert float(tref["tri_alpha"].abs().max()) > 0 and float(vref.abs().max()) > 0
    r = Rasterizer("cuda:0", own_stream=True)
    r.set_proxy(s.proxy.V_rest, s.proxy.faces)
    step = BatchedStep(r, cams, sc, deform=deform, backward=True, triangle_grads=True, proxy_grads=True)
    step.prepare()
    step.set_loss_gradient(dL)
    for k in range(3):
        step()
        torch.cuda.synchronize()
        for n in ("tri_rgb", "tri_alpha"):
            torch.testing.assert_close(step.tgrads[n], tref[n], rtol=1e-4,
                                       atol=1e-6 * float(tref[n].abs().max()) + 1e-12)
        torch.testing.assert_close(step.vgrad, vref, rtol=1e-4, atol=1e-6 * float(vref.abs().max()))
        _ = dL.sum().item()
