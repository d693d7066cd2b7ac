"""Full-size workloads on the GPU, checked against the oracle on sampled
outputs.

* 1920x1080, 1M deformed Gaussians + 100,128 triangles (the benchmark frame,
  same launch configuration): pinned deformed means and depth keys of every
  primitive bit-exact; 160 sampled pixels within 1e-4 (plus the last blended
  fragment's id); sampled gradients of the backward and of the triangle
  backward (pixels drawn where triangles are blended) against the oracle
  gradient restricted to those pixels.
* 800x800, 300k Gaussians with SH degree 3 + 50,176 triangles: sampled
  pixels; gradients on four 16 x 16 windows against FP64 central finite
  differences of the forward oracle for 256 Gaussians x 17 parameters
  (tests/golden/cfg2_fd_256.json, written by tests/golden/cfg2_fd.py) and
  against the oracle gradient for every Gaussian the windows touch.
* 64 views of uneven size, 500k Gaussians (captured graph, persistent
  schedule): sampled pixels on four views, each view bit-identical to its
  plain per-view frame.
* 16 views at 1080p, 2M deformed Gaussians with SH degree 3 + 200k
  triangles (captured forward+backward graph): sampled pixels on two views;
  the batched gradients of a loss on sampled pixels of those two views
  against the oracle gradient.

Gradients: 1e-3 relative per element with an absolute floor of 1e-5 times
the largest magnitude of the same parameter array (FP32 sums of many terms
against FP64); pixels with a decision within 1e-4 (relative) of its
threshold get zero loss weight.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import grad as OG
from oracle import render as OR
from oracle import transfer as OT
from paper_2601_19233_amd import scenes
from tests import _parity as PT

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def sample_pixels(cam, n, seed):
    rng = np.random.default_rng(seed)
    return list(zip(rng.integers(0, cam.width, n).tolist(), rng.integers(0, cam.height, n).tolist()))


def dev_tensors(s):
    import torch
    dev = torch.device("cuda:0")
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    out = dict(means=f(s.means), scales=f(s.scales), quats=f(s.quats), opacity=f(s.opacity),
               sh=f(s.sh.reshape(s.N, -1)), tri_xyz=f(s.tri_xyz.reshape(s.T, 9)),
               tri_rgb=f(s.tri_rgb.reshape(s.T, 9)), tri_alpha=f(s.tri_alpha))
    if s.proxy is not None:
        out["deform"] = dict(V_def=f(s.proxy.V_def),
                             bind_face=torch.from_numpy(s.bind_face.astype(np.int32)).to(dev),
                             bind_bary=f(s.bind_bary))
    return out


def check_view(fr, r, out, v, pixels):
    """r: the Rasterizer or BatchedStep whose packed outputs these are."""
    img = r.split_views(out["image"], 3)[v].cpu().numpy()
    Tf = r.split_views(out["T_final"], 1)[v].cpu().numpy()
    return PT.compare_pixels(fr, img, Tf, None, pixels)


@pytest.fixture(scope="module")
def cfg1():
    return scenes.make_config(1)


def test_cfg1_full_frame(gpu, cfg1):
    import torch
    from paper_2601_19233_amd import _lib as L
    from paper_2601_19233_amd.render import Rasterizer
    from tests.test_gpu_forward import last_gids
    s = cfg1
    cam = s.cams[0]
    note(f"cfg1 full: N={s.N} T={s.T} {cam.width}x{cam.height}")
    d = dev_tensors(s)
    r = Rasterizer("cuda:0", tile=(16, 16), frag_batch=128)
    r.set_proxy(s.proxy.V_rest, s.proxy.faces)
    df = d["deform"]
    dt = r.bind_transfer(df["V_def"], df["bind_face"], df["bind_bary"], d["means"], d["quats"], d["scales"])
    out = r.render([cam], means=dt["means"], cov3d=dt["cov3d"], opacity=d["opacity"], sh=d["sh"],
                   tri_xyz=d["tri_xyz"], tri_rgb=d["tri_rgb"], tri_alpha=d["tri_alpha"])
    torch.cuda.synchronize()
    ot = OT.transfer(s.proxy.V_rest, s.proxy.faces, s.proxy.V_def, s.means, s.quats, s.scales,
                     s.bind_face, s.bind_bary)
    assert np.array_equal(dt["means"].cpu().numpy(), ot["means"])
    fr = OR.Frame(cam, ot["means"], s.opacity, s.sh, 0, s.tri_xyz, s.tri_rgb, s.tri_alpha, cov3d=ot["cov3d"])
    keys = r.copy_state(L.STATE_KEYS).cpu().numpy().view(np.uint32)
    live = s.opacity.astype(np.float32) * np.float32(255) > 1
    gk = np.where(fr.g.valid & live, fr.g.key.view(np.uint32), np.uint32(0xFFFFFFFF))
    tk = np.where(fr.t.valid, fr.t.key.view(np.uint32), np.uint32(0xFFFFFFFF))
    # a Gaussian whose FP32 2D covariance loses positive definiteness could be
    # culled on one side only; none may differ in its key otherwise
    g_gpu = keys[: s.N]
    both = (g_gpu != 0xFFFFFFFF) & (gk != 0xFFFFFFFF)
    assert np.array_equal(g_gpu[both], gk[both])
    assert np.sum((g_gpu == 0xFFFFFFFF) != (gk == 0xFFFFFFFF)) <= 2
    assert np.array_equal(keys[s.N:], tk)
    # order: 64 sampled tiles' lists are in the stable (oracle key, id) order
    ranges = r.copy_state(L.STATE_RANGES).cpu().numpy().astype(np.int64)
    vals = r.copy_state(L.STATE_SORTED_VALS).cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    okey = np.concatenate([fr.g.key, fr.t.key]).astype(np.float32)
    busy = np.flatnonzero(ranges[:, 1] > ranges[:, 0])
    n_checked = 0
    for t in np.random.default_rng(14).choice(busy, 64, replace=False):
        ids = vals[ranges[t, 0]:ranges[t, 1]]
        assert np.all(ids < s.N + s.T)
        gk = ids < s.N
        assert fr.g.valid[ids[gk]].all() and fr.t.valid[ids[~gk] - s.N].all()
        order = np.lexsort((ids, okey[ids]))
        assert np.array_equal(order, np.arange(ids.size)), int(t)
        assert np.unique(ids).size == ids.size
        n_checked += ids.size
    note(f"cfg1 order: 64 tiles, {n_checked} list entries in (key, id) order")
    nc = r.split_views(out["n_contrib"], 1)[0].cpu().numpy()
    lg = last_gids(r, nc)
    px = sample_pixels(cam, 160, 11)
    # bias half the samples to the proxy sphere's silhouette region, where lists are long
    px += [(int(cam.cx + 330 * np.cos(a)), int(cam.cy + 330 * np.sin(a))) for a in np.linspace(0, 6.2, 40)]
    img = r.split_views(out["image"], 3)[0].cpu().numpy()
    Tf = r.split_views(out["T_final"], 1)[0].cpu().numpy()
    res = PT.compare_pixels(fr, img, Tf, lg, px)
    note(f"cfg1 full frame: {res}")

    # gradients: dL nonzero only at 48 sampled pixels and up to 64 pixels
    # that blend triangles (the centres of 120 sampled triangles)
    note("cfg1 full backward (sampled pixels)")
    gp = sample_pixels(cam, 48, 12)
    tv = np.random.default_rng(15).choice(np.flatnonzero(fr.t.valid), 120, replace=False)
    cx = (fr.t.X[tv].astype(np.float64).mean(1) / 256).astype(int)
    cy = (fr.t.Y[tv].astype(np.float64).mean(1) / 256).astype(int)
    cand = [(int(x), int(y)) for x, y in zip(cx, cy) if 0 <= x < cam.width and 0 <= y < cam.height]
    gp += [p for p in dict.fromkeys(cand) if any(i >= s.N for i in fr.pixel(*p).order)][:64]
    assert len(gp) >= 90
    amb = [fr.pixel(x, y).margin <= 1e-4 for x, y in gp]
    rng = np.random.default_rng(13)
    w = rng.normal(size=(len(gp), 3))
    w[np.array(amb)] = 0.0
    dL = np.zeros((3, cam.height, cam.width), np.float32)
    for (x, y), wi in zip(gp, w):
        dL[:, y, x] = wi
    dLt = torch.from_numpy(dL.reshape(-1)).cuda()
    g = r.backward(dLt, out, dt["means"], d["scales"], d["quats"], d["sh"], dt["xform"])
    off = ot["means"].astype(np.float64) - s.means.astype(np.float64)
    ref = OG.gradients(cam, gp, w, s.means, s.scales, s.quats, s.opacity, s.sh, 0, s.tri_xyz,
                       s.tri_rgb, s.tri_alpha, xform=ot["A"], mean_offset=off)
    touched = np.flatnonzero(np.abs(ref["opacity"]) > 0)
    assert touched.size > 50
    for n in ("means", "scales", "quats", "opacity", "sh"):
        gg = g[n].cpu().numpy().astype(np.float64).reshape(ref[n].shape)
        rr = ref[n]
        scale = np.abs(rr).max()
        err = np.abs(gg - rr)
        bad = err > 1e-3 * np.abs(rr) + 1e-5 * scale
        assert not bad.any(), (n, int(bad.sum()), float(err.max()), float(scale))
    # triangle colour and opacity gradients of the same frame and loss
    tg = r.backward_triangles(dLt, out)
    hit = np.flatnonzero(np.abs(ref["tri_alpha"]) > 0)
    note(f"cfg1 triangle backward: {hit.size} triangles touched")
    assert hit.size > 30
    for n in ("tri_rgb", "tri_alpha"):
        gg = tg[n].cpu().numpy().astype(np.float64).reshape(ref[n].shape)
        rr = ref[n]
        scale = np.abs(rr).max()
        err = np.abs(gg - rr)
        bad = err > 1e-3 * np.abs(rr) + 1e-5 * scale
        assert not bad.any(), (n, int(bad.sum()), float(err.max()), float(scale))


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GRAD_NAMES = ("means", "scales", "quats", "opacity", "sh")


def assert_grad_close(gg, rr, name, rtol=1e-3, floor=1e-5):
    gg = np.asarray(gg, np.float64).reshape(rr.shape)
    scale = np.abs(rr).max()
    err = np.abs(gg - rr)
    bad = err > rtol * np.abs(rr) + floor * scale
    assert not bad.any(), (name, int(bad.sum()), float(err.max()), float(scale))


def clear_colours(cam, means, sh, degree, ids=None, margin=1e-5):
    """Gaussians whose SH colour channels all lie more than ``margin`` from
    the clamp at 0 (the colour is max(0, raw + 0.5), a decision that FP32
    and FP64 may take differently right at it)."""
    from oracle import sh as SH
    ids = np.arange(means.shape[0]) if ids is None else ids
    W = np.asarray(cam.R, np.float32).astype(np.float64)
    t = np.asarray(cam.t, np.float32).astype(np.float64)
    d = means[ids].astype(np.float64) + (W.T @ t)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    nc = (degree + 1) ** 2
    raw = np.einsum("nk,nkc->nc", SH.basis(d, degree), sh[ids, :nc].astype(np.float64)) + 0.5
    return np.all(np.abs(raw) > margin, axis=1)


def sub_scene(frames, pixel_sets, N, T):
    """Gaussian and triangle ids that can reach any of the listed pixels of
    the listed oracle frames (the frame's conservative pixel boxes), sorted
    ascending, so a scene of just these keeps the tie order of ids."""
    gs, ts = set(), set()
    for fr, pixels in zip(frames, pixel_sets):
        for x, y in pixels:
            gs.update(fr._gauss_at(x, y, 1e-4)[0].tolist())
            ts.update(fr._tris_at(x, y)[0].tolist())
    return np.array(sorted(gs), np.int64), np.array(sorted(ts), np.int64)


def test_cfg2_gradients_match_finite_differences(gpu):
    """800x800 SH-3 frame, loss on four 16 x 16 windows: the GPU gradient
    against FP64 central finite differences of the forward oracle for 256
    Gaussians x 17 parameters (mean, scale, quaternion, opacity, six SH
    coefficients), and against the oracle gradient for every Gaussian."""
    import torch
    from paper_2601_19233_amd.render import Rasterizer
    with open(os.path.join(GOLDEN, "cfg2_fd_256.json")) as f:
        gold = json.load(f)
    s = scenes.make_config(2)
    assert gold["workload"] == s.name
    cam = s.cams[0]
    note(f"cfg2 gradients: N={s.N} T={s.T}, {len(gold['pixels'])} window pixels")
    d = dev_tensors(s)
    r = Rasterizer("cuda:0", sh_degree=3)
    out = r.render([cam], **{k: d[k] for k in ("means", "scales", "quats", "opacity", "sh",
                                               "tri_xyz", "tri_rgb", "tri_alpha")})
    w = np.array(gold["weights"])
    dL = np.zeros((3, cam.height, cam.width), np.float32)
    for (x, y), wi in zip(gold["pixels"], w):
        dL[:, y, x] = wi
    g = r.backward(torch.from_numpy(dL.reshape(-1)).cuda(), out, d["means"], d["scales"],
                   d["quats"], d["sh"], None)
    torch.cuda.synchronize()
    gn = {k: g[k].cpu().numpy().astype(np.float64) for k in GRAD_NAMES}
    gn["sh"] = gn["sh"].reshape(s.N, 16, 3)
    # finite differences
    fd = np.array([[np.nan if v is None else v for v in row] for row in gold["fd"]])
    assert np.isfinite(fd).sum() >= 0.98 * fd.size
    # a colour channel right at its clamp is a decision FP32 may take the other way
    fd[~clear_colours(cam, s.means, s.sh, 3, np.array(gold["gaussians"]))] = np.nan
    an = np.empty_like(fd)
    for j, (name, comp) in enumerate(gold["params"]):
        for i, gid in enumerate(gold["gaussians"]):
            an[i, j] = gn[name][(gid,) + tuple(comp)]
    groups = {}
    for j, (name, _) in enumerate(gold["params"]):
        groups.setdefault(name, []).append(j)
    for name, cols in groups.items():
        a, f_ = an[:, cols], fd[:, cols]
        ok = np.isfinite(f_)
        scale = np.abs(f_[ok]).max()
        err = np.abs(a - f_)
        for fl in (1e-5, 1e-6, 1e-7):
            nb = int((ok & (err > 1e-3 * np.abs(f_) + fl * scale)).sum())
            note(f"cfg2 fd {name}: {nb} of {int(ok.sum())} beyond 1e-3 rel + {fl:g} max")
        bad = ok & (err > 1e-3 * np.abs(f_) + 1e-6 * scale)
        assert not bad.any(), (name, int(bad.sum()), float(np.nanmax(err)), float(scale))
    # the oracle gradient, every Gaussian
    live = np.any(w != 0, 1)
    px = [tuple(p) for p, l in zip(gold["pixels"], live) if l]
    ref = OG.gradients(cam, px, w[live], s.means, s.scales, s.quats, s.opacity, s.sh, 3, s.tri_xyz,
                       s.tri_rgb, s.tri_alpha)
    assert np.count_nonzero(ref["opacity"]) > 300
    clear = clear_colours(cam, s.means, s.sh, 3)
    note(f"cfg2: {int((~clear).sum())} Gaussians with a colour channel at the clamp left out")
    for n in GRAD_NAMES:
        assert_grad_close(gn[n][clear], ref[n][clear], n)


def test_cfg2_full_frame(gpu):
    import torch
    from paper_2601_19233_amd.render import Rasterizer
    s = scenes.make_config(2)
    cam = s.cams[0]
    note(f"cfg2 full: N={s.N} T={s.T}")
    d = dev_tensors(s)
    r = Rasterizer("cuda:0", sh_degree=3)
    out = r.render([cam], **{k: d[k] for k in ("means", "scales", "quats", "opacity", "sh", "tri_xyz",
                                               "tri_rgb", "tri_alpha")})
    torch.cuda.synchronize()
    fr = OR.Frame(cam, s.means, s.opacity, s.sh, 3, s.tri_xyz, s.tri_rgb, s.tri_alpha,
                  scales=s.scales, quats=s.quats)
    note(f"cfg2: {check_view(fr, r, out, 0, sample_pixels(cam, 200, 21))}")


def test_cfg3_batched_graph(gpu):
    import torch
    from paper_2601_19233_amd.batched import BatchedStep
    from paper_2601_19233_amd.render import Rasterizer
    s = scenes.make_config(3)
    note(f"cfg3 full: N={s.N} T={s.T} views={len(s.cams)}")
    d = dev_tensors(s)
    sc = {k: d[k] for k in ("means", "scales", "quats", "opacity", "sh", "tri_xyz", "tri_rgb", "tri_alpha")}
    r = Rasterizer("cuda:0", own_stream=True, tile=(16, 16), frag_batch=64, schedule=1)
    step = BatchedStep(r, s.cams, sc)
    step()
    out = step()
    torch.cuda.synchronize()
    assert not r.overflowed()
    rp = Rasterizer("cuda:0", tile=(16, 16), frag_batch=64, schedule=0)
    imgs = step.split_views(out["image"], 3)
    for v in (0, 17, 40, 63):
        # the plain per-view frame is bit-identical to the batched one
        plain = rp.render([s.cams[v]], **sc)
        torch.cuda.synchronize()
        assert torch.equal(plain["image"].view_as(imgs[v]), imgs[v]), v
        fr = OR.Frame(s.cams[v], s.means, s.opacity, s.sh, 0, s.tri_xyz, s.tri_rgb, s.tri_alpha,
                      scales=s.scales, quats=s.quats)
        note(f"cfg3 view {v} {s.cams[v].width}x{s.cams[v].height}: "
             f"{check_view(fr, step, out, v, sample_pixels(s.cams[v], 40, 30 + v))}")


def test_cfg4_batched_forward_backward(gpu):
    import torch
    from paper_2601_19233_amd.batched import BatchedStep
    from paper_2601_19233_amd.render import Rasterizer
    s = scenes.make_config(4)
    note(f"cfg4 full: N={s.N} T={s.T} views={len(s.cams)}")
    d = dev_tensors(s)
    sc = {k: d[k] for k in ("means", "scales", "quats", "opacity", "sh", "tri_xyz", "tri_rgb", "tri_alpha")}
    r = Rasterizer("cuda:0", own_stream=True, sh_degree=3, schedule=1)
    r.set_proxy(s.proxy.V_rest, s.proxy.faces)
    step = BatchedStep(r, s.cams, sc, deform=d["deform"], backward=True)
    step.prepare()
    ot = OT.transfer(s.proxy.V_rest, s.proxy.faces, s.proxy.V_def, s.means, s.quats, s.scales,
                     s.bind_face, s.bind_bary)
    views = (0, 9)
    frames = [OR.Frame(s.cams[v], ot["means"], s.opacity, s.sh, 3, s.tri_xyz, s.tri_rgb,
                       s.tri_alpha, cov3d=ot["cov3d"]) for v in views]
    # loss on 24 sampled pixels of each of the two views (zero elsewhere, so
    # the batched gradient, summed over all 16 views, sees only these)
    rng = np.random.default_rng(54)
    dL = torch.zeros_like(step.out["image"])
    gpx, gw = [], []
    for v, fr in zip(views, frames):
        cam = s.cams[v]
        px = [p for p in sample_pixels(cam, 40, 60 + v) if fr.pixel(*p).margin > 1e-4][:24]
        w = rng.normal(size=(len(px), 3))
        img = step.split_views(dL, 3)[v]
        for (x, y), wi in zip(px, w):
            img[:, y, x] = torch.tensor(wi, dtype=torch.float32)
        gpx.append(px)
        gw.append(w)
    step.set_loss_gradient(dL)
    out = step()
    torch.cuda.synchronize()
    assert not r.overflowed()
    for name, gt in step.grads.items():
        assert torch.isfinite(gt).all(), name
    for v, fr in zip(views, frames):
        note(f"cfg4 view {v}: {check_view(fr, step, out, v, sample_pixels(s.cams[v], 25, 50 + v))}")
    note(f"cfg4 groups {step.groups}")
    # oracle gradient on a scene of the primitives that reach those pixels
    gs, ts = sub_scene(frames, gpx, s.N, s.T)
    note(f"cfg4 gradient check: {gs.size} Gaussians, {ts.size} triangles reach the pixels")
    off = ot["means"][gs].astype(np.float64) - s.means[gs].astype(np.float64)
    ref = None
    for v, px, w in zip(views, gpx, gw):
        rv = OG.gradients(s.cams[v], px, w, s.means[gs], s.scales[gs], s.quats[gs], s.opacity[gs],
                          s.sh[gs], 3, s.tri_xyz[ts], s.tri_rgb[ts], s.tri_alpha[ts],
                          xform=ot["A"][gs], mean_offset=off)
        ref = rv if ref is None else {k: ref[k] + rv[k] for k in GRAD_NAMES}
    assert np.count_nonzero(ref["opacity"]) > 100
    rest = np.ones(s.N, bool)
    rest[gs] = False
    clear = np.ones(gs.size, bool)
    for v in views:
        clear &= clear_colours(s.cams[v], ot["means"], s.sh, 3, gs)
    for n in GRAD_NAMES:
        gt = step.grads[n].cpu().numpy().astype(np.float64).reshape((s.N,) + ref[n].shape[1:])
        assert_grad_close(gt[gs][clear], ref[n][clear], n)
        assert np.abs(gt[rest]).max() == 0.0, n


def test_cfg1_binding_association_sampled(gpu, cfg1):
    """Section 3.3.1 binding at the size the bench times: the frame's 1M
    Gaussians (8 box corners each) into its 20,480-face rest proxy from 8
    orbit cameras, in one call; 60 sampled Gaussians (480 targets) checked
    against the FP64 oracle one by one."""
    import torch
    from oracle import binding as OB
    from paper_2601_19233_amd.render import Rasterizer
    from tests import test_gpu_binding as TB
    s = cfg1
    rng = np.random.default_rng(7)
    cams = scenes.orbit_cameras(rng, 8, [(64, 64)] * 8)
    oc = np.stack([OB.camera_center(c.R, c.t) for c in cams]).astype(np.float32)
    note("binding association: 1M Gaussians x 8 corners x 8 cameras")
    r = Rasterizer("cuda:0", k_bind=8)
    r.set_proxy(s.proxy.V_rest, s.proxy.faces)
    dev = torch.device("cuda:0")
    means, scales, quats = (torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(dev)
                            for x in (s.means, s.scales, s.quats))
    out = r.bind_raycast(means, scales, quats, 8, oc)
    torch.cuda.synchronize()
    pick = np.random.default_rng(1).choice(s.N, 60, replace=False)
    face = out["face"].cpu().numpy()[pick].reshape(-1)
    bary = out["bary"].cpu().numpy()[pick].reshape(-1, 2).astype(np.float64)
    dist = out["dist"].cpu().numpy()[pick].reshape(-1).astype(np.float64)
    P = OB.target_points(s.means[pick], s.scales[pick], s.quats[pick], 8).reshape(-1, 3)
    clear, amb = TB.compare(P, oc, s.proxy.V_rest, s.proxy.faces, face, bary, dist)
    note(f"binding sampled: {clear} clear, {amb} ambiguous")
    assert amb <= 0.02 * (clear + amb)
    r.close()


def test_cfg1_proxy_gradient_sampled(gpu, cfg1):
    """The transfer backward at the benchmark's size (1M Gaussians, K = 8,
    the 20,480-face proxy) with dL/dmu' and dL/dA nonzero for 3,000 sampled
    Gaussians: dL/dV' against the transfer gradient oracle on those
    Gaussians (the others contribute nothing)."""
    import torch
    from oracle import transfer_grad as TG
    from paper_2601_19233_amd.render import Rasterizer
    s = cfg1
    rng = np.random.default_rng(31)
    pick = np.sort(rng.choice(s.N, 3000, replace=False))
    gm = np.zeros((s.N, 3), np.float32)
    gA = np.zeros((s.N, 9), np.float32)
    gm[pick] = rng.normal(size=(pick.size, 3))
    gA[pick] = rng.normal(size=(pick.size, 9))
    note(f"cfg1 proxy gradient: N={s.N}, {pick.size} Gaussians with a gradient")
    ref = TG.proxy_gradient(s.proxy.V_rest, s.proxy.faces, s.proxy.V_def, s.means[pick],
                            s.bind_face[pick], s.bind_bary[pick], gm[pick].astype(np.float64),
                            gA[pick].reshape(-1, 3, 3).astype(np.float64))
    d = dev_tensors(s)
    r = Rasterizer("cuda:0", tile=(16, 16), frag_batch=128)
    r.set_proxy(s.proxy.V_rest, s.proxy.faces)
    df = d["deform"]
    f = lambda a: torch.from_numpy(a).cuda()
    g = r.backward_transfer(df["V_def"], df["bind_face"], df["bind_bary"], f(gm), f(gA))
    torch.cuda.synchronize()
    gg = g.cpu().numpy().astype(np.float64)
    hit = np.abs(ref).sum(1) > 0
    assert hit.sum() > 1000
    scale = np.abs(ref).max()
    err = np.abs(gg - ref)
    bad = err > 1e-3 * np.abs(ref) + 1e-5 * scale
    assert not bad.any(), (int(bad.sum()), float(err.max()), float(scale))
    r.close()
