#!/usr/bin/env python3
"""Benchmark of the mixed Gaussian/triangle rasterizer on one MI355X.

Workload (default): one 1920x1080 view of 1M Gaussians bound (8 bounding-box
corners each) to a 20,480-face proxy sphere bent by 0.2 sin(2 pi x), plus
100,128 occluder triangles.  One step = the whole hot path on that frame:
per-vertex proxy transforms and per-Gaussian deformation transfer, Gaussian
projection and triangle set-up, binning, the (tile, depth) radix sort and the
front-to-back blend.  Inputs are resident in device memory before timing.

Also measured: the forward+backward step on the same frame (gradients to
every Gaussian parameter through the deformation); an 800x800 frame of 300k
SH-3 Gaussians and 50k triangles, forward + backward of an L2 loss; 64 views
of uneven size (500k Gaussians) in one captured graph with the persistent
blend against rendering them one by one; and the batched training step -- 16
views at 1920x1080 of 2M SH-3 Gaussians bound to a deformed 50k-face proxy
with 200k triangles, one captured graph per step (forward, and forward +
backward), blend launch autotuned -- against the plain per-view forward,
and the same batched step on the 1M-Gaussian scene from 16 orbit cameras.
Every backward differentiates an L2 loss against the render of perturbed
parameters.

Prints ONE JSON line (metric, value = forward Mpixels/s, roofline of the
dominant kernel measured live with HIP events, CPU-oracle baseline).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixels/s forward and fwd+bwd at 1080p, 1M Gaussians + 100k tris; batched vs plain"
HBM_PEAK_GBS = 8000.0
# VALU lane-instructions per second with packed FP32 disabled:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_GOPS = 256 * 4 * 16 * 2.4
# VALU lane-operations per evaluated (pixel, fragment) pair of the blend:
# a Gaussian costs 14 to evaluate alpha (2 sub, 4 mul, 2 fma, exp with its
# scale, min, 2 compares) and 7 more when it is blended; a triangle about 60
# (FP64 edge functions with the quick reject/accept tests, the per-sample
# tests when the pixel straddles an edge, colour and the entity update).
OPS_PER_GAUSS_PAIR = 20
OPS_PER_TRI_PAIR = 60
# ... and per (pixel, fragment) pair the backward walks: a Gaussian costs 51
# (alpha again 14; T in front of it 3: 1 - alpha, reciprocal, product;
# dL/dalpha 7; the colour behind it 6; colour terms 4; power and opacity
# terms 8; the 9 terms added into the tile's sums 9), a triangle 96 (its
# coverage and colour as in the forward, 60, and the reverse recursion of
# the four sub-samples' colour and transmittance, 9 each).
OPS_PER_GAUSS_PAIR_BWD = 51
OPS_PER_TRI_PAIR_BWD = 96
# ... and per pair of the triangle backward's walk (from each pixel's last
# blended fragment down to its tile's first triangle): a Gaussian costs 23
# (alpha 14, T in front 3, the colour behind 6), a triangle 126 (its walk
# step as in the backward, 96, and its gradient: the four sub-samples'
# visibility and colour terms 16, the 10 products added to the tile's
# accumulators 14); the closing re-walk of each entity is extra work, not
# counted.
OPS_PER_GAUSS_PAIR_TRI_BWD = 23
OPS_PER_TRI_PAIR_TRI_BWD = 126


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


TRAFFIC_TABLE = os.path.join(ROOT, "profiles", "traffic_1080p_1m_gaussians_100k_tris.md")


def measured_traffic():
    """HBM bytes per launch from the committed hardware-counter table, for
    the kernels whose sources still hash to what was profiled."""
    import hashlib
    out = {}
    try:
        lines = open(TRAFFIC_TABLE).read().splitlines()
    except OSError:
        return out
    for ln in lines:
        cells = [c.strip() for c in ln.strip().strip("|").split("|")]
        if len(cells) != 6 or not cells[3].isdigit():
            continue
        kernel, _, _, nbytes, srcs, sha = cells
        h = hashlib.sha256()
        try:
            for s in srcs.split():
                with open(os.path.join(ROOT, "paper_2601_19233_amd", s), "rb") as f:
                    h.update(f.read())
        except OSError:
            continue
        if h.hexdigest()[:16] == sha:
            out[kernel] = int(nbytes)
    return out


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


_CB = {}


def _cb_pixels(chunk):
    fr = _CB["frame"]
    for x, y in chunk:
        fr.pixel(x, y)
    return len(chunk)


def cpu_baseline(scene, single_pixels=300, per_worker=120, seed=0):
    """Time the CPU FP64 oracle on a bounded sample of the same frame: the
    frame set-up (transfer and projection of every primitive, one thread),
    then pixels blended by one thread and by one process per host core (at
    most 16, the host share of one GPU), extrapolated to the whole frame.
    Runs before the GPU is initialised, so the worker processes are plain
    forks of a CPU-only process."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle import render as OR
    from oracle import transfer as OT
    cam = scene.cams[0]
    workers = max(1, min(16, os.cpu_count() or 1))
    rng = np.random.default_rng(seed)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ot = OT.transfer(scene.proxy.V_rest, scene.proxy.faces, scene.proxy.V_def, scene.means,
                         scene.quats, scene.scales, scene.bind_face, scene.bind_bary)
        fr = OR.Frame(cam, ot["means"], scene.opacity, scene.sh, scene.sh_degree, scene.tri_xyz,
                      scene.tri_rgb, scene.tri_alpha, cov3d=ot["cov3d"])
        t_setup = time.perf_counter() - t0
        px = list(zip(rng.integers(0, cam.width, single_pixels).tolist(),
                      rng.integers(0, cam.height, single_pixels).tolist()))
        t1 = time.perf_counter()
        for x, y in px:
            fr.pixel(x, y)
        t_pix1 = (time.perf_counter() - t1) / single_pixels
    npix = cam.width * cam.height
    full1 = t_setup + t_pix1 * npix
    n_par = workers * per_worker
    pxp = list(zip(rng.integers(0, cam.width, n_par).tolist(),
                   rng.integers(0, cam.height, n_par).tolist()))
    _CB["frame"] = fr
    ctx = mp.get_context("fork")
    with threadpool_limits(limits=1):
        with ctx.Pool(workers) as pool:
            pool.map(_cb_pixels, [pxp[:workers]], chunksize=1)      # start the workers
            t2 = time.perf_counter()
            done = sum(pool.map(_cb_pixels, [pxp[i::workers] for i in range(workers)], chunksize=1))
            t_parw = time.perf_counter() - t2
    _CB.clear()
    t_pixp = t_parw / done
    full = t_setup + t_pixp * npix
    return {"value": npix / full / 1e6, "unit": "Mpixels/s", "cores": workers, "kind": "oracle",
            "cpu": cpu_model(), "host_cpus": os.cpu_count(),
            "single_thread_value": npix / full1 / 1e6,
            "sample": f"frame set-up (transfer + projection of all primitives, one thread, "
                      f"{t_setup:.1f} s) plus {done} uniformly sampled pixels blended by {workers} "
                      f"processes ({t_parw:.1f} s wall, {t_pixp * 1e3:.2f} ms/pixel), extrapolated "
                      f"to {cam.width}x{cam.height}: {full:.0f} s per frame; one thread: "
                      f"{single_pixels} pixels at {t_pix1 * 1e3:.1f} ms/pixel, {full1:.0f} s per frame"}


def device_scene(s, dev):
    import torch
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    out = dict(means=f(s.means), scales=f(s.scales), quats=f(s.quats), opacity=f(s.opacity),
               sh=f(s.sh.reshape(s.N, -1)), tri_xyz=f(s.tri_xyz.reshape(s.T, 9)),
               tri_rgb=f(s.tri_rgb.reshape(s.T, 9)), tri_alpha=f(s.tri_alpha))
    deform = None
    if s.proxy is not None:
        deform = dict(V_def=f(s.proxy.V_def),
                      bind_face=torch.from_numpy(s.bind_face.astype(np.int32)).to(dev),
                      bind_bary=f(s.bind_bary))
    return out, deform


def timed(fn, steps):
    """Average wall-clock ms of fn over `steps` calls after one untimed call,
    bracketed by device synchronisation (covers every stream)."""
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def algorithmic_bytes(r, scene, n_dup, n_rec, views=1):
    """Algorithmic HBM bytes per launch of the bandwidth-bound kernels (n1
    supertile entries; their ids are 16-bit while a frame has at most 2^16
    supertiles)."""
    n_st, n1 = r.query_bins()
    kb = 2.0 if n_st <= 65536 else 4.0
    out = {
        # first level: per record its order, offsets and rectangle; per entry
        # its supertile id and record id
        "emit_keys": 28.0 * n_rec + (kb + 4.0) * n1,
        "sort_downsweep": 2.0 * (kb + 12.0) * n1,  # read and write id, record id, mask
        "sort_upsweep": kb * n1,                   # read the ids
        # masks: per entry its supertile id, record id, rectangle and
        # Gaussian record read, the mask written
        "st_mask": (kb + 4.0 + 8.0 + 48.0 + 8.0) * n1,
        # counts: the sorted masks read
        "tile_count": 8.0 * n1,
        # per entry its mask and record id; per duplicate one record id written
        "tile_scatter": 12.0 * n1 + 4.0 * n_dup,
        "project_gaussians": views * scene.N * (12 + 24 + 4 + 12 * (scene.sh_degree + 1) ** 2
                                                + 4 + 8 + 8 + 48.0),
    }
    if scene.proxy is not None:
        out["transfer"] = scene.N * (40.0 + 12.0 * scene.bind_face.shape[1] + 88.0)
    return out, n1


def kernel_rooflines(prof, algo_bytes, traffic=None, pairs=None, bpairs=None, tpairs=None):
    """Roofline entry per timed kernel: algorithmic work per launch over the
    launch's average duration (the library's HIP events on its stream)."""
    traffic = traffic or {}
    per_launch = {k: v[1] / v[0] for k, v in prof.items()}

    def one(k):
        if k in algo_bytes:
            ach = algo_bytes[k] / (per_launch[k] * 1e-3) / 1e9
            return {"kernel": k, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic.get(k),
                    "ms_per_launch": round(per_launch[k], 4)}
        if k == "blend" and pairs is not None:
            g, t = pairs["gauss"], pairs["tri"]
            ops = OPS_PER_GAUSS_PAIR * g + OPS_PER_TRI_PAIR * t
            ach = ops / (per_launch[k] * 1e-3) / 1e9
            return {"kernel": k, "bound": "alu", "achieved": round(ach, 1), "peak": VALU_PEAK_GOPS,
                    "unit": "Gop/s", "frac": round(ach / VALU_PEAK_GOPS, 4), "traffic": traffic.get(k),
                    "ms_per_launch": round(per_launch[k], 4), "gauss_pairs": g, "tri_pairs": t,
                    "wave_iters": pairs["wave_iters"], "staged_fragments": pairs["staged"],
                    "lane_occupancy": round((g + t) / max(1, 64 * pairs["wave_iters"]), 4)}
        if k == "blend_backward" and bpairs is not None:
            g, t = bpairs["gauss"], bpairs["tri"]
            ops = OPS_PER_GAUSS_PAIR_BWD * g + OPS_PER_TRI_PAIR_BWD * t
            ach = ops / (per_launch[k] * 1e-3) / 1e9
            return {"kernel": k, "bound": "alu", "achieved": round(ach, 1), "peak": VALU_PEAK_GOPS,
                    "unit": "Gop/s", "frac": round(ach / VALU_PEAK_GOPS, 4), "traffic": traffic.get(k),
                    "ms_per_launch": round(per_launch[k], 4), "gauss_pairs": g, "tri_pairs": t}
        if k == "blend_backward_tri" and tpairs is not None:
            g, t = tpairs["gauss"], tpairs["tri"]
            ops = OPS_PER_GAUSS_PAIR_TRI_BWD * g + OPS_PER_TRI_PAIR_TRI_BWD * t
            ach = ops / (per_launch[k] * 1e-3) / 1e9
            return {"kernel": k, "bound": "alu", "achieved": round(ach, 1), "peak": VALU_PEAK_GOPS,
                    "unit": "Gop/s", "frac": round(ach / VALU_PEAK_GOPS, 4), "traffic": traffic.get(k),
                    "ms_per_launch": round(per_launch[k], 4), "gauss_pairs": g, "tri_pairs": t}
        return None

    out = {}
    for k in prof:
        e = one(k)
        if e is not None:
            out[k] = e
    return out


def run_batched(args):
    """16 views at 1920x1080 of a 2M-Gaussian SH-3 scene bound to a deformed
    50k-face proxy, 200k triangles (plus the same step on the 1M-Gaussian
    1080p scene seen from 16 orbit cameras): rendering the views one by one
    (eager, forward only) against the batched step captured in one HIP graph
    (forward, and forward + backward of the L2 loss against the render of
    perturbed parameters, gradients to every Gaussian parameter), blend
    launch autotuned."""
    from paper_2601_19233_amd import scenes
    t0 = time.time()
    s = scenes.make_config(4, scale=args.scale, res_scale=args.res_scale)
    log(f"batched scene {s.name}: N={s.N} T={s.T} views={len(s.cams)} in {time.time() - t0:.1f} s")
    return batched_leg(s, s.cams, s.name, args)


def run_batched_orbit(args, scene):
    """The 1080p, 1M-Gaussian frame's scene from 16 orbit cameras (direction
    uniform on the sphere, distance U[2.5, 4]), batched against plain."""
    from paper_2601_19233_amd import scenes
    rng = np.random.default_rng(1001)
    cam0 = scene.cams[0]
    cams = scenes.orbit_cameras(rng, 16, [(cam0.width, cam0.height)] * 16)
    return batched_leg(scene, cams, scene.name + "_x16_orbit", args)


def batched_leg(s, cams, name, args):
    import torch
    from paper_2601_19233_amd import autotune, scenes
    from paper_2601_19233_amd.batched import BatchedStep
    from paper_2601_19233_amd.render import Rasterizer
    dev = torch.device("cuda:0")
    V = len(cams)
    W, H = cams[0].width, cams[0].height
    sc, deform = device_scene(s, dev)
    k_bind = int(s.bind_face.shape[1])
    r0 = Rasterizer("cuda:0", sh_degree=s.sh_degree, k_bind=k_bind)
    r0.set_proxy(s.proxy.V_rest, s.proxy.faces)
    dt = r0.bind_transfer(deform["V_def"], deform["bind_face"], deform["bind_bary"], sc["means"],
                          sc["quats"], sc["scales"])
    tsc = dict(means=dt["means"], cov3d=dt["cov3d"], opacity=sc["opacity"], sh=sc["sh"],
               tri_xyz=sc["tri_xyz"], tri_rgb=sc["tri_rgb"], tri_alpha=sc["tri_alpha"])
    t0 = time.time()
    # tuned on the first four views (one frame of them fits the key buffers at
    # every tile shape); the step itself renders all views in budgeted groups
    best = autotune.tune(cams[:4], tsc, sh_degree=s.sh_degree, k_bind=k_bind, reps=2,
                         batches=(32, 64, 128), use_cache=False)
    log(f"autotune {best['tile']} batch {best['frag_batch']} schedule {best['schedule']} "
        f"in {time.time() - t0:.1f} s")
    del r0, dt, tsc
    steps = max(2, min(args.steps, 5))
    # plain: the same views one at a time, deformation once per step
    rp = Rasterizer("cuda:0", sh_degree=s.sh_degree, k_bind=k_bind)
    rp.set_proxy(s.proxy.V_rest, s.proxy.faces)

    def plain_views():
        d = rp.bind_transfer(deform["V_def"], deform["bind_face"], deform["bind_bary"], sc["means"],
                             sc["quats"], sc["scales"])
        for c in cams:
            rp.project([c], means=d["means"], cov3d=d["cov3d"], opacity=sc["opacity"], sh=sc["sh"],
                       tri_xyz=sc["tri_xyz"], tri_rgb=sc["tri_rgb"], tri_alpha=sc["tri_alpha"])
            rp.bin()
            rp.sort()
            rp.blend(want_state=False)

    ms_plain = timed(plain_views, steps)
    del rp
    torch.cuda.empty_cache()
    res = {"workload": name, "views": V, "width": W, "height": H, "gaussians": s.N,
           "triangles": s.T, "sh_degree": s.sh_degree, "tile": "%dx%d" % best["tile"],
           "frag_batch": best["frag_batch"], "schedule": ["tile_grid", "persistent"][best["schedule"]],
           "plain_fwd_views_s": round(V / (ms_plain * 1e-3), 2),
           "plain_fwd_ms_per_step": round(ms_plain, 3),
           "loss": "L2 against the batched render of N(0, 0.01)-perturbed parameters"}
    target = None
    for bwd in (False, True):
        rb = Rasterizer("cuda:0", sh_degree=s.sh_degree, k_bind=k_bind, tile=best["tile"],
                        frag_batch=best["frag_batch"], schedule=best["schedule"], own_stream=True)
        rb.set_proxy(s.proxy.V_rest, s.proxy.faces)
        if bwd:
            # target frame: the same step on perturbed parameters, rendered once
            tsc, _ = device_scene(scenes.perturbed(s, seed=1000 + 4), dev)
            tstep = BatchedStep(rb, cams, tsc, deform=deform)
            tstep.prepare()
            target = tstep()["image"].clone()
            torch.cuda.synchronize()
            del tstep, tsc
            rb.close()
            rb = Rasterizer("cuda:0", sh_degree=s.sh_degree, k_bind=k_bind, tile=best["tile"],
                            frag_batch=best["frag_batch"], schedule=best["schedule"], own_stream=True)
            rb.set_proxy(s.proxy.V_rest, s.proxy.faces)
        def l2_grad(img, dl, p0, p1):
            torch.sub(img, target[3 * p0:3 * p1], out=dl)
            dl.mul_(2.0)

        step = BatchedStep(rb, cams, sc, deform=deform, backward=bwd,
                           loss_grad=l2_grad if bwd else None)
        step.prepare()
        ms = timed(step, steps)
        if rb.overflowed():
            raise RuntimeError("batched step overflowed its reserved key capacity")
        key = "fwd_bwd" if bwd else "fwd"
        if len(step.groups) == 1:
            # the same step once more, eagerly, with the kernels timed (a
            # captured graph cannot be), for the rooflines of this step
            rb.set_profiling(True)
            step._step()
            prof = rb.profile()
            rb.set_profiling(False)
            n_dup_b, _, n_rec_b = rb.query()
            ab, _ = algorithmic_bytes(rb, s, n_dup_b, n_rec_b, views=V)
            pairs = rb.blend_pairs()
            bp = rb.backward_pairs(step.out["n_contrib"]) if bwd else None
            rl = kernel_rooflines(prof, ab, None, pairs, bp)
            res[f"{key}_rooflines"] = {k: rl[k] for k in ("blend", "blend_backward", "tile_scatter",
                                                         "transfer") if k in rl}
            res[f"{key}_kernel_ms"] = {k: round(v[1], 4) for k, v in prof.items()}
        res[f"{key}_views_s"] = round(V / (ms * 1e-3), 2)
        res[f"{key}_mpix_s"] = round(V * W * H / (ms * 1e-3) / 1e6, 2)
        res[f"{key}_ms_per_step"] = round(ms, 3)
        res["n_dup"] = int(step.n_dup_seen)
        res["groups"] = [list(g) for g in step.groups]
        log(f"batched {name} {key}: {ms:.2f} ms per {V}-view step")
        del step, rb
        torch.cuda.empty_cache()
    # the whole training step: also the triangles' colour and opacity
    # gradients and the deformed proxy's vertex gradient, in the same graph
    rb = Rasterizer("cuda:0", sh_degree=s.sh_degree, k_bind=k_bind, tile=best["tile"],
                    frag_batch=best["frag_batch"], schedule=best["schedule"], own_stream=True)
    rb.set_proxy(s.proxy.V_rest, s.proxy.faces)

    def l2_grad_all(img, dl, p0, p1):
        torch.sub(img, target[3 * p0:3 * p1], out=dl)
        dl.mul_(2.0)

    step = BatchedStep(rb, cams, sc, deform=deform, backward=True, loss_grad=l2_grad_all,
                       triangle_grads=True, proxy_grads=True)
    step.prepare()
    ms = timed(step, steps)
    if rb.overflowed():
        raise RuntimeError("batched step overflowed its reserved key capacity")
    res["fwd_bwd_all_views_s"] = round(V / (ms * 1e-3), 2)
    res["fwd_bwd_all_ms_per_step"] = round(ms, 3)
    res["fwd_bwd_all_path"] = ("forward + backward with the Gaussians', the triangles' (colour, "
                               "opacity) and the proxy vertices' gradients, one graph")
    log(f"batched {name} fwd_bwd_all: {ms:.2f} ms per {V}-view step")
    del step, rb
    torch.cuda.empty_cache()
    res["fwd_bwd_vs_plain_fwd"] = round(res["fwd_bwd_views_s"] / res["plain_fwd_views_s"], 3)
    return res


def run_uneven(args):
    """64 orbit views of uneven size (256^2 .. 1920x1080 log-uniform area) of
    a 500k-Gaussian scene: one captured graph with the persistent
    longest-first blend against the views rendered one by one."""
    import torch
    from paper_2601_19233_amd import scenes
    from paper_2601_19233_amd.batched import BatchedStep
    from paper_2601_19233_amd.render import Rasterizer
    dev = torch.device("cuda:0")
    s = scenes.make_config(3, scale=args.scale, res_scale=args.res_scale)
    sc, _ = device_scene(s, dev)
    cams = s.cams
    npix = sum(c.width * c.height for c in cams)
    steps = max(2, min(args.steps, 5))
    rp = Rasterizer("cuda:0", sh_degree=s.sh_degree)

    def plain():
        for c in cams:
            rp.project([c], **sc)
            rp.bin()
            rp.sort()
            rp.blend(want_state=False)

    ms_plain = timed(plain, steps)
    del rp
    torch.cuda.empty_cache()
    from paper_2601_19233_amd import autotune
    # tuned on 8 views spread over the size range (one frame of them fits the
    # key buffers at every tile shape); the step renders all 64
    order = sorted(range(len(cams)), key=lambda v: cams[v].width * cams[v].height)
    probe = [cams[order[i]] for i in np.linspace(0, len(cams) - 1, 8).astype(int)]
    t0 = time.time()
    best = autotune.tune(probe, sc, sh_degree=s.sh_degree, reps=2, batches=(32, 64, 128, 256),
                         use_cache=False)
    log(f"uneven autotune {best['tile']} batch {best['frag_batch']} schedule {best['schedule']} "
        f"in {time.time() - t0:.1f} s")
    torch.cuda.empty_cache()
    rb = Rasterizer("cuda:0", sh_degree=s.sh_degree, tile=best["tile"], frag_batch=best["frag_batch"],
                    schedule=best["schedule"], own_stream=True)
    step = BatchedStep(rb, cams, sc)
    step.prepare()
    ms = timed(step, steps)
    if rb.overflowed():
        raise RuntimeError("batched step overflowed its reserved key capacity")
    res = {"workload": s.name, "views": len(cams), "pixels": npix, "gaussians": s.N, "triangles": s.T,
           "plain_views_s": round(len(cams) / (ms_plain * 1e-3), 2),
           "batched_views_s": round(len(cams) / (ms * 1e-3), 2),
           "batched_mpix_s": round(npix / (ms * 1e-3) / 1e6, 2),
           "tile": "%dx%d" % best["tile"], "frag_batch": best["frag_batch"],
           "schedule": ["tile_grid", "persistent"][best["schedule"]],
           "plain_config": "16x16 tiles, batch 128, one workgroup per tile, eager per-view calls",
           "groups": [list(g) for g in step.groups]}
    log(f"uneven: plain {ms_plain:.2f} ms, batched {ms:.2f} ms per {len(cams)}-view step")
    del step, rb
    torch.cuda.empty_cache()
    return res


def run_backward_800(args):
    """800x800, 300k Gaussians with SH degree 3 and 50k triangles: one
    forward + backward step of the L2 loss against the image rendered from
    parameters perturbed by N(0, 0.01)."""
    import torch
    from paper_2601_19233_amd import scenes
    from paper_2601_19233_amd.render import Rasterizer
    dev = torch.device("cuda:0")
    s = scenes.make_config(2, scale=args.scale, res_scale=args.res_scale)
    cam = s.cams[0]
    sc, _ = device_scene(s, dev)
    tgt_sc, _ = device_scene(scenes.perturbed(s, seed=102), dev)
    r = Rasterizer("cuda:0", sh_degree=s.sh_degree)
    target = r.render([cam], **tgt_sc)["image"].clone()
    state = {}

    def step():
        out = r.render([cam], **sc)
        dL = 2.0 * (out["image"] - target)
        state["g"] = r.backward(dL, out, sc["means"], sc["scales"], sc["quats"], sc["sh"], None)

    steps = max(2, min(args.steps, 10))
    ms = timed(step, steps)
    npix = cam.width * cam.height
    log(f"backward 800: {ms:.3f} ms per forward+backward step")
    return {"workload": s.name, "width": cam.width, "height": cam.height, "gaussians": s.N,
            "triangles": s.T, "sh_degree": s.sh_degree, "fwd_bwd_ms_per_step": round(ms, 4),
            "fwd_bwd_mpix_s": round(npix / (ms * 1e-3) / 1e6, 2),
            "loss": "L2 against the render of N(0, 0.01)-perturbed parameters"}


def run_binding(args, scene, n_cams=8):
    """Section 3.3.1 binding association at the frame's full size: the
    frame's Gaussians (8 box corners each) against its rest proxy, rays from
    n_cams orbit camera centres; one call = BVH build + cast + readback."""
    import torch
    from paper_2601_19233_amd import scenes
    from paper_2601_19233_amd.render import Rasterizer
    rng = np.random.default_rng(7)
    cams = scenes.orbit_cameras(rng, n_cams, [(64, 64)] * n_cams)
    oc = np.stack([-(c.R.astype(np.float64).T @ c.t.astype(np.float64)) for c in cams])
    oc = oc.astype(np.float32)
    r = Rasterizer("cuda:0", k_bind=8)
    r.set_proxy(scene.proxy.V_rest, scene.proxy.faces)
    dev = torch.device("cuda:0")
    means, scales, quats = (torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(dev)
                            for x in (scene.means, scene.scales, scene.quats))
    state = {}

    def call():
        state["out"] = r.bind_raycast(means, scales, quats, 8, oc)

    ms = timed(call, max(2, min(args.steps, 10)))
    unbound = float((state["out"]["face"] < 0).float().mean().item())
    rays = scene.N * 8 * n_cams
    log(f"binding: {ms:.3f} ms for {rays} rays")
    r.close()
    return {"workload": f"{scene.N} Gaussians x 8 box corners x {n_cams} cameras, "
                        f"{scene.proxy.faces.shape[0]}-face proxy",
            "ms_per_call": round(ms, 4), "rays_per_s": round(rays / (ms * 1e-3), 1),
            "unbound_fraction": round(unbound, 6)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0, help="primitive-count scale (1 = full workload)")
    ap.add_argument("--res-scale", type=float, default=1.0)
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--schedule", type=int, default=0, help="blend schedule: 0 tile grid, 1 persistent")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-binding", action="store_true")
    ap.add_argument("--binding-only", action="store_true",
                    help="time only the ray-cast binding association and print its JSON")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 256 MiB device to device once (a reference dispatch for "
                         "hardware traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the path "
              f"is built and measured on a single GPU (views would shard across GPUs with no "
              f"exchange in the forward and one gradient all-reduce per step).")
        sys.exit(2)

    from paper_2601_19233_amd import scenes
    t0 = time.time()
    scene = scenes.make_config(1, scale=args.scale, res_scale=args.res_scale)
    cpu = None
    if not args.no_cpu_baseline and not args.binding_only:
        # before the GPU is initialised: the oracle's worker processes fork
        # from a CPU-only process
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(scene)
        log(f"cpu baseline: {cpu['value']:.3g} Mpixels/s on {cpu['cores']} processes")

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_2601_19233_amd.render import Rasterizer

    if args.copy_calibration:
        src = torch.ones(64 << 20, device="cuda:0")           # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 268435456 bytes read, 268435456 bytes written")

    if args.binding_only:
        print(json.dumps({"binding": run_binding(args, scene)}), flush=True)
        return
    log(f"scene {scene.name}: N={scene.N} T={scene.T} in {time.time() - t0:.1f} s")
    cam = scene.cams[0]
    tw, th = (int(x) for x in args.tile.split("x"))
    dev = torch.device("cuda:0")
    r = Rasterizer("cuda:0", tile=(tw, th), frag_batch=args.batch, sh_degree=scene.sh_degree,
                   k_bind=scene.bind_face.shape[1], schedule=args.schedule)
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    V_def = f32(scene.proxy.V_def)
    bface = torch.from_numpy(scene.bind_face.astype(np.int32)).to(dev)
    bbary = f32(scene.bind_bary)
    means, quats, scales = f32(scene.means), f32(scene.quats), f32(scene.scales)
    opac, sh = f32(scene.opacity), f32(scene.sh.reshape(scene.N, -1))
    txyz, trgb, tal = f32(scene.tri_xyz.reshape(scene.T, 9)), f32(scene.tri_rgb.reshape(scene.T, 9)), f32(scene.tri_alpha)
    r.set_proxy(scene.proxy.V_rest, scene.proxy.faces)
    torch.cuda.synchronize()

    def step():
        dt = r.bind_transfer(V_def, bface, bbary, means, quats, scales)
        r.project([cam], means=dt["means"], cov3d=dt["cov3d"], opacity=opac, sh=sh,
                  tri_xyz=txyz, tri_rgb=trgb, tri_alpha=tal)
        r.bin()
        r.sort()
        return r.blend(want_state=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    n_dup, n_tiles, n_rec = r.query()
    log(f"n_dup={n_dup} tiles={n_tiles} records={n_rec}")

    # the timed steps run as a user runs them, with no per-kernel events
    # (recording two events around each of the frame's ~30 launches adds
    # about 0.14 ms per 1080p frame); the same steps again with the
    # library's events on give each kernel's launch duration for the
    # rooflines and stages_ms
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1) / args.steps
    r.set_profiling(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = r.profile()
    r.set_profiling(False)
    npix = cam.width * cam.height
    fwd_mpix = npix / (ms * 1e-3) / 1e6

    stages = {k: round(v[1] / args.steps, 4) for k, v in prof.items()}
    dominant = max(prof, key=lambda k: prof[k][1])
    bp = r.blend_pairs()
    log(f"blend work: {bp}")
    algo_bytes, n1 = algorithmic_bytes(r, scene, n_dup, n_rec)
    traffic = measured_traffic() if (cam.width, cam.height, scene.N) == (1920, 1080, 1000000) else {}
    rooflines = kernel_rooflines(prof, algo_bytes, traffic, pairs=bp)
    roof = rooflines.get(dominant)

    # ---- forward + backward (plain, eager) ---------------------------------
    # L2 loss against the frame rendered from N(0, 0.01)-perturbed raw
    # Gaussian parameters (same deformation, camera and triangles)
    pert = scenes.perturbed(scene, seed=1000 + 1)
    pm, pq, ps = f32(pert.means), f32(pert.quats), f32(pert.scales)
    po, psh = f32(pert.opacity), f32(pert.sh.reshape(scene.N, -1))
    dtp = r.bind_transfer(V_def, bface, bbary, pm, pq, ps)
    r.project([cam], means=dtp["means"], cov3d=dtp["cov3d"], opacity=po, sh=psh,
              tri_xyz=txyz, tri_rgb=trgb, tri_alpha=tal)
    r.bin()
    r.sort()
    target = r.blend(want_state=False)["image"].clone()
    del pert, pm, pq, ps, po, psh, dtp
    dL = torch.empty(3 * npix, device=dev)
    fwd_state = {}

    def step_fb():
        dt = r.bind_transfer(V_def, bface, bbary, means, quats, scales)
        r.project([cam], means=dt["means"], cov3d=dt["cov3d"], opacity=opac, sh=sh,
                  tri_xyz=txyz, tri_rgb=trgb, tri_alpha=tal)
        r.bin()
        r.sort()
        o = r.blend(want_state=True)
        fwd_state["out"] = o
        torch.sub(o["image"], target, out=dL)
        dL.mul_(2.0)
        return r.backward(dL, o, dt["means"], scales, quats, sh, dt["xform"])

    for _ in range(args.warmup):
        step_fb()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step_fb()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_fb = e0.elapsed_time(e1) / args.steps
    # the same steps again with the kernels timed, for the backward's roofline
    r.set_profiling(True)
    for _ in range(args.steps):
        step_fb()
    prof_fb = r.profile()
    r.set_profiling(False)
    bpairs = r.backward_pairs(fwd_state["out"]["n_contrib"])
    log(f"backward work: {bpairs}")
    rl_fb = kernel_rooflines(prof_fb, {}, traffic, pairs=None, bpairs=bpairs)
    fwd_bwd = {"mpix_s": round(npix / (ms_fb * 1e-3) / 1e6, 2), "ms_per_step": round(ms_fb, 4),
               "path": "plain forward + backward (eager), gradients to means/scales/quats/opacity/SH",
               "loss": "L2 against the render of N(0, 0.01)-perturbed raw Gaussian parameters",
               "stages_ms": {k: round(v[1] / args.steps, 4) for k, v in prof_fb.items()},
               "roofline": rl_fb.get("blend_backward")}
    log(f"fwd+bwd {ms_fb:.3f} ms/step")

    # ---- triangle colour and opacity gradients of the same frame ------------
    o = fwd_state["out"]
    tg = r.backward_triangles(dL, o)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        r.backward_triangles(dL, o, out=tg)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_tri = e0.elapsed_time(e1) / args.steps
    r.set_profiling(True)
    for _ in range(args.steps):
        r.backward_triangles(dL, o, out=tg)
    prof_tri = r.profile()
    r.set_profiling(False)
    tpairs = r.backward_pairs(o["n_contrib"], triangles=True)
    log(f"triangle backward {ms_tri:.3f} ms, work {tpairs}")
    # ---- proxy-vertex gradients of the same loss ----------------------------
    gl = step_fb()
    gV = r.backward_transfer(V_def, bface, bbary, gl["means"], gl["xform"])
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        r.backward_transfer(V_def, bface, bbary, gl["means"], gl["xform"], out=gV)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_px = e0.elapsed_time(e1) / args.steps
    r.set_profiling(True)
    for _ in range(args.steps):
        r.backward_transfer(V_def, bface, bbary, gl["means"], gl["xform"], out=gV)
    prof_px = r.profile()
    r.set_profiling(False)
    log(f"proxy backward {ms_px:.3f} ms")
    # algorithmic bytes of one call: per Gaussian its K bindings (12 B each),
    # dL/dmu' and dL/dA read (48 B), its gradient row and corner keys and ids
    # written (48 + 8 K B); per corner its key, id and barycentrics read
    # (16 B) and its Gaussian's row gathered (48 B); per face row 144 B read
    # (the gather rounds) and 144 B of sums; per vertex its frame inputs
    K = scene.bind_face.shape[1]
    nF = int(scene.proxy.faces.shape[0])
    px_bytes = scene.N * (12 * K + 48 + 48 + 8 * K) + scene.N * K * (16 + 48) + nF * 288
    px_ms = prof_px["transfer_backward"][1] / prof_px["transfer_backward"][0]
    px_ach = px_bytes / (px_ms * 1e-3) / 1e9
    fwd_bwd["proxy"] = {
        "ms_per_call": round(ms_px, 4),
        "path": "umgs_backward_transfer: dL/dV' of the deformed proxy from dL/dmu' and dL/dA",
        "stages_ms": {k: round(v[1] / args.steps, 4) for k, v in prof_px.items()},
        "nV": int(scene.proxy.V_rest.shape[0]), "gaussians": scene.N,
        "roofline": {"kernel": "transfer_backward (all of its launches)", "bound": "hbm",
                     "achieved": round(px_ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(px_ach / HBM_PEAK_GBS, 4), "traffic": None,
                     "ms_per_launch": round(px_ms, 4), "bytes": int(px_bytes)}}
    del gl, gV
    fwd_bwd["triangles"] = {
        "ms_per_call": round(ms_tri, 4),
        "path": "umgs_backward_triangles on the same frame: dL/d(per-vertex colour, opacity)",
        "stages_ms": {k: round(v[1] / args.steps, 4) for k, v in prof_tri.items()},
        "roofline": kernel_rooflines(prof_tri, {}, traffic, tpairs=tpairs).get("blend_backward_tri")}
    del tg

    # ---- the same frame captured in one HIP graph ---------------------------
    # (sizes stay on the device after one eager frame and a reservation, so
    # the bin stage needs no host synchronisation)
    from paper_2601_19233_amd.batched import BatchedStep
    rg = Rasterizer("cuda:0", tile=(tw, th), frag_batch=args.batch, sh_degree=scene.sh_degree,
                    k_bind=scene.bind_face.shape[1], schedule=args.schedule, own_stream=True)
    rg.set_proxy(scene.proxy.V_rest, scene.proxy.faces)
    gsc = dict(means=means, scales=scales, quats=quats, opacity=opac, sh=sh, tri_xyz=txyz,
               tri_rgb=trgb, tri_alpha=tal)
    gstep = BatchedStep(rg, [cam], gsc, deform=dict(V_def=V_def, bind_face=bface, bind_bary=bbary))
    gstep.prepare()
    for _ in range(args.warmup):
        gstep()
    torch.cuda.synchronize()
    gs = rg.stream
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record(gs)
    for _ in range(args.steps):
        gstep()
    g1.record(gs)
    torch.cuda.synchronize()
    ms_graph = g0.elapsed_time(g1) / args.steps
    if rg.overflowed():
        raise RuntimeError("graph frame overflowed its reservation")
    fwd_graph = {"mpix_s": round(npix / (ms_graph * 1e-3) / 1e6, 2), "ms_per_step": round(ms_graph, 4),
                 "path": "the forward step captured in one HIP graph (one launch per frame)"}
    log(f"graph fwd {ms_graph:.3f} ms/step")
    del gstep, rg

    del r, fwd_state
    torch.cuda.empty_cache()
    batched = uneven = bwd800 = orbit = binding = None
    if not args.no_batched and not args.no_binding:
        binding = run_binding(args, scene)
        torch.cuda.empty_cache()
    if not args.no_batched:
        bwd800 = run_backward_800(args)
        torch.cuda.empty_cache()
        uneven = run_uneven(args)
        torch.cuda.empty_cache()
        orbit = run_batched_orbit(args, scene)
        torch.cuda.empty_cache()
        batched = run_batched(args)

    out = {
        "metric": METRIC, "value": round(fwd_mpix, 2), "unit": "Mpixels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": scene.name, "width": cam.width, "height": cam.height,
                   "gaussians": scene.N, "triangles": scene.T, "k_bind": int(scene.bind_face.shape[1]),
                   "tile": args.tile, "frag_batch": args.batch,
                   "schedule": ["tile_grid", "persistent"][args.schedule], "path": "plain forward"},
        "n_dup": n_dup, "n_supertile_entries": n1, "stages_ms": stages, "roofline": roof, "rooflines": rooflines,
        "wall_s": round(wall, 3),
        "fwd_graph": fwd_graph, "fwd_bwd": fwd_bwd, "backward_800": bwd800, "batched": batched,
        "batched_1080p_x16_orbit": orbit, "batched_uneven": uneven, "binding": binding,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
