#!/usr/bin/env python3
"""Benchmark of the mixed Gaussian/triangle rasterizer on one MI355X.

Workload (default): one 1920x1080 view of 1M Gaussians bound (8 bounding-box
corners each) to a 20,480-face proxy sphere bent by 0.2 sin(2 pi x), plus
100,128 occluder triangles.  One step = the whole hot path on that frame:
per-vertex proxy transforms and per-Gaussian deformation transfer, Gaussian
projection and triangle set-up, binning, the (tile, depth) radix sort and the
front-to-back blend.  Inputs are resident in device memory before timing.

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


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(scene, budget_pixels=400, seed=0):
    """Time the CPU FP64 oracle on a bounded sample of the same frame."""
    from threadpoolctl import threadpool_limits
    from oracle import render as OR
    from oracle import transfer as OT
    cam = scene.cams[0]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ot = OT.transfer(scene.proxy.V_rest, scene.proxy.faces, scene.proxy.V_def, scene.means,
                         scene.quats, scene.scales, scene.bind_face, scene.bind_bary)
        fr = OR.Frame(cam, ot["means"], scene.opacity, scene.sh, scene.sh_degree, scene.tri_xyz,
                      scene.tri_rgb, scene.tri_alpha, cov3d=ot["cov3d"])
        t_setup = time.perf_counter() - t0
        rng = np.random.default_rng(seed)
        px = rng.integers(0, cam.width, budget_pixels)
        py = rng.integers(0, cam.height, budget_pixels)
        t1 = time.perf_counter()
        for x, y in zip(px.tolist(), py.tolist()):
            fr.pixel(x, y)
        t_pix = (time.perf_counter() - t1) / budget_pixels
    npix = cam.width * cam.height
    full = t_setup + t_pix * npix
    return {"value": npix / full / 1e6, "unit": "Mpixels/s", "cores": 1, "kind": "oracle",
            "sample": f"frame set-up (transfer + projection of all primitives, {t_setup:.1f} s) "
                      f"plus {budget_pixels} uniformly sampled pixels ({t_pix * 1e3:.1f} ms/pixel), "
                      f"extrapolated to {cam.width}x{cam.height}: {full:.0f} s per frame"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0, help="primitive-count scale (1 = full workload)")
    ap.add_argument("--res-scale", type=float, default=1.0)
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the path is single-GPU by design; see the sharding notes in DESIGN.md).")
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_2601_19233_amd import scenes
    from paper_2601_19233_amd.render import Rasterizer

    t0 = time.time()
    scene = scenes.make_config(1, scale=args.scale, res_scale=args.res_scale)
    log(f"scene {scene.name}: N={scene.N} T={scene.T} in {time.time() - t0:.1f} s")
    cam = scene.cams[0]
    tw, th = (int(x) for x in args.tile.split("x"))
    dev = torch.device("cuda:0")
    r = Rasterizer("cuda:0", tile=(tw, th), frag_batch=args.batch, sh_degree=scene.sh_degree,
                   k_bind=scene.bind_face.shape[1])
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

    r.set_profiling(True)
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
    prof = r.profile()
    r.set_profiling(False)
    npix = cam.width * cam.height
    fwd_mpix = npix / (ms * 1e-3) / 1e6

    stages = {k: round(v[1] / args.steps, 4) for k, v in prof.items()}
    per_launch = {k: v[1] / v[0] for k, v in prof.items()}
    dominant = max(prof, key=lambda k: prof[k][1])
    # algorithmic HBM bytes per launch of the bandwidth-bound kernels
    algo_bytes = {
        "sort_downsweep": 24.0 * n_dup,          # read key+value, write key+value
        "sort_upsweep": 8.0 * n_dup,             # read key
        "emit_keys": 12.0 * n_dup + 24.0 * n_rec,
        "tile_ranges": 8.0 * n_dup + 8.0 * n_tiles,
        "transfer": scene.N * (40.0 + 12.0 * scene.bind_face.shape[1] + 88.0),
        "project_gaussians": scene.N * (12 + 24 + 4 + 12 + 4 + 8 + 8 + 48.0),
    }
    roof = None
    if dominant in algo_bytes:
        ach = algo_bytes[dominant] / (per_launch[dominant] * 1e-3) / 1e9
        roof = {"kernel": dominant, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "ms_per_launch": round(per_launch[dominant], 4)}
    else:
        roof = {"kernel": dominant, "bound": "alu", "achieved": None, "peak": VALU_PEAK_GOPS,
                "unit": "Gop/s", "frac": None, "traffic": None,
                "ms_per_launch": round(per_launch[dominant], 4)}

    out = {
        "metric": METRIC, "value": round(fwd_mpix, 2), "unit": "Mpixels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": scene.name, "width": cam.width, "height": cam.height,
                   "gaussians": scene.N, "triangles": scene.T, "k_bind": int(scene.bind_face.shape[1]),
                   "tile": args.tile, "frag_batch": args.batch, "path": "plain forward"},
        "n_dup": n_dup, "stages_ms": stages, "roofline": roof, "wall_s": round(wall, 3),
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(scene)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
