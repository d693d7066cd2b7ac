"""Comparison helpers for GPU-vs-oracle parity tests."""
import numpy as np

from oracle import render as OR

TOL = 1e-4          # absolute per channel, FP32 GPU vs FP64 oracle


class Mismatch(AssertionError):
    pass


def oracle_frame(scene, cam, mode=0, cov3d=None, means=None, bg=(0.0, 0.0, 0.0)):
    kw = dict(scales=None, quats=None, cov3d=cov3d) if cov3d is not None else dict(
        scales=scene.scales, quats=scene.quats)
    return OR.Frame(cam, scene.means if means is None else means, scene.opacity, scene.sh,
                    scene.sh_degree, scene.tri_xyz, scene.tri_rgb, scene.tri_alpha, bg=bg,
                    mode=mode, **kw)


def compare_pixels(fr, img, Tf, last_gid, pixels, tol=TOL, margin_rel=1e-4, Tent=None):
    """Check GPU outputs at pixels (list of (px, py)) against the oracle.

    img: (3,H,W), Tf: (H,W), last_gid: (H,W) global id of the GPU's last
    blended fragment (-1 if none) or None.  A pixel passes if the nominal
    oracle result matches, or, when it holds decisions within margin_rel of
    their thresholds, one of the results with up to two of those decisions
    inverted (all of them valid).  Returns counts."""
    n_ok = n_amb = 0
    worst = 0.0
    for px, py in pixels:
        g = img[:, py, px].astype(np.float64)
        gT = float(Tf[py, px])
        gl = None if last_gid is None else int(last_gid[py, px])
        cands = [fr.pixel(px, py, margin_rel)]
        matched = None
        for attempt in range(2):
            for r in cands:
                dc = float(np.max(np.abs(g - r.C)))
                dT = abs(gT - r.T)
                dE = 0.0 if Tent is None else abs(float(Tent[py, px]) - r.T_entity_in)
                if dc <= tol and dT <= tol and dE <= tol and (gl is None or gl == r.last_id):
                    matched = r
                    worst = max(worst, dc)
                    break
            if matched is not None or attempt == 1:
                break
            cands = fr.pixel_variants(px, py, margin_rel)[1:]
        if matched is None:
            r = fr.pixel(px, py, margin_rel)
            raise Mismatch(f"pixel ({px},{py}): gpu C={g} T={gT} last={gl}; oracle C={r.C} T={r.T} "
                           f"last={r.last_id} margin={r.margin:.3g} amb={r.ambiguous[:4]}")
        if matched is cands[0] and attempt == 0:
            n_ok += 1
        else:
            n_amb += 1
    return dict(ok=n_ok, ambiguous=n_amb, worst=worst)


def gpu_last_gid(n_contrib, ranges, vals, view_tile_base, ntx, tw, th, W, H, per_view, view):
    """Map per-pixel 1-based list positions to global fragment ids."""
    nc = n_contrib.reshape(H, W)
    out = np.full((H, W), -1, np.int64)
    ys, xs = np.nonzero(nc > 0)
    tiles = view_tile_base + (ys // th) * ntx + (xs // tw)
    starts = ranges[tiles, 0].astype(np.int64)
    rid = vals[starts + nc[ys, xs] - 1].astype(np.int64)
    out[ys, xs] = rid - view * per_view
    return out
