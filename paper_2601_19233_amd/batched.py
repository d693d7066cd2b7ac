"""Batched multi-view step: one frame of V views rendered (and optionally
differentiated) by a captured HIP graph.

Planning runs once: the deformation transfer and the projection of all views
give every view's duplicate count (``view_dups``) before anything is sorted;
consecutive views are grouped so that no group exceeds ``group_budget``
duplicates (32-bit list positions, 4 bytes each) or ``group_tiles`` screen
tiles (2^22 tiles keep supertile ids within 16 bits).  One eager step then
renders every group (allocating buffers and storing one device view table
per group), key capacity is reserved for the largest group times
``headroom``, and the whole step -- transfer, then per group project, bin,
sort, blend and (optionally) backward, gradients summed over groups -- is
captured on the rasterizer's stream.  Each later step is one graph launch
with all sizes read on the device.
"""
from __future__ import annotations

from typing import Callable, Dict, List, Optional, Sequence, Tuple

import torch

from .render import Rasterizer


class BatchedStep:
    def __init__(self, rast: Rasterizer, cams: Sequence, scene: Dict[str, torch.Tensor],
                 deform: Optional[Dict[str, torch.Tensor]] = None, backward: bool = False,
                 headroom: float = 1.25, group_budget: int = 3_000_000_000,
                 group_tiles: int = 1 << 22, loss_grad: Optional[Callable] = None,
                 triangle_grads: bool = False, proxy_grads: bool = False):
        """scene: device tensors means, opacity, sh (N, nc*3), scales, quats and
        optionally tri_xyz, tri_rgb, tri_alpha.  deform: V_def, bind_face,
        bind_bary (the proxy must already be set on ``rast``).  ``rast`` must
        own its stream (Rasterizer(own_stream=True)): the null stream cannot
        be captured.

        With ``backward``, the gradient of the loss with respect to the image
        is either copied in by set_loss_gradient, or -- with ``loss_grad`` --
        computed inside the step: ``loss_grad(image, dL, p0, p1)`` is called
        after each group's blend with that group's image slice, the slice of
        the dL buffer to fill and the group's pixel range [p0, p1), on the
        rasterizer's stream; it is captured with the rest, so it must launch
        device work only (no allocation, no synchronisation).
        ``triangle_grads`` adds the triangles' colour and opacity gradients
        (``tgrads``: tri_rgb, tri_alpha, summed over the groups),
        ``proxy_grads`` (with ``deform``) the deformed proxy's vertex
        gradient (``vgrad``, (nV, 3)), both inside the captured step."""
        if rast.stream.cuda_stream == 0:
            raise ValueError("BatchedStep needs a Rasterizer created with own_stream=True")
        self.r = rast
        self.cams = list(cams)
        self.scene = scene
        self.deform = deform
        self.do_backward = backward or triangle_grads or proxy_grads
        self.triangle_grads = triangle_grads
        self.proxy_grads = proxy_grads and deform is not None
        self.tgrads = None
        self.vgrad = None
        self.loss_grad = loss_grad
        self.headroom = headroom
        self.group_budget = int(group_budget)
        self.group_tiles = int(group_tiles)
        self.graph_ready = False
        self.tout = None
        self.out = None
        self.grads = None
        self.dL = None
        self.groups: List[Tuple[int, int]] = []
        self.n_dup_seen = 0
        npix = [c.width * c.height for c in self.cams]
        self.pix0 = [0]
        for n in npix:
            self.pix0.append(self.pix0[-1] + n)

    # -- helpers ------------------------------------------------------------
    def _tris(self):
        return {k: self.scene[k] for k in ("tri_xyz", "tri_rgb", "tri_alpha") if k in self.scene}

    def _transfer(self):
        s, d = self.scene, self.deform
        if d is None:
            return
        self.tout = self.r.bind_transfer(d["V_def"], d["bind_face"], d["bind_bary"], s["means"],
                                         s["quats"], s["scales"], out=self.tout)

    def _project(self, cams):
        s = self.scene
        if self.deform is not None:
            self.r.project(cams, means=self.tout["means"], cov3d=self.tout["cov3d"],
                           opacity=s["opacity"], sh=s["sh"], **self._tris())
        else:
            self.r.project(cams, means=s["means"], scales=s["scales"], quats=s["quats"],
                           opacity=s["opacity"], sh=s["sh"], **self._tris())

    def _slice(self, a, b):
        p0, p1 = self.pix0[a], self.pix0[b]
        o = self.out
        return dict(image=o["image"][3 * p0:3 * p1], T_final=o["T_final"][p0:p1],
                    n_contrib=o["n_contrib"][p0:p1], T_entity_in=o["T_entity_in"][p0:p1])

    # -- planning -----------------------------------------------------------
    def plan(self) -> List[Tuple[int, int]]:
        """Group consecutive views so each group stays within the duplicate
        budget and within ``group_tiles`` screen tiles."""
        self._transfer()
        dups: List[int] = []
        step = max(1, min(len(self.cams), 64))
        for a in range(0, len(self.cams), step):
            self._project(self.cams[a:a + step])
            dups += self.r.view_dups()
        tw, th = self.r.opts.tile_w, self.r.opts.tile_h
        tiles = [((c.width + tw - 1) // tw) * ((c.height + th - 1) // th) for c in self.cams]
        groups, a, acc, acc_t = [], 0, 0, 0
        for v, n in enumerate(dups):
            if n >= 0xFFFF0000:
                raise RuntimeError(f"view {v} alone produces {n} duplicates (32-bit positions)")
            if v > a and (acc + n > self.group_budget or acc_t + tiles[v] > self.group_tiles):
                groups.append((a, v))
                a, acc, acc_t = v, 0, 0
            acc += n
            acc_t += tiles[v]
        groups.append((a, len(dups)))
        self.view_dup_counts = dups
        self.groups = groups
        self.max_group_dups = max(sum(dups[a:b]) for a, b in groups)
        return groups

    # -- the step -----------------------------------------------------------
    def _step(self):
        s, r = self.scene, self.r
        self._transfer()
        for gi, (a, b) in enumerate(self.groups):
            self._project(self.cams[a:b])
            r.bin()
            r.sort()
            part = self._slice(a, b)
            r.blend(want_state=True, out=part)
            if self.do_backward:
                pm = self.tout["means"] if self.deform is not None else s["means"]
                xf = self.tout["xform"] if self.deform is not None else None
                p0, p1 = self.pix0[a], self.pix0[b]
                if self.loss_grad is not None:
                    with torch.cuda.stream(r.stream):
                        self.loss_grad(part["image"], self.dL[3 * p0:3 * p1], p0, p1)
                self.grads = r.backward(self.dL[3 * p0:3 * p1], part, pm, s["scales"], s["quats"],
                                        s["sh"], xf, out=self.grads, accumulate=gi > 0)
                if self.triangle_grads:
                    self.tgrads = r.backward_triangles(self.dL[3 * p0:3 * p1], part, out=self.tgrads,
                                                       accumulate=gi > 0)
        if self.proxy_grads:
            d = self.deform
            self.vgrad = r.backward_transfer(d["V_def"], d["bind_face"], d["bind_bary"],
                                             self.grads["means"], self.grads["xform"], out=self.vgrad)
        return self.out

    def prepare(self):
        """Plan, render one eager step, reserve, capture."""
        dev = self.r.device
        P = self.pix0[-1]
        self.out = dict(image=torch.empty(3 * P, device=dev), T_final=torch.empty(P, device=dev),
                        n_contrib=torch.empty(P, device=dev, dtype=torch.int32),
                        T_entity_in=torch.empty(P, device=dev))
        if self.do_backward:
            self.dL = torch.zeros(3 * P, device=dev)
        self.plan()
        self._step()
        self.n_dup_seen = sum(self.view_dup_counts)
        self.r.reserve(max(1, int(self.max_group_dups * self.headroom)))
        torch.cuda.synchronize()
        self.r.capture(self._step)
        self.graph_ready = True

    def __call__(self):
        if not self.graph_ready:
            self.prepare()
        self.r.replay()
        return self.out

    def split_views(self, flat: torch.Tensor, channels: int):
        """Per-view (channels, H, W) views of a packed output of all groups."""
        out = []
        for v, c in enumerate(self.cams):
            a, b = channels * self.pix0[v], channels * self.pix0[v + 1]
            out.append(flat[a:b].view(channels, c.height, c.width) if channels > 1
                       else flat[a:b].view(c.height, c.width))
        return out

    def set_loss_gradient(self, dL: torch.Tensor):
        """Copy dL/dimage into the buffer the captured backward reads."""
        self.dL.copy_(dL.reshape(-1))

    def update_views(self, new_cams: Sequence):
        """New cameras (same sizes) for the next replays."""
        new_cams = list(new_cams)
        for a, b in self.groups:
            self.r.update_views(self.cams[a:b], new_cams[a:b])
        self.cams = new_cams
