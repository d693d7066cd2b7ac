"""Batched multi-view step: one frame of V views rendered (and optionally
differentiated) by a captured HIP graph.

The first call runs the step eagerly to size every buffer, reserves key
capacity for ``headroom`` times the duplicates it saw, captures the step on
the rasterizer's stream, and from then on each step is one graph launch with
all sizes read on the device.  Views share one global tile space: every
kernel of the path runs once for all views.
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence

import torch

from .render import Rasterizer


class BatchedStep:
    def __init__(self, rast: Rasterizer, cams: Sequence, scene: Dict[str, torch.Tensor],
                 deform: Optional[Dict[str, torch.Tensor]] = None, backward: bool = False,
                 headroom: float = 1.25):
        """scene: device tensors means, opacity, sh (N, nc*3), scales, quats and
        optionally tri_xyz, tri_rgb, tri_alpha.  deform: V_def, bind_face,
        bind_bary (the proxy must already be set on ``rast``).  ``rast`` must
        own its stream (Rasterizer(own_stream=True)): the null stream cannot
        be captured."""
        if rast.stream.cuda_stream == 0:
            raise ValueError("BatchedStep needs a Rasterizer created with own_stream=True")
        self.r = rast
        self.cams = list(cams)
        self.scene = scene
        self.deform = deform
        self.do_backward = backward
        self.headroom = headroom
        self.graph_ready = False
        self.tout = None
        self.out = None
        self.grads = None
        self.dL = None

    def _step(self):
        s, r = self.scene, self.r
        tris = {k: s[k] for k in ("tri_xyz", "tri_rgb", "tri_alpha") if k in s}
        if self.deform is not None:
            d = self.deform
            self.tout = r.bind_transfer(d["V_def"], d["bind_face"], d["bind_bary"], s["means"],
                                        s["quats"], s["scales"], out=self.tout)
            r.project(self.cams, means=self.tout["means"], cov3d=self.tout["cov3d"],
                      opacity=s["opacity"], sh=s["sh"], **tris)
        else:
            r.project(self.cams, means=s["means"], scales=s["scales"], quats=s["quats"],
                      opacity=s["opacity"], sh=s["sh"], **tris)
        r.bin()
        r.sort()
        self.out = r.blend(want_state=True, out=self.out)
        if self.do_backward:
            if self.dL is None:
                self.dL = torch.zeros_like(self.out["image"])
            pm = self.tout["means"] if self.deform is not None else s["means"]
            xf = self.tout["xform"] if self.deform is not None else None
            self.grads = r.backward(self.dL, self.out, pm, s["scales"], s["quats"], s["sh"], xf,
                                    out=self.grads)
        return self.out

    def prepare(self):
        """Eager frame, reservation and capture."""
        self._step()
        n_dup, _, _ = self.r.query()
        self.n_dup_seen = n_dup
        self.r.reserve(max(1, int(n_dup * self.headroom)))
        torch.cuda.synchronize()
        self.r.capture(self._step)
        self.graph_ready = True

    def __call__(self):
        if not self.graph_ready:
            self.prepare()
        self.r.replay()
        return self.out

    def set_loss_gradient(self, dL: torch.Tensor):
        """Copy dL/dimage into the buffer the captured backward reads."""
        self.dL.copy_(dL.reshape(-1))
