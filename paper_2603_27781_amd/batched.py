"""Batched multi-view mapping / tracking step (GS^3LAM Sec. 3.3.3-3.4).

RSKM mapping samples keyframes that all render the same SG-Field; here the
V keyframes of one step are rendered, compared with their targets and
back-propagated together: one projection launch over all (view, Gaussian)
pairs, one binning over all views (global tile ids carry the view), one
forward and one backward compositing launch over every (view, tile) item
(optionally persistent, pulling items from a device queue), the loss
gradient (in the forward kernel's epilogue where gs_render_fwd_loss
supports the channel and class counts, else its own kernel), and the
projection backward summing the views' gradients
per Gaussian in registers.  The whole step is captured once in a HIP graph
(torch.cuda.graph) and replayed; poses change between replays through
Views.set_poses, parameters in place.

`PerViewStep` is the plain alternative it is compared against: V
independent single-view passes on the same stream, no graph.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from .raster import Config, Gaussians, Rasterizer, Views

# Launch configuration the benchmark times (chosen with autotune.tune on the
# 8 x 1200x680, 1M-Gaussian, F=16 mapping step).
BENCH_CONFIG = {"tile": 16, "lds_batch": 256, "persistent": 0, "lds_batch_bwd": 128}


class MappingStep:
    def __init__(self, g: Gaussians, views: Sequence, cfg: Config, rgb_t: torch.Tensor, depth_t: torch.Tensor,
                 labels: Optional[torch.Tensor], decoder: Optional[torch.Tensor], weights=(0.5, 1.0, 0.01),
                 params: bool = True, pose: bool = False, capacity: Optional[int] = None,
                 fuse_loss: bool = True):
        self.g = g
        self.cfg = cfg
        self.views = Views(views, cfg.tile)
        self.r = Rasterizer(g.n, g.n_feat, self.views, cfg, capacity=capacity)
        self.rgb_t, self.depth_t, self.labels, self.decoder = rgb_t, depth_t, labels, decoder
        self.weights = weights
        self.flags = (_lib.GS_GRAD_PARAMS if params else 0) | (_lib.GS_GRAD_POSE if pose else 0)
        self.grads = g.zeros_like() if params else None
        self.graph = None
        self.fuse_loss = fuse_loss and self.r.fused_loss_supported(decoder)
        if self.fuse_loss:
            self.r.ensure_fused_ws()

    def ensure_capacity(self, slack: float = 1.25) -> int:
        return self.r.ensure_capacity(self.g, slack)

    def run(self) -> None:
        """One eager step: project, bin, render, loss, backward; the
        projection backward writes the parameter gradients (one launch sums
        every view), so they need no clearing first."""
        r = self.r
        r.project(self.g)
        r.bin_sort()
        if self.fuse_loss:
            r.render_fwd_loss(self.rgb_t, self.depth_t, self.labels, self.decoder, self.weights)
        else:
            r.render_fwd()
            r.loss_grad(self.rgb_t, self.depth_t, self.labels, self.decoder, self.weights)
        r.render_bwd(self.g, r.grad_out, self.flags, self.grads, write=True)
        if self.flags & _lib.GS_GRAD_POSE:
            r.pose_grad(self.g)

    def capture(self, warmup: int = 2) -> None:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(warmup):
                self.run()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()
        torch.cuda.synchronize()

    def replay(self) -> None:
        if self.graph is None:
            self.run()
        else:
            self.graph.replay()

    @property
    def loss(self) -> torch.Tensor:
        return self.r.loss

    @property
    def twist(self) -> torch.Tensor:
        return self.r.twist


class PerViewStep:
    """V plain single-view passes (no batching, no graph)."""

    def __init__(self, g: Gaussians, views: Sequence, cfg: Config, rgb_t, depth_t, labels, decoder,
                 weights=(0.5, 1.0, 0.01), params: bool = True, pose: bool = False, fuse_loss: bool = True):
        self.g = g
        self.steps = []
        off = 0
        for v in views:
            P = v.width * v.height
            sl = slice(off, off + P)
            st = MappingStep(g, [v], cfg, rgb_t[:, sl].contiguous(), depth_t[sl].contiguous(),
                             labels[sl].contiguous() if labels is not None else None, decoder, weights,
                             params=False, pose=pose, fuse_loss=fuse_loss)
            st.flags = (_lib.GS_GRAD_PARAMS if params else 0) | (_lib.GS_GRAD_POSE if pose else 0)
            self.steps.append(st)
            off += P
        self.grads = g.zeros_like() if params else None

    def ensure_capacity(self) -> None:
        for st in self.steps:
            st.ensure_capacity()

    def run(self) -> None:
        if self.grads is not None:
            for t in self.grads.tensors():
                t.zero_()
        for st in self.steps:
            st.grads = self.grads
            r = st.r
            r.project(self.g)
            r.bin_sort()
            if st.fuse_loss:
                r.render_fwd_loss(st.rgb_t, st.depth_t, st.labels, st.decoder, st.weights)
            else:
                r.render_fwd()
                r.loss_grad(st.rgb_t, st.depth_t, st.labels, st.decoder, st.weights)
            r.render_bwd(self.g, r.grad_out, st.flags, self.grads)
            if st.flags & _lib.GS_GRAD_POSE:
                r.pose_grad(self.g)
