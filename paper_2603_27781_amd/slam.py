"""Tracking and mapping iterations of GS^3LAM on top of the C ABI (Sec. 3.3,
3.4; learning rates and iteration counts of Supp. C.1).

Host orchestration only: every computation is a call into libsgs (render,
SLAM loss, backward, pose gradient, optimiser steps, expansion, DSR), with
the state (Gaussian planes, Adam moments, poses) in device memory.

  Tracker.track   -- frame-to-model tracking (Sec. 3.4; the map is frozen, so
      the appearance records are written once per call): the pose starts
      from the constant-velocity prediction T_t = T_{t-1} T_{t-2}^-1 T_{t-1}
      (Eq. 19) and is refined for `iters` iterations of: render, tracking
      loss (every term under M_obs, Eq. 21), pose-only backward, twist
      gradient, Adam + left update T <- Exp(dxi) T (gs_pose_step).
  Mapper.iterate  -- one mapping iteration (Sec. 3.3.4): an RSKM-sampled
      keyframe (Eq. 13) is rendered, the mapping loss (L1 + SSIM colour,
      depth, semantic, Eq. 18) and the scale regulariser (Eq. 12) are
      back-propagated to every Gaussian parameter and one Adam step updates
      them with the per-attribute learning rates.
  rskm_pick       -- the keyframe sampling of Eq. (13), read as: every
      t_opt-th iteration the current frame, otherwise a keyframe drawn
      uniformly (the printed p(f) is not normalised as written).
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib, raster
from ._lib import GsAdamGroup, GsSlamLossOpts, check

# Supp. C.1
TRACK_LR_RHO, TRACK_LR_PHI = 0.002, 0.0004  # translation, rotation (the paper's quaternion rate)
MAP_LR = {"mu": 0.0001, "color": 0.0025, "quat": 0.001, "logit": 0.05, "log_scale": 0.001, "feat": 0.0025}
TRACK_ITERS, MAP_ITERS = 40, 60             # Replica
ADAM_BETAS, ADAM_EPS = (0.9, 0.999), 1e-8


def constant_velocity(T1: np.ndarray, T2: np.ndarray) -> np.ndarray:
    """Eq. (19): T_t = T_{t-1} T_{t-2}^-1 T_{t-1} (4x4 world-to-camera)."""
    return T1 @ np.linalg.inv(T2) @ T1


def rskm_pick(rng: np.random.Generator, n_keyframes: int, current: int, k_m: int, t_opt: int) -> int:
    """Eq. (13): the current frame on every t_opt-th mapping iteration,
    otherwise one of the keyframes uniformly."""
    if t_opt > 0 and k_m % t_opt == 0:
        return current
    return int(rng.integers(0, n_keyframes))


def _opts(mode: str) -> GsSlamLossOpts:
    L = _lib.load()
    o = GsSlamLossOpts()
    check(L.gs_default_slam_loss_opts(ctypes.byref(o)), "gs_default_slam_loss_opts")
    if mode == "tracking":
        o.ssim_lambda, o.w_sem, o.flags = 0.0, 0.001, _lib.GS_LOSS_OBS_MASK
    return o


class Tracker:
    """Pose refinement of one view against a fixed map."""

    def __init__(self, r: raster.Rasterizer, g: raster.Gaussians, decoder: Optional[torch.Tensor] = None):
        assert r.views.n == 1
        self.r, self.g, self.decoder = r, g, decoder
        dev = dict(device=r.device)
        self.m = torch.zeros(1, 6, dtype=torch.float32, **dev)
        self.v = torch.zeros(1, 6, dtype=torch.float32, **dev)
        self.step = torch.zeros(1, dtype=torch.int32, **dev)  # Adam's step count (graph mode)
        self.opts = _opts("tracking")
        self.graph = None

    def set_pose(self, T: np.ndarray) -> None:
        self.r.views.set_poses(torch.from_numpy(np.ascontiguousarray(T[:3, :4], np.float32)).to(self.r.device))

    def pose(self) -> np.ndarray:
        Rt = self.r.views.dev.view(torch.float32)[0, 6:18].cpu().numpy().reshape(3, 4).astype(np.float64)
        return np.vstack([Rt, [0, 0, 0, 1]])

    def iteration(self, rgb_t, depth_t, labels, step: Optional[int]) -> None:
        """One iteration; step None takes Adam's step count from self.step on
        the device (gs_pose_step_dev), as a captured iteration must."""
        r, g = self.r, self.g
        r.project(g, write_app=False)  # the map is frozen: appearance records from refresh()
        r.bin_sort()
        r.render_fwd()
        r.slam_loss(rgb_t, depth_t, labels, self.decoder, self.opts, masks=True)
        r.render_bwd(g, r.grad_out, _lib.GS_GRAD_POSE, None)
        tw = r.pose_grad(g)
        L = _lib.load()
        args = (r.views.dev_ptr(), 1, tw.data_ptr(), self.m.data_ptr(), self.v.data_ptr(), TRACK_LR_RHO, TRACK_LR_PHI,
                ADAM_BETAS[0], ADAM_BETAS[1], ADAM_EPS)
        if step is None:
            check(L.gs_pose_step_dev(*args, self.step.data_ptr(), raster._stream()), "gs_pose_step_dev")
        else:
            check(L.gs_pose_step(*args, step, raster._stream()), "gs_pose_step")

    def refresh(self) -> None:
        """Writes the appearance records of the current map (colours and
        features, which tracking does not change), once per tracked frame."""
        self.r.project(self.g)

    def capture(self, rgb_t, depth_t, labels) -> None:
        """Captures one iteration (device step count) in a HIP graph for
        replay by track(..., graph=True); the targets' buffers are baked in.
        One eager iteration first sets up the lazily allocated workspaces; the
        state it changes is reset by track."""
        self.refresh()
        self.iteration(rgb_t, depth_t, labels, None)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.iteration(rgb_t, depth_t, labels, None)
        torch.cuda.synchronize()
        self.graph_targets = (rgb_t, depth_t, labels)

    def track(self, rgb_t, depth_t, labels, T_init: np.ndarray, iters: int = TRACK_ITERS,
              graph: bool = False) -> np.ndarray:
        """Frame-to-model tracking from T_init; with graph, the iterations
        are replays of a captured one (captured on first use with these
        targets, which must then stay the same buffers)."""
        if graph and (self.graph is None or any(a is not b for a, b in zip(self.graph_targets,
                                                                           (rgb_t, depth_t, labels)))):
            self.capture(rgb_t, depth_t, labels)
        self.set_pose(T_init)
        self.m.zero_()
        self.v.zero_()
        self.step.zero_()
        self.refresh()
        for k in range(1, iters + 1):
            if graph:
                self.graph.replay()
            else:
                self.iteration(rgb_t, depth_t, labels, k)
        return self.pose()


class Mapper:
    """Mapping iterations over a set of keyframes (one view rendered per
    iteration) with Adam on every Gaussian parameter and the scale
    regulariser."""

    def __init__(self, r: raster.Rasterizer, g: raster.Gaussians, decoder: Optional[torch.Tensor] = None,
                 w_big: float = 0.01, w_small: float = 0.001):
        assert r.views.n == 1
        self.r, self.g, self.decoder = r, g, decoder
        self.grads = g.zeros_like()
        self.m = g.zeros_like()
        self.v = g.zeros_like()
        self.w_big, self.w_small = w_big, w_small
        self.opts = _opts("mapping")
        self.step = 0

    def iteration(self, rgb_t, depth_t, labels, T: np.ndarray) -> torch.Tensor:
        r, g = self.r, self.g
        r.views.set_poses(torch.from_numpy(np.ascontiguousarray(T[:3, :4], np.float32)).to(r.device))
        r.project(g)
        r.bin_sort()
        r.render_fwd()
        r.slam_loss(rgb_t, depth_t, labels, self.decoder, self.opts, masks=True)
        # the projection backward writes the gradients; DSR then adds to them
        r.render_bwd(g, r.grad_out, _lib.GS_GRAD_PARAMS, self.grads, write=True)
        dsr_out = raster.dsr(g.log_scale, self.w_big, self.w_small, self.grads.log_scale)
        self.step += 1
        names = ("mu", "log_scale", "quat", "logit", "color", "feat")
        groups = []
        for nm, p, gr, m, v in zip(names, g.tensors(), self.grads.tensors(), self.m.tensors(), self.v.tensors()):
            if p is None or p.numel() == 0:
                continue
            groups.append(GsAdamGroup(p.data_ptr(), gr.data_ptr(), m.data_ptr(), v.data_ptr(), p.numel(),
                                      MAP_LR[nm], 0))
        arr = (GsAdamGroup * len(groups))(*groups)
        L = _lib.load()
        check(L.gs_adam_step(ctypes.cast(arr, ctypes.c_void_p), len(groups), ADAM_BETAS[0], ADAM_BETAS[1], ADAM_EPS,
                             self.step, raster._stream()), "gs_adam_step")
        return dsr_out
