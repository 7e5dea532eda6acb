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
  SlamRun         -- the loop over a sequence of RGB-D-semantic frames
      (Sec. 3.3-3.4): the first frame fixes the world frame, every pixel of
      it with a depth becomes a Gaussian and is mapped; every later frame is
      tracked from the constant-velocity guess, expanded at its M_unobs
      pixels (Sec. 3.3.1), kept as a keyframe every kf_every frames and
      mapped with RSKM over the keyframes, the decoder learned with the field.

Every call that bins instances ORs a capacity overflow or a scan wait that
gave up into the rasterizer's sticky flag; tracking checks it after its
iterations (and redoes them with a larger capacity), a mapping batch after
its iterations (and raises: the map has already moved).
"""
from __future__ import annotations

import ctypes
import dataclasses
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
DECODER_LR = 0.0025                         # not stated: the semantic feature's rate


class CapacityError(RuntimeError):
    """A binning in a batch of iterations overflowed the instance capacity
    or gave up a scan wait, so some iteration worked on truncated lists."""


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

    def __init__(self, r: raster.Rasterizer, g: raster.Gaussians, decoder: Optional[torch.Tensor] = None,
                 bias: Optional[torch.Tensor] = None):
        assert r.views.n == 1
        self.r, self.g, self.decoder, self.bias = r, g, decoder, bias
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
        r.slam_loss(rgb_t, depth_t, labels, self.decoder, self.opts, masks=True, bias=self.bias)
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
        targets, which must then stay the same buffers).  If any iteration's
        binning overflowed the instance capacity (the pose moved to where
        more Gaussians are seen) or gave up a scan wait, the capacity is
        enlarged and the whole tracking run redone from T_init."""
        for attempt in range(3):
            if graph and (self.graph is None or any(a is not b for a, b in zip(self.graph_targets,
                                                                               (rgb_t, depth_t, labels)))):
                self.capture(rgb_t, depth_t, labels)
            self.set_pose(T_init)
            self.m.zero_()
            self.v.zero_()
            self.step.zero_()
            self.refresh()
            self.r.clear_trouble()
            for k in range(1, iters + 1):
                if graph:
                    self.graph.replay()
                else:
                    self.iteration(rgb_t, depth_t, labels, k)
                if k == 1:
                    # the loss terms at the starting pose (device copy, no sync)
                    self.first_terms = self.r.slam_terms.clone()
            self.last_terms = self.r.slam_terms.clone()  # at the pose before the last step
            if not self.r.trouble():
                return self.pose()
            # enlarge for the pose reached, with room to spare; the captured
            # graph holds the old buffers, so it is captured again
            self.r.set_capacity(max(2 * self.r.capacity, self.r.ensure_capacity(self.g, slack=2.0)))
            self.graph = None
        raise CapacityError("tracking kept overflowing the instance capacity")


class Mapper:
    """Mapping iterations over a set of keyframes (one view rendered per
    iteration) with Adam on every Gaussian parameter and the scale
    regulariser."""

    def __init__(self, r: raster.Rasterizer, g: raster.Gaussians, decoder: Optional[torch.Tensor] = None,
                 w_big: float = 0.01, w_small: float = 0.001, bias: Optional[torch.Tensor] = None,
                 learn_decoder: bool = False):
        assert r.views.n == 1
        self.r, self.g, self.decoder, self.bias = r, g, decoder, bias
        self.grads = g.zeros_like()
        self.m = g.zeros_like()
        self.v = g.zeros_like()
        self.w_big, self.w_small = w_big, w_small
        self.opts = _opts("mapping")
        self.step = 0
        # the decoder (W [F][K] and its bias [K]) in the same Adam steps
        self.learn_decoder = learn_decoder and decoder is not None
        if self.learn_decoder:
            assert bias is not None, "a learned decoder needs its bias tensor"
            self.dec_m = [torch.zeros_like(decoder), torch.zeros_like(bias)]
            self.dec_v = [torch.zeros_like(decoder), torch.zeros_like(bias)]

    def iteration(self, rgb_t, depth_t, labels, T: np.ndarray) -> torch.Tensor:
        r, g = self.r, self.g
        r.views.set_poses(torch.from_numpy(np.ascontiguousarray(T[:3, :4], np.float32)).to(r.device))
        r.project(g)
        r.bin_sort()
        r.render_fwd()
        r.slam_loss(rgb_t, depth_t, labels, self.decoder, self.opts, masks=True, bias=self.bias,
                    decoder_grads=self.learn_decoder)
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
        if self.learn_decoder:
            for p, gr, m, v in zip((self.decoder, self.bias), (r.grad_decoder_w, r.grad_decoder_b), self.dec_m,
                                   self.dec_v):
                groups.append(GsAdamGroup(p.data_ptr(), gr.data_ptr(), m.data_ptr(), v.data_ptr(), p.numel(),
                                          DECODER_LR, 0))
        arr = (GsAdamGroup * len(groups))(*groups)
        L = _lib.load()
        check(L.gs_adam_step(ctypes.cast(arr, ctypes.c_void_p), len(groups), ADAM_BETAS[0], ADAM_BETAS[1], ADAM_EPS,
                             self.step, raster._stream()), "gs_adam_step")
        return dsr_out

    def batch(self, frames: Sequence, poses: Sequence[np.ndarray]) -> None:
        """Mapping iterations over (frame, pose) pairs, frame = (rgb, depth,
        labels); afterwards one check of the sticky flag: CapacityError if
        any iteration's binning was truncated."""
        self.r.clear_trouble()
        for (rgb_t, depth_t, labels), T in zip(frames, poses):
            self.iteration(rgb_t, depth_t, labels, T)
        if self.r.trouble():
            raise CapacityError("a mapping iteration overflowed the instance capacity or gave up a scan wait; "
                                "enlarge the capacity (Rasterizer.set_capacity) and map again")


@dataclasses.dataclass
class Frame:
    """One RGB-D-semantic observation on the device: rgb [3][P], depth [P]
    (0 = no measurement), labels [P] int32."""
    rgb: torch.Tensor
    depth: torch.Tensor
    labels: torch.Tensor


PLANES = ("mu", "log_scale", "quat", "logit", "color", "feat")


class SlamRun:
    """The GS^3LAM loop over a sequence of frames of one pinhole camera
    (Sec. 3.3-3.4, schedule of Supp. C.1).

    process(frame) for the first frame: its pose T0 fixes the world frame;
    every pixel with a depth becomes a Gaussian (expansion with the map
    empty: M_unobs holds everywhere) and the map is optimised for init_iters
    mapping iterations.  For every later frame: the pose starts from the
    constant-velocity guess (Eq. 19; the previous pose for the second
    frame), is tracked against the frozen map (Eq. 20-21), the map grows at
    the frame's M_unobs pixels (Sec. 3.3.1-3.3.2), every kf_every-th frame
    joins the keyframe set, and map_iters mapping iterations follow, each on
    a frame RSKM picks (Eq. 13).  The decoder W, b is optimised with the
    field.  Adam's moments start afresh for each frame's tracking and
    mapping (the paper does not say whether they carry over).

    The map lives in contiguous [k][n] planes; growth appends into planes
    with room for one Gaussian per pixel (gs_expand counts on the device),
    reads the new count back once per frame and repacks."""

    def __init__(self, width: int, height: int, fx: float, fy: float, cx: float, cy: float, n_feat: int,
                 n_classes: int, cfg: Optional[raster.Config] = None, track_iters: int = TRACK_ITERS,
                 map_iters: int = MAP_ITERS, init_iters: Optional[int] = None, kf_every: int = 5, t_opt: int = 5,
                 seed: int = 0, device: str = "cuda"):
        self.W, self.H, self.fx, self.fy, self.cx, self.cy = width, height, fx, fy, cx, cy
        self.F, self.K = n_feat, n_classes
        self.cfg = cfg if cfg is not None else raster.Config()
        self.track_iters, self.map_iters = track_iters, map_iters
        self.init_iters = map_iters if init_iters is None else init_iters
        self.kf_every, self.t_opt = kf_every, t_opt
        self.rng = np.random.default_rng(seed)
        self.device = device
        dev = dict(device=device, dtype=torch.float32)
        self.planes = {"mu": torch.zeros(3, 0, **dev), "log_scale": torch.zeros(3, 0, **dev),
                       "quat": torch.zeros(4, 0, **dev), "logit": torch.zeros(0, **dev),
                       "color": torch.zeros(3, 0, **dev), "feat": torch.zeros(n_feat, 0, **dev)}
        W0 = self.rng.normal(size=(n_feat, n_classes)) / np.sqrt(max(n_feat, 1))
        self.decoder = torch.from_numpy(W0.astype(np.float32)).to(device)
        self.bias = torch.zeros(n_classes, **dev)
        self.poses: List[np.ndarray] = []
        self.track_losses: List = []  # per tracked frame: loss terms at the first and last iteration
        self.keyframes: List[int] = []
        self.frames: List[Frame] = []
        self.r: Optional[raster.Rasterizer] = None

    # ------------------------------------------------------------ map state
    @property
    def n(self) -> int:
        return int(self.planes["mu"].shape[1])

    def gaussians(self) -> raster.Gaussians:
        return raster.Gaussians(*(self.planes[k] for k in PLANES))

    def _view(self, T: np.ndarray):
        from .workloads import View
        return View(self.W, self.H, self.fx, self.fy, self.cx, self.cy, np.ascontiguousarray(T[:3, :4], np.float32))

    def _rasterizer(self, T: np.ndarray) -> raster.Rasterizer:
        """A rasterizer for the current map size, its instance capacity sized
        for every pose it will render this frame (the pose T and the
        keyframes' poses), with room to spare."""
        views = raster.Views([self._view(T)], self.cfg.tile, device=self.device)
        r = raster.Rasterizer(self.n, self.F, views, self.cfg, device=self.device)
        g = self.gaussians()
        need = 0
        for P in [T] + [self.poses[k] for k in self.keyframes]:
            r.views.set_poses(torch.from_numpy(np.ascontiguousarray(P[:3, :4], np.float32)).to(self.device))
            need = max(need, r.ensure_capacity(g, slack=1.5))
        r.set_capacity(int(need * 1.5) + 4096)
        return r

    def _grow(self, frame: Frame, T: np.ndarray) -> int:
        """Expansion at the frame's M_unobs pixels with a depth (everywhere
        when the map is empty); returns the number of Gaussians added."""
        P = self.W * self.H
        views = raster.Views([self._view(T)], self.cfg.tile, device=self.device)
        if self.n == 0:
            masks = torch.full((P,), 2, dtype=torch.uint8, device=self.device)  # M_unobs everywhere
        else:
            r = self.r
            r.views.set_poses(torch.from_numpy(np.ascontiguousarray(T[:3, :4], np.float32)).to(self.device))
            r.project(self.gaussians())
            r.bin_sort()
            r.render_fwd()
            r.slam_loss(frame.rgb, frame.depth, frame.labels, self.decoder, _opts("mapping"), masks=True,
                        bias=self.bias)
            masks = r.masks[:P]
        n0, cap = self.n, self.n + P
        big = {k: torch.zeros((t.shape[0], cap) if t.dim() == 2 else (cap,), dtype=t.dtype, device=self.device)
               for k, t in self.planes.items()}
        for k, t in self.planes.items():
            big[k][..., :n0] = t
        feat_init = torch.from_numpy(self.rng.normal(size=(max(self.F, 1), P)).astype(np.float32)).to(self.device)
        n_dev = torch.tensor([n0], dtype=torch.int64, device=self.device)
        raster.expand(views, masks, frame.rgb, frame.depth, feat_init, big, cap, n_dev, self.F)
        n1 = int(n_dev.item())
        self.planes = {k: t[..., :n1].contiguous() for k, t in big.items()}
        return n1 - n0

    # ---------------------------------------------------------------- steps
    def _map(self, current: int, iters: int) -> None:
        g = self.gaussians()
        mp = Mapper(self.r, g, self.decoder, bias=self.bias, learn_decoder=self.K > 0 and self.F > 0)
        frames, poses = [], []
        for k_m in range(iters):
            f = rskm_pick(self.rng, len(self.keyframes), -1, k_m, self.t_opt) if self.keyframes else -1
            idx = current if f < 0 else self.keyframes[f]
            fr = self.frames[idx]
            frames.append((fr.rgb, fr.depth, fr.labels))
            poses.append(self.poses[idx])
        mp.batch(frames, poses)

    def process(self, frame: Frame, T0: Optional[np.ndarray] = None) -> np.ndarray:
        """Tracks (or, for the first frame, places at T0) and maps one frame;
        returns its world-to-camera pose."""
        t = len(self.frames)
        self.frames.append(frame)
        if t == 0:
            T = np.asarray(T0 if T0 is not None else np.eye(4), np.float64)
            self.poses.append(T)
            self._grow(frame, T)
            self.keyframes.append(0)
            self.r = self._rasterizer(T)
            self._map(0, self.init_iters)
            return T
        T_init = constant_velocity(self.poses[-1], self.poses[-2]) if t >= 2 else self.poses[-1]
        self.r = self._rasterizer(T_init)
        tr = Tracker(self.r, self.gaussians(), self.decoder, bias=self.bias)
        T = tr.track(frame.rgb, frame.depth, frame.labels, T_init, self.track_iters)
        self.track_losses.append((tr.first_terms, tr.last_terms))
        self.poses.append(T)
        self._grow(frame, T)
        if t % self.kf_every == 0:
            self.keyframes.append(t)
        self.r = self._rasterizer(T)
        self._map(t, self.map_iters)
        return T
