"""Torch-facing driver of the HIP rasterizer.

PyTorch provides device memory and the stream; every step of the path runs
in libsgs kernels called through the C ABI (see include/sgs.h).  A
`Rasterizer` owns the buffers of one workload shape (n Gaussians, F feature
channels, a fixed set of view sizes) so that a whole fwd+bwd step can be
captured once in a HIP graph and replayed; poses can change between replays
through `set_poses`.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, NamedTuple, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import GsConfig, GsGaussianGrads, GsGaussians, GsView, check

VIEW_WORDS = ctypes.sizeof(GsView) // 4  # 22 x 32-bit words per view


@dataclasses.dataclass
class Config:
    z_near: float = 0.2
    blur: float = 0.3
    guard: float = 1.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    tile: int = 16
    lds_batch: int = 256
    persistent: int = 0
    lds_batch_bwd: int = 0   # 0: same as lds_batch

    def c(self) -> GsConfig:
        return GsConfig(self.z_near, self.blur, self.guard, self.alpha_min, self.alpha_max, self.T_min, self.tile,
                        self.lds_batch, self.persistent, self.lds_batch_bwd)


@dataclasses.dataclass
class Gaussians:
    """FP32 structure-of-arrays planes on the GPU (GS^3LAM Eq. 1)."""
    mu: torch.Tensor         # [3][n]
    log_scale: torch.Tensor  # [3][n]
    quat: torch.Tensor       # [4][n]
    logit: torch.Tensor      # [n]
    color: torch.Tensor      # [3][n]
    feat: torch.Tensor       # [F][n]

    @property
    def n(self) -> int:
        return int(self.mu.shape[1])

    @property
    def n_feat(self) -> int:
        return int(self.feat.shape[0])

    @staticmethod
    def from_numpy(scene, device="cuda") -> "Gaussians":
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return Gaussians(t(scene.mu), t(scene.log_scale), t(scene.quat), t(scene.logit), t(scene.color),
                         t(scene.feat))

    def tensors(self):
        return [self.mu, self.log_scale, self.quat, self.logit, self.color, self.feat]

    def c(self) -> GsGaussians:
        for t in self.tensors():
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous(), "Gaussian planes: contiguous fp32 cuda"
        return GsGaussians(self.mu.data_ptr(), self.log_scale.data_ptr(), self.quat.data_ptr(), self.logit.data_ptr(),
                           self.color.data_ptr(), self.feat.data_ptr() if self.n_feat > 0 else None, self.n,
                           self.n_feat)

    def zeros_like(self) -> "Gaussians":
        return Gaussians(*(torch.zeros_like(t) for t in self.tensors()))


def _grads_c(gr: Gaussians) -> GsGaussianGrads:
    return GsGaussianGrads(gr.mu.data_ptr(), gr.log_scale.data_ptr(), gr.quat.data_ptr(), gr.logit.data_ptr(),
                           gr.color.data_ptr(), gr.feat.data_ptr() if gr.n_feat > 0 else None)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Views:
    """Host and device copies of the gs_view array (back-to-back layout)."""

    def __init__(self, views: Sequence, tile: int, device="cuda"):
        L = _lib.load()
        V = len(views)
        self.n = V
        self.tile = tile
        self.host = (GsView * V)()
        for i, v in enumerate(views):
            h = self.host[i]
            h.width, h.height = int(v.width), int(v.height)
            h.fx, h.fy, h.cx, h.cy = float(v.fx), float(v.fy), float(v.cx), float(v.cy)
            Rt = np.asarray(v.Rt, np.float32).reshape(-1)
            for k in range(12):
                h.Rt[k] = float(Rt[k])
        tp, tt = ctypes.c_int64(0), ctypes.c_int32(0)
        check(L.gs_views_layout(self.host, V, tile, ctypes.byref(tp), ctypes.byref(tt)), "gs_views_layout")
        self.total_pixels = int(tp.value)
        self.total_tiles = int(tt.value)
        raw = np.frombuffer(bytes(self.host), dtype=np.int32).reshape(V, VIEW_WORDS).copy()
        self.dev = torch.from_numpy(raw).to(device)
        self.sizes = [(int(v.width), int(v.height)) for v in views]

    def set_poses(self, Rts: torch.Tensor) -> None:
        """Overwrite the device poses ([V][3][4] float32, on the GPU) in place:
        graph-safe (a device copy into the buffer the captured kernels read)."""
        self.dev.view(torch.float32)[:, 6:18].copy_(Rts.reshape(self.n, 12))

    def dev_ptr(self):
        return ctypes.c_void_p(self.dev.data_ptr())

    def check(self) -> int:
        """Number of views whose device copy differs from the host array in
        the sizes, offsets or intrinsics (gs_views_check; the poses are not
        compared) -- synchronises."""
        out = torch.full((1,), -1, dtype=torch.int32, device=self.dev.device)
        check(_lib.load().gs_views_check(self.host, self.dev_ptr(), self.n, self.tile,
                                         ctypes.c_void_p(out.data_ptr()), _stream()), "gs_views_check")
        return int(out.item())


class BinCounts(NamedTuple):
    instances: int
    visible_pairs: int
    overflow: bool
    lookback_gave_up: bool


class Rasterizer:
    """Buffers and calls of one fwd+bwd pass for a fixed workload shape."""

    def __init__(self, n: int, n_feat: int, views: Views, cfg: Config, capacity: Optional[int] = None,
                 device="cuda"):
        L = _lib.load()
        self.L, self.n, self.F, self.views, self.cfg, self.device = L, n, n_feat, views, cfg, device
        self.cc = cfg.c()
        V, P = views.n, views.total_pixels
        self.AS = int(L.gs_app_stride(n_feat))
        dev = dict(device=device)
        self.rec = torch.empty(V * n * 8, dtype=torch.float32, **dev)
        self.rect = torch.empty(V * n * 4, dtype=torch.int32, **dev)
        self.touched = torch.empty(V * n, dtype=torch.int32, **dev)
        self.app = torch.empty(n * self.AS, dtype=torch.float32, **dev)
        self.counts = torch.zeros(5, dtype=torch.int64, **dev)
        self.ranges = torch.empty(views.total_tiles * 2, dtype=torch.int32, **dev)
        self.out = torch.empty(5 + n_feat, P, dtype=torch.float32, **dev)
        self.T_final = torch.empty(P, dtype=torch.float32, **dev)
        self.last = torch.empty(P, dtype=torch.int32, **dev)
        self.queue = torch.zeros(8, dtype=torch.int32, **dev)
        b, b2 = ctypes.c_size_t(0), ctypes.c_size_t(0)
        check(L.gs_render_bwd_workspace(n, n_feat, V, 1, _lib.GS_GRAD_PARAMS, ctypes.byref(b), ctypes.byref(b2)),
              "gs_render_bwd_workspace")
        self.grad2d = torch.empty(b.value // 4, dtype=torch.float32, **dev)
        self.pair_first = torch.empty(V * n, dtype=torch.int32, **dev)
        check(L.gs_pose_grad_workspace(n, V, ctypes.byref(b)), "gs_pose_grad_workspace")
        self.pose_ws = torch.empty(max(b.value, 16) // 8 + 1, dtype=torch.float64, **dev)
        self.twist = torch.zeros(V, 6, dtype=torch.float32, **dev)
        self.loss = torch.zeros(4, dtype=torch.float64, **dev)
        check(L.gs_loss_grad_workspace(P, ctypes.byref(b)), "gs_loss_grad_workspace")
        self.loss_ws = torch.empty(b.value // 8 + 2, dtype=torch.float64, **dev)
        self.grad_out = torch.empty_like(self.out)
        self.capacity = 0
        self.set_capacity(capacity if capacity is not None else max(4 * V * n, 1 << 16))

    # ------------------------------------------------------------------ buffers
    def set_capacity(self, capacity: int) -> None:
        capacity = int(capacity)
        if capacity == self.capacity:
            return
        b = ctypes.c_size_t(0)
        check(self.L.gs_bin_sort_workspace(self.n, self.views.n, capacity, ctypes.byref(b)), "gs_bin_sort_workspace")
        self.ws = torch.empty(b.value + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_view = self.ws[off:off + b.value]
        self.keys = torch.empty(max(capacity, 1), dtype=torch.int32, device=self.device)
        self.inst = torch.empty(max(capacity, 1), dtype=torch.int32, device=self.device)
        self.inst_gid = torch.empty(max(capacity, 1), dtype=torch.int32, device=self.device)
        g2, rb = ctypes.c_size_t(0), ctypes.c_size_t(0)
        check(self.L.gs_render_bwd_workspace(self.n, self.F, self.views.n, capacity, _lib.GS_GRAD_PARAMS,
                                             ctypes.byref(g2), ctypes.byref(rb)), "gs_render_bwd_workspace")
        self.records = torch.empty(rb.value // 4, dtype=torch.float32, device=self.device)
        self.capacity = capacity

    def sorted_gids(self, count: int) -> torch.Tensor:
        """Gaussian index of each of the first `count` sorted instances."""
        return self.inst_gid[self.inst[:count].long()]

    def instance_counts(self) -> "BinCounts":
        """(instances, visible pairs, capacity overflow, look-back gave up)
        of the last bin_sort -- synchronises."""
        c = self.counts.cpu().tolist()
        return BinCounts(int(c[0]), int(c[1]), bool(c[2]), bool(c[3]))

    def trouble(self) -> bool:
        """Whether any bin_sort since the last clear_trouble() overflowed its
        capacity or gave up a scan wait (the sticky flag) -- synchronises."""
        return bool(self.counts[4].item())

    def clear_trouble(self) -> None:
        """Clears the sticky flag (a fill kernel: safe inside a graph)."""
        self.counts[4:5].zero_()

    def ensure_capacity(self, g: Gaussians, slack: float = 1.25) -> int:
        """Run projection + binning once and size the instance buffers to the
        measured count times `slack` (one host synchronisation; call before
        capturing a graph, and again if the scene changes a lot)."""
        self.project(g)
        self.bin_sort()
        inst, _, over, gave_up = self.instance_counts()
        want = int(inst * slack) + 1024
        if over or inst > self.capacity or self.capacity > 2 * want:
            self.set_capacity(want)
            self.project(g)
            self.bin_sort()
        elif gave_up:
            self.bin_sort()
        return inst

    # -------------------------------------------------------------------- calls
    def project(self, g: Gaussians, write_app: bool = True) -> None:
        """gs_project; write_app False keeps the appearance records of the
        previous call (for a map whose colours and features have not changed)."""
        check(self.L.gs_project(ctypes.byref(g.c()), self.views.host, self.views.dev_ptr(), self.views.n,
                                ctypes.byref(self.cc), self.rec.data_ptr(), self.rect.data_ptr(),
                                self.touched.data_ptr(), self.app.data_ptr() if write_app else None, _stream()),
              "gs_project")

    def bin_sort(self) -> None:
        check(self.L.gs_bin_sort(self.rect.data_ptr(), self.touched.data_ptr(), self.n,
                                 self.views.host, self.views.dev_ptr(), self.views.n, ctypes.byref(self.cc),
                                 self.ws_view.data_ptr(), self.ws_view.numel(), self.capacity, self.keys.data_ptr(),
                                 self.inst.data_ptr(), self.inst_gid.data_ptr(), self.pair_first.data_ptr(),
                                 self.ranges.data_ptr(), self.counts.data_ptr(), _stream()), "gs_bin_sort")

    def render_fwd(self) -> None:
        check(self.L.gs_render_fwd(self.rec.data_ptr(), self.app.data_ptr(), self.n, self.F, self.inst.data_ptr(),
                                   self.inst_gid.data_ptr(), self.ranges.data_ptr(), self.views.host, self.views.dev_ptr(), self.views.n,
                                   ctypes.byref(self.cc), self.out.data_ptr(), self.T_final.data_ptr(),
                                   self.last.data_ptr(), self.queue.data_ptr(), _stream()), "gs_render_fwd")

    def forward(self, g: Gaussians) -> torch.Tensor:
        self.project(g)
        self.bin_sort()
        self.render_fwd()
        return self.out

    def loss_grad(self, rgb_t, depth_t, labels=None, decoder=None, weights=(0.5, 1.0, 0.0),
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """L1 colour + L1 depth + CE(W^T F) per view; writes self.grad_out and
        the loss terms (colour, depth, semantic, total) to self.loss."""
        out = self.out if out is None else out
        K = 0 if decoder is None else int(decoder.shape[1])
        w = (ctypes.c_float * 3)(*[float(x) for x in weights])
        check(self.L.gs_loss_grad(out.data_ptr(), self.F, rgb_t.data_ptr(), depth_t.data_ptr(),
                                  labels.data_ptr() if labels is not None else None,
                                  decoder.data_ptr() if decoder is not None else None, K, w, self.views.host,
                                  self.views.dev_ptr(), self.views.n, self.grad_out.data_ptr(),
                                  self.loss.data_ptr(), self.loss_ws.data_ptr(), self.loss_ws.numel() * 8,
                                  _stream()), "gs_loss_grad")
        return self.grad_out

    def fused_loss_supported(self, decoder=None) -> bool:
        K = 0 if decoder is None else int(decoder.shape[1])
        return self.F <= _lib.GS_FUSED_MAX_FEAT and K <= _lib.GS_FUSED_MAX_CLASSES

    def ensure_fused_ws(self) -> None:
        """Allocates the workspace of render_fwd_loss (before any graph capture)."""
        if getattr(self, "fused_ws", None) is None:
            b = ctypes.c_size_t(0)
            check(self.L.gs_render_fwd_loss_workspace(self.views.host, self.views.n, self.cfg.tile, ctypes.byref(b)),
                  "gs_render_fwd_loss_workspace")
            self.fused_ws = torch.empty(b.value // 8 + 2, dtype=torch.float64, device=self.out.device)

    def render_fwd_loss(self, rgb_t, depth_t, labels=None, decoder=None, weights=(0.5, 1.0, 0.0)) -> None:
        """render_fwd and loss_grad in one pass (gs_render_fwd_loss): writes
        self.out, T_final, last, self.grad_out and self.loss."""
        L = self.L
        self.ensure_fused_ws()
        K = 0 if decoder is None else int(decoder.shape[1])
        w = (ctypes.c_float * 3)(*[float(x) for x in weights])
        check(L.gs_render_fwd_loss(self.rec.data_ptr(), self.app.data_ptr(), self.n, self.F, self.inst.data_ptr(),
                                   self.inst_gid.data_ptr(), self.ranges.data_ptr(), self.views.host,
                                   self.views.dev_ptr(), self.views.n, ctypes.byref(self.cc), self.out.data_ptr(),
                                   self.T_final.data_ptr(), self.last.data_ptr(), self.queue.data_ptr(),
                                   rgb_t.data_ptr(), depth_t.data_ptr(),
                                   labels.data_ptr() if labels is not None else None,
                                   decoder.data_ptr() if decoder is not None else None, K, w,
                                   self.grad_out.data_ptr(), self.loss.data_ptr(), self.fused_ws.data_ptr(),
                                   self.fused_ws.numel() * 8, _stream()), "gs_render_fwd_loss")

    def slam_loss(self, rgb_t, depth_t, labels=None, decoder=None, opts=None,
                  out: Optional[torch.Tensor] = None, masks: bool = True, bias: Optional[torch.Tensor] = None,
                  decoder_grads: bool = False) -> torch.Tensor:
        """SLAM losses with masks (gs_slam_loss): writes self.grad_out, the
        terms (colour L1, SSIM, depth, semantic, total) to self.slam_terms,
        the per-view median depth error to self.median, with masks=True
        M_obs | M_unobs << 1 per pixel to self.masks and, with
        decoder_grads=True, dL/dW and dL/db of the decoder (W [F][K], bias
        [K] or None) to self.grad_decoder_w / self.grad_decoder_b.  `opts`
        is a GsSlamLossOpts (default: gs_default_slam_loss_opts)."""
        out = self.out if out is None else out
        L = self.L
        if opts is None:
            opts = _lib.GsSlamLossOpts()
            check(L.gs_default_slam_loss_opts(ctypes.byref(opts)), "gs_default_slam_loss_opts")
        K = 0 if decoder is None else int(decoder.shape[1])
        dev = dict(device=self.device)
        dec = None
        if decoder is not None:
            dec = _lib.GsDecoder(decoder.data_ptr(), bias.data_ptr() if bias is not None else None, None, None, K, 0)
            if decoder_grads:
                if getattr(self, "grad_decoder_w", None) is None or self.grad_decoder_w.shape != (self.F, K):
                    self.grad_decoder_w = torch.zeros(max(self.F, 1), K, dtype=torch.float32, **dev)[:self.F]
                    self.grad_decoder_b = torch.zeros(K, dtype=torch.float32, **dev)
                dec.grad_weight = self.grad_decoder_w.data_ptr()
                dec.grad_bias = self.grad_decoder_b.data_ptr()
        pdec = ctypes.byref(dec) if dec is not None else None
        b = ctypes.c_size_t(0)
        check(L.gs_slam_loss_workspace(self.views.host, self.views.n, self.F, pdec, ctypes.byref(opts),
                                       ctypes.byref(b)), "gs_slam_loss_workspace")
        if getattr(self, "slam_ws", None) is None or self.slam_ws_bytes < b.value:
            self.slam_ws = torch.empty(b.value + 256, dtype=torch.uint8, **dev)
            self.slam_ws_bytes = b.value
        off = (-self.slam_ws.data_ptr()) % 256
        if getattr(self, "slam_terms", None) is None:
            self.slam_terms = torch.zeros(5, dtype=torch.float64, **dev)
            self.median = torch.zeros(self.views.n, dtype=torch.float32, **dev)
            self.masks = torch.zeros(self.views.total_pixels, dtype=torch.uint8, **dev)
        check(L.gs_slam_loss(out.data_ptr(), self.F, rgb_t.data_ptr(), depth_t.data_ptr(),
                             labels.data_ptr() if labels is not None else None, pdec, ctypes.byref(opts),
                             self.views.host, self.views.dev_ptr(), self.views.n, self.grad_out.data_ptr(),
                             self.slam_terms.data_ptr(), self.median.data_ptr(),
                             self.masks.data_ptr() if masks else None, self.slam_ws.data_ptr() + off,
                             self.slam_ws_bytes, _stream()), "gs_slam_loss")
        return self.grad_out

    def render_bwd(self, g: Gaussians, grad_out: torch.Tensor, flags: int, grads: Optional[Gaussians],
                   write: bool = False) -> None:
        """Backward of the compositing into the 2D gradient buffer and, with
        GS_GRAD_PARAMS, of the projection into `grads` (+=, or = with write)."""
        self.render_bwd_2d(g, grad_out, flags)
        if flags & _lib.GS_GRAD_PARAMS:
            self.project_bwd(g, grads, write)

    def render_bwd_2d(self, g: Gaussians, grad_out: torch.Tensor, flags: int) -> None:
        check(self.L.gs_render_bwd(ctypes.byref(g.c()), self.rec.data_ptr(), self.app.data_ptr(),
                                   self.inst.data_ptr(), self.inst_gid.data_ptr(), self.pair_first.data_ptr(),
                                   self.touched.data_ptr(), self.capacity, self.ranges.data_ptr(), self.views.host,
                                   self.views.dev_ptr(), self.views.n, ctypes.byref(self.cc),
                                   self.T_final.data_ptr(), self.last.data_ptr(), grad_out.data_ptr(), flags,
                                   self.grad2d.data_ptr(), self.grad2d.numel() * 4, self.records.data_ptr(),
                                   self.records.numel() * 4, self.queue.data_ptr(), _stream()), "gs_render_bwd")

    def render_bwd_records(self, g: Gaussians, grad_out: torch.Tensor, flags: int) -> None:
        """First half of render_bwd_2d: per-instance records only."""
        check(self.L.gs_render_bwd_records(ctypes.byref(g.c()), self.rec.data_ptr(), self.app.data_ptr(),
                                           self.inst.data_ptr(), self.inst_gid.data_ptr(), self.capacity,
                                           self.ranges.data_ptr(), self.views.host, self.views.dev_ptr(), self.views.n,
                                           ctypes.byref(self.cc), self.T_final.data_ptr(), self.last.data_ptr(),
                                           grad_out.data_ptr(), flags, self.records.data_ptr(),
                                           self.records.numel() * 4, self.queue.data_ptr(), _stream()),
              "gs_render_bwd_records")

    def reduce_records(self, flags: int) -> None:
        """Second half of render_bwd_2d: records -> grad2d."""
        check(self.L.gs_reduce_records(self.records.data_ptr(), self.records.numel() * 4, self.pair_first.data_ptr(),
                                       self.touched.data_ptr(), self.n, self.F, self.views.n, self.capacity, flags,
                                       self.grad2d.data_ptr(), self.grad2d.numel() * 4, _stream()),
              "gs_reduce_records")

    def project_bwd(self, g: Gaussians, grads: Gaussians, write: bool = False) -> None:
        """gs_project_bwd (adds to `grads`), or gs_project_bwd_write (writes them)."""
        gc = _grads_c(grads)
        fn = self.L.gs_project_bwd_write if write else self.L.gs_project_bwd
        check(fn(ctypes.byref(g.c()), self.views.host, self.views.dev_ptr(), self.views.n, ctypes.byref(self.cc),
                 self.touched.data_ptr(), self.grad2d.data_ptr(), self.grad2d.numel() * 4, ctypes.byref(gc),
                 _stream()), "gs_project_bwd_write" if write else "gs_project_bwd")

    def pose_grad(self, g: Gaussians, noalloc: bool = False) -> torch.Tensor:
        """gs_pose_grad into self.twist; noalloc=True calls
        gs_pose_grad_noalloc (the library's own scratch, no workspace)."""
        if noalloc:
            check(self.L.gs_pose_grad_noalloc(ctypes.byref(g.c()), self.views.host, self.views.dev_ptr(),
                                              self.views.n, ctypes.byref(self.cc), self.touched.data_ptr(),
                                              self.grad2d.data_ptr(), self.twist.data_ptr(), _stream()),
                  "gs_pose_grad_noalloc")
            return self.twist
        check(self.L.gs_pose_grad(ctypes.byref(g.c()), self.views.host, self.views.dev_ptr(), self.views.n,
                                  ctypes.byref(self.cc), self.touched.data_ptr(), self.grad2d.data_ptr(),
                                  self.pose_ws.data_ptr(), self.pose_ws.numel() * 8, self.twist.data_ptr(),
                                  _stream()), "gs_pose_grad")
        return self.twist

    # ------------------------------------------------------------ views of state
    @property
    def grad_geo(self) -> torch.Tensor:
        """[V][n][8] 2D gradients; entries of pairs that are not visible are
        zeroed here (the library leaves them unwritten)."""
        geo = self.grad2d[: self.views.n * self.n * 8].view(self.views.n, self.n, 8)
        vis = self.touched[: self.views.n * self.n].view(self.views.n, self.n, 1) > 0
        return torch.where(vis, geo, torch.zeros((), dtype=geo.dtype, device=geo.device))

    @property
    def grad_app(self) -> torch.Tensor:
        o = self.views.n * self.n * 8
        return self.grad2d[o: o + self.n * (4 + self.F)].view(self.n, 4 + self.F)

    def n_instances_dev(self) -> torch.Tensor:
        return self.counts[0]


class RasterizeFunction(torch.autograd.Function):
    """Autograd wrapper: inputs (xi, mu, log_scale, quat, logit, color, feat),
    output the planar image [5+F][P].  `xi` is a [V][6] twist placeholder
    whose value is not applied (render at the poses held by the rasterizer's
    views; update them between steps with Views.set_poses); its gradient is
    the twist gradient of the left perturbation Exp(xi) T_CW at xi = 0."""

    @staticmethod
    def forward(ctx, rast: Rasterizer, xi, mu, log_scale, quat, logit, color, feat):
        g = Gaussians(mu.detach().contiguous(), log_scale.detach().contiguous(), quat.detach().contiguous(),
                      logit.detach().contiguous(), color.detach().contiguous(), feat.detach().contiguous())
        rast.forward(g)
        ctx.rast = rast
        ctx.g = g
        ctx.want_pose = xi is not None and xi.requires_grad
        return rast.out.clone()

    @staticmethod
    def backward(ctx, grad_out):
        rast, g = ctx.rast, ctx.g
        need_params = any(ctx.needs_input_grad[2:8])
        flags = (_lib.GS_GRAD_PARAMS if need_params else 0) | (_lib.GS_GRAD_POSE if ctx.want_pose else 0)
        if flags == 0:
            return (None,) * 8
        grads = g.zeros_like() if need_params else None
        rast.render_bwd(g, grad_out.contiguous(), flags, grads)
        gxi = rast.pose_grad(g).clone() if ctx.want_pose else None
        if grads is None:
            return (None, gxi) + (None,) * 6
        return (None, gxi, grads.mu, grads.log_scale, grads.quat, grads.logit, grads.color, grads.feat)


def rasterize(rast: Rasterizer, xi, mu, log_scale, quat, logit, color, feat) -> torch.Tensor:
    return RasterizeFunction.apply(rast, xi, mu, log_scale, quat, logit, color, feat)


# ---------------------------------------------------------------------------
# map growth and scale regularisation (Sec. 3.3.1-3.3.2)
# ---------------------------------------------------------------------------
def expand(views: Views, masks, rgb_t, depth_t, feat_init, planes: dict, capacity: int, n_dev: torch.Tensor,
           n_feat: int, candidates: Optional[torch.Tensor] = None) -> None:
    """gs_expand: appends Gaussians for the pixels with M_unobs and a valid
    depth to `planes` (device tensors mu [3][cap], log_scale [3][cap],
    quat [4][cap], logit [cap], color [3][cap], feat [F][cap]); n_dev (int64
    device scalar) is the count, updated on the device."""
    L = _lib.load()
    b = ctypes.c_size_t(0)
    check(L.gs_expand_workspace(views.total_pixels, ctypes.byref(b)), "gs_expand_workspace")
    ws = torch.empty(b.value + 256, dtype=torch.uint8, device=masks.device)
    off = (-ws.data_ptr()) % 256
    dst = GsGaussianGrads(planes["mu"].data_ptr(), planes["log_scale"].data_ptr(), planes["quat"].data_ptr(),
                          planes["logit"].data_ptr(), planes["color"].data_ptr(),
                          planes["feat"].data_ptr() if n_feat > 0 else None)
    check(L.gs_expand(masks.data_ptr(), rgb_t.data_ptr(), depth_t.data_ptr(),
                      feat_init.data_ptr() if feat_init is not None else None, n_feat, views.host, views.dev_ptr(),
                      views.n, ctypes.byref(dst), capacity, n_dev.data_ptr(),
                      candidates.data_ptr() if candidates is not None else None, ws.data_ptr() + off, b.value,
                      _stream()), "gs_expand")


def dsr(log_scale: torch.Tensor, w_big: float = 0.01, w_small: float = 0.001,
        grad_log_scale: Optional[torch.Tensor] = None) -> torch.Tensor:
    """gs_dsr: Eq. (12) over log_scale [3][n]; returns the device double[7]
    (L_big, L_small, loss, mu, sigma, n_big, n_small) and accumulates the
    gradient into grad_log_scale when given."""
    L = _lib.load()
    n = log_scale.shape[-1]
    b = ctypes.c_size_t(0)
    check(L.gs_dsr_workspace(n, ctypes.byref(b)), "gs_dsr_workspace")
    ws = torch.empty(b.value + 256, dtype=torch.uint8, device=log_scale.device)
    off = (-ws.data_ptr()) % 256
    out = torch.zeros(7, dtype=torch.float64, device=log_scale.device)
    check(L.gs_dsr(log_scale.data_ptr(), n, w_big, w_small,
                   grad_log_scale.data_ptr() if grad_log_scale is not None else None, out.data_ptr(),
                   ws.data_ptr() + off, b.value, _stream()), "gs_dsr")
    return out

