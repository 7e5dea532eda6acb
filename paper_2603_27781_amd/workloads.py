"""Seeded synthetic inputs for the semantic Gaussian-splatting rasterizer.

This module only *generates data*: Gaussian parameter arrays, camera poses,
image-space targets and class labels.  It contains none of the rasterizer's
arithmetic (no projection, no compositing, no gradients), so that both the
FP64 CPU oracle and the HIP path can consume the very same inputs without
sharing any of the method's code.

The scenes stand in for the paper's indoor RGB-D sequences (Replica at
1200x680 and ScanNet at 640x480, Sec. 4 "Experiments"), which are not used:
every array here is drawn from a seeded ``numpy.random.default_rng``.

Layouts (all float32, structure-of-arrays, Sec. 3.2 Eq. (1) "SG-Field"):
    mu[3][N], log_scale[3][N], quat[4][N] (w, x, y, z), logit[N],
    color[3][N], feat[F][N].
A view is a pinhole camera (W, H, fx, fy, cx, cy) plus a world->camera
rigid transform T_CW stored as a row-major 3x4 [R|t] (Sec. 3.2.1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


# ----------------------------------------------------------------------------
# containers
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Scene:
    mu: np.ndarray          # [3][N]
    log_scale: np.ndarray   # [3][N]
    quat: np.ndarray        # [4][N]  (w, x, y, z), not necessarily unit
    logit: np.ndarray       # [N]     opacity logit
    color: np.ndarray       # [3][N]
    feat: np.ndarray        # [F][N]

    @property
    def n(self) -> int:
        return int(self.mu.shape[1])

    @property
    def n_feat(self) -> int:
        return int(self.feat.shape[0])

    def copy(self) -> "Scene":
        return Scene(*(np.array(a, copy=True) for a in dataclasses.astuple(self)))

    def subset(self, idx: np.ndarray) -> "Scene":
        return Scene(self.mu[:, idx].copy(), self.log_scale[:, idx].copy(),
                     self.quat[:, idx].copy(), self.logit[idx].copy(),
                     self.color[:, idx].copy(), self.feat[:, idx].copy())


@dataclasses.dataclass
class View:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    Rt: np.ndarray          # [3][4] float32, world -> camera


@dataclasses.dataclass
class Targets:
    rgb: np.ndarray         # [3][P] float32
    depth: np.ndarray       # [P]    float32
    labels: np.ndarray      # [P]    int32 in [0, K)


@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    views: List[View]
    tile: int
    n_classes: int                      # K (0: no semantic term)
    decoder: Optional[np.ndarray]       # [F][K] float32 fixed linear decode
    weights: tuple                      # (lambda_c, lambda_d, lambda_s)
    pose_only: bool                     # tracking step: gradient to the pose only
    pose_grad: bool                     # twist gradients requested
    target_scene: Optional[Scene] = None  # seed-perturbed copy (targets are its render)
    target_views: Optional[List[View]] = None
    targets: Optional[Targets] = None   # analytic targets (room scenes)
    seed: int = 0

    @property
    def total_pixels(self) -> int:
        return sum(v.width * v.height for v in self.views)


# ----------------------------------------------------------------------------
# small pose helpers (input generation only)
# ----------------------------------------------------------------------------
def _hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def se3_exp(xi: np.ndarray) -> np.ndarray:
    """4x4 SE(3) exponential of a twist (rho, phi), translation first (FP64)."""
    rho = np.asarray(xi[:3], dtype=np.float64)
    phi = np.asarray(xi[3:], dtype=np.float64)
    th = float(np.linalg.norm(phi))
    K = _hat(phi)
    if th < 1e-12:
        R = np.eye(3) + K
        V = np.eye(3) + 0.5 * K
    else:
        A = math.sin(th) / th
        B = (1.0 - math.cos(th)) / th ** 2
        C = (th - math.sin(th)) / th ** 3
        R = np.eye(3) + A * K + B * (K @ K)
        V = np.eye(3) + B * K + C * (K @ K)
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = V @ rho
    return T


def look_from(center, forward, down) -> np.ndarray:
    """World->camera 4x4 for a camera at `center` (OpenCV axes: x right,
    y down, z forward)."""
    f = np.asarray(forward, np.float64)
    f = f / np.linalg.norm(f)
    d = np.asarray(down, np.float64)
    d = d - f * float(d @ f)
    d = d / np.linalg.norm(d)
    r = np.cross(d, f)
    Rwc = np.stack([r, d, f], axis=1)          # camera axes in world coords
    T = np.eye(4)
    T[:3, :3] = Rwc.T
    T[:3, 3] = -Rwc.T @ np.asarray(center, np.float64)
    return T


def make_view(W, H, f, T4, cx=None, cy=None) -> View:
    return View(int(W), int(H), float(f), float(f),
                float(W / 2 if cx is None else cx), float(H / 2 if cy is None else cy),
                np.ascontiguousarray(T4[:3, :4], dtype=np.float32))


def _random_twist(rng, rot, trans):
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    b = rng.normal(size=3)
    b /= np.linalg.norm(b)
    return np.concatenate([trans * b, rot * a])


def _unit_quats(rng, n):
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _quat_from_matrix(R):
    """Rotation matrices [n][3][3] -> unit quaternions [4][n] (w, x, y, z),
    choosing per matrix the numerically largest of the four candidates."""
    R = np.asarray(R, np.float64)
    m00, m11, m22 = R[:, 0, 0], R[:, 1, 1], R[:, 2, 2]
    tr = m00 + m11 + m22
    case = np.stack([tr, m00, m11, m22], axis=1).argmax(axis=1)
    q = np.zeros((R.shape[0], 4))
    c = case == 0
    s = np.sqrt(np.maximum(1.0 + tr[c], 1e-30)) * 2
    q[c] = np.stack([0.25 * s, (R[c, 2, 1] - R[c, 1, 2]) / s, (R[c, 0, 2] - R[c, 2, 0]) / s,
                     (R[c, 1, 0] - R[c, 0, 1]) / s], axis=1)
    c = case == 1
    s = np.sqrt(np.maximum(1.0 + m00[c] - m11[c] - m22[c], 1e-30)) * 2
    q[c] = np.stack([(R[c, 2, 1] - R[c, 1, 2]) / s, 0.25 * s, (R[c, 0, 1] + R[c, 1, 0]) / s,
                     (R[c, 0, 2] + R[c, 2, 0]) / s], axis=1)
    c = case == 2
    s = np.sqrt(np.maximum(1.0 + m11[c] - m00[c] - m22[c], 1e-30)) * 2
    q[c] = np.stack([(R[c, 0, 2] - R[c, 2, 0]) / s, (R[c, 0, 1] + R[c, 1, 0]) / s, 0.25 * s,
                     (R[c, 1, 2] + R[c, 2, 1]) / s], axis=1)
    c = case == 3
    s = np.sqrt(np.maximum(1.0 + m22[c] - m00[c] - m11[c], 1e-30)) * 2
    q[c] = np.stack([(R[c, 1, 0] - R[c, 0, 1]) / s, (R[c, 0, 2] + R[c, 2, 0]) / s,
                     (R[c, 1, 2] + R[c, 2, 1]) / s, 0.25 * s], axis=1)
    return q.T


def _quat_from_frames(e1, e2, n):
    """Quaternions of the frames with columns (e1, e2, n)."""
    return _quat_from_matrix(np.stack([e1, e2, n], axis=2))


# ----------------------------------------------------------------------------
# scene generators
# ----------------------------------------------------------------------------
def box_scene(rng, n, lo, hi, log_scale_mu, log_scale_sd, n_feat) -> Scene:
    mu = np.stack([rng.uniform(lo[k], hi[k], size=n) for k in range(3)])
    ls = rng.normal(log_scale_mu, log_scale_sd, size=(3, n))
    quat = _unit_quats(rng, n)
    logit = rng.normal(0.0, 1.0, size=n)
    color = rng.uniform(0.0, 1.0, size=(3, n))
    feat = rng.normal(0.0, 1.0, size=(n_feat, n))
    return Scene(*(np.ascontiguousarray(a, dtype=np.float32) for a in (mu, ls, quat, logit, color, feat)))


ROOM_LO = np.array([-4.0, 0.0, -4.0])
ROOM_HI = np.array([4.0, 3.0, 4.0])


def room_scene(rng, n, n_feat, lo=ROOM_LO, hi=ROOM_HI) -> Scene:
    """Surface Gaussians on the six faces of an axis-aligned room, drawn
    area-weighted; the local z axis is the inward normal (flat scale -7),
    the in-plane axes get a random angle and log-scales N(-4.5, 0.4)."""
    ext = hi - lo
    # faces: (axis, side)  side 0 -> at lo (normal +axis), side 1 -> at hi (normal -axis)
    faces = [(a, s) for a in range(3) for s in range(2)]
    areas = np.array([ext[(a + 1) % 3] * ext[(a + 2) % 3] for a, _ in faces])
    face = rng.choice(6, size=n, p=areas / areas.sum())
    u = rng.uniform(0.0, 1.0, size=(3, n))
    mu = lo[:, None] + u * ext[:, None]
    normal = np.zeros((n, 3))
    for fi, (a, s) in enumerate(faces):
        sel = face == fi
        mu[a, sel] = lo[a] if s == 0 else hi[a]
        normal[sel, a] = 1.0 if s == 0 else -1.0
    # tangent frame with a random in-plane angle
    ref = np.where(np.abs(normal[:, 1:2]) > 0.5, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
    t1 = np.cross(ref, normal)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(normal, t1)
    ang = rng.uniform(0.0, 2 * math.pi, size=n)
    c, s_ = np.cos(ang)[:, None], np.sin(ang)[:, None]
    e1 = c * t1 + s_ * t2
    e2 = np.cross(normal, e1)
    quat = _quat_from_frames(e1, e2, normal)
    flip = quat[0] < 0
    quat[:, flip] *= -1
    ls = np.stack([rng.normal(-4.5, 0.4, size=n), rng.normal(-4.5, 0.4, size=n), np.full(n, -7.0)])
    logit = rng.normal(0.0, 1.0, size=n)
    color = rng.uniform(0.0, 1.0, size=(3, n))
    feat = rng.normal(0.0, 1.0, size=(n_feat, n))
    return Scene(*(np.ascontiguousarray(a, dtype=np.float32) for a in (mu, ls, quat, logit, color, feat)))


def perturbed_copy(rng, sc: Scene) -> Scene:
    """Seed-perturbed copy of a scene; its render is the loss target."""
    n, F = sc.n, sc.n_feat
    out = sc.copy()
    out.mu += rng.normal(0, 0.02, size=(3, n)).astype(np.float32)
    out.log_scale += rng.normal(0, 0.05, size=(3, n)).astype(np.float32)
    out.logit += rng.normal(0, 0.1, size=n).astype(np.float32)
    out.color += rng.normal(0, 0.05, size=(3, n)).astype(np.float32)
    out.feat += rng.normal(0, 0.1, size=(F, n)).astype(np.float32)
    return out


def trajectory_poses(n_poses=100, height=1.5, radius=1.0) -> List[np.ndarray]:
    """Smooth yaw sweep of 2*pi at fixed height, looking radially outward."""
    poses = []
    for k in range(n_poses):
        th = 2 * math.pi * k / n_poses
        c = np.array([radius * math.cos(th), height, radius * math.sin(th)])
        fwd = np.array([math.cos(th), 0.0, math.sin(th)])
        poses.append(look_from(c, fwd, [0.0, -1.0, 0.0]))
    return poses


# ----------------------------------------------------------------------------
# analytic room targets (RGB-D + labels) for throughput runs
# ----------------------------------------------------------------------------
def room_targets(view: View, n_classes: int, lo=ROOM_LO, hi=ROOM_HI) -> Targets:
    """Ground-truth-like observation of the empty room: z-depth of the first
    wall hit along each pixel ray, a smooth per-wall colour texture and a
    label per (wall, texture cell).  Pure input generation."""
    W, H = view.width, view.height
    Rt = view.Rt.astype(np.float64)
    Rcw, t = Rt[:, :3], Rt[:, 3]
    center = -Rcw.T @ t
    u, v = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    dirs_c = np.stack([(u - view.cx) / view.fx, (v - view.cy) / view.fy, np.ones_like(u)], axis=0).reshape(3, -1)
    dirs_w = Rcw.T @ dirs_c                       # z-depth 1 rays in world
    best = np.full(dirs_w.shape[1], np.inf)
    wall = np.zeros(dirs_w.shape[1], np.int64)
    for a in range(3):
        for s, plane in enumerate((lo[a], hi[a])):
            with np.errstate(divide="ignore", invalid="ignore"):
                lam = (plane - center[a]) / dirs_w[a]
            ok = lam > 1e-6
            upd = ok & (lam < best)
            best[upd] = lam[upd]
            wall[upd] = 2 * a + s
    best[~np.isfinite(best)] = 0.0
    hit = center[:, None] + dirs_w * best[None]
    tex = np.sin(3.0 * hit[0]) * np.cos(2.0 * hit[1]) + np.sin(2.5 * hit[2])
    base = np.array([[0.8, 0.3, 0.3], [0.3, 0.8, 0.3], [0.3, 0.3, 0.8],
                     [0.8, 0.8, 0.3], [0.3, 0.8, 0.8], [0.8, 0.3, 0.8]])
    rgb = np.clip(base[wall].T * (0.75 + 0.2 * tex[None]), 0.0, 1.0)
    cell = (np.floor(hit[0] * 2) + np.floor(hit[1] * 2) * 3 + np.floor(hit[2] * 2) * 7).astype(np.int64)
    labels = ((wall * 5 + cell) % max(n_classes, 1)).astype(np.int32)
    return Targets(np.ascontiguousarray(rgb, np.float32), best.astype(np.float32), labels)


def decoder_matrix(rng, F, K) -> np.ndarray:
    return (rng.normal(size=(F, K)) / math.sqrt(F)).astype(np.float32)


@dataclasses.dataclass
class LossImages:
    """A render and its targets for the image-space losses alone (no scene):
    out[5+F][P] (colour, depth, opacity, feature planes), rgb_t[3][P],
    depth_t[P] (0 = no valid depth), labels[P]; views back to back."""
    out: np.ndarray
    rgb_t: np.ndarray
    depth_t: np.ndarray
    labels: np.ndarray
    sizes: List[tuple]


def loss_images(rng, sizes, F: int, K: int, missing: float = 0.02, front: float = 0.05,
                behind: float = 0.03) -> LossImages:
    """Smooth synthetic renders with noisy targets, shaped like a SLAM frame:
    colour fields of a few random waves in [0, 1] and targets a noisy copy;
    depth a tilted wavy surface at 1-3.5 m, observed with 1 cm noise, a
    fraction `front` of pixels observed further away (rendered geometry in
    front) and `behind` observed nearer (rendered geometry behind), and
    `missing` with no depth (0); opacity near 1 except a low-opacity blob (a
    region the map does not cover); features N(0, 1); labels uniform."""
    outs, rgbs, deps, labs = [], [], [], []
    for (W, H) in sizes:
        yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
        col = np.empty((3, H, W))
        for c in range(3):
            a = rng.uniform(0.05, 0.4, 2)
            col[c] = 0.5 + 0.25 * np.sin(a[0] * xx + rng.uniform(0, 6.3)) * np.cos(a[1] * yy + rng.uniform(0, 6.3))
            col[c] += 0.1 * np.sin(rng.uniform(0.5, 1.5) * (xx + yy))
        col = np.clip(col, 0.0, 1.0)
        rgb = np.clip(col + rng.normal(0, 0.05, col.shape), 0.0, 1.0)
        dep = 1.5 + 0.5 * np.sin(0.07 * xx + rng.uniform(0, 6.3)) + 1.0 * yy / max(H, 1)
        dt = dep + rng.normal(0, 0.01, dep.shape)
        u = rng.random(dep.shape)
        dt = np.where(u < front, dt + rng.uniform(0.3, 1.5, dep.shape), dt)
        dt = np.where((u >= front) & (u < front + behind), np.maximum(dt - rng.uniform(0.5, 1.0, dep.shape), 0.05),
                      dt)
        dt = np.where(rng.random(dep.shape) < missing, 0.0, dt)
        cx, cy, sg = rng.uniform(0, W), rng.uniform(0, H), 0.1 * max(W, H)
        op = np.clip(1.02 - 0.8 * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * sg * sg)), 0.0, 1.0)
        op = op - rng.uniform(0, 0.004, op.shape) * (op > 0.99)
        o = np.empty((5 + F, H * W))
        o[:3] = col.reshape(3, -1)
        o[3] = dep.reshape(-1)
        o[4] = op.reshape(-1)
        o[5:] = rng.normal(0, 1, (F, H * W))
        outs.append(o)
        rgbs.append(rgb.reshape(3, -1))
        deps.append(dt.reshape(-1))
        labs.append(rng.integers(0, max(K, 1), H * W))
    return LossImages(np.ascontiguousarray(np.concatenate(outs, 1), np.float32),
                      np.ascontiguousarray(np.concatenate(rgbs, 1), np.float32),
                      np.ascontiguousarray(np.concatenate(deps), np.float32),
                      np.ascontiguousarray(np.concatenate(labs), np.int32), list(sizes))


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
MAPPING_WEIGHTS = (0.5, 1.0, 0.01)    # Supp. C.1: lambda_c^m, lambda_d^m, lambda_s^m
TRACKING_WEIGHTS = (0.5, 1.0, 0.001)  # Supp. C.1: lambda_c^t, lambda_d^t, lambda_s^t


def config1(scale: float = 1.0) -> Workload:
    """64x64, 2,000 Gaussians in x,y in [-1,1], z in [2,4]; identity pose."""
    rng = np.random.default_rng(1)
    n = max(1, int(round(2000 * scale)))
    sc = box_scene(rng, n, (-1, -1, 2), (1, 1, 4), -3.0, 0.3, 16)
    T = np.eye(4)
    views = [make_view(64, 64, 64.0, T, 32.0, 32.0)]
    tgt = perturbed_copy(np.random.default_rng(101), sc)
    return Workload("cfg1-64x64-2k", sc, views, 16, 0, None, (0.5, 1.0, 0.0),
                    pose_only=False, pose_grad=True, target_scene=tgt, target_views=views, seed=1)


def config2(n: int = 200_000, width: int = 640, height: int = 480) -> Workload:
    """640x480, 200k Gaussians in a 6x3x6 m box in front of the camera,
    F=16, CE over 20 classes, pose = Exp(xi0) with |phi|=0.02, |rho|=0.02."""
    rng = np.random.default_rng(2)
    sc = box_scene(rng, n, (-3, -1.5, 1), (3, 1.5, 7), -4.0, 0.5, 16)
    f = 525.0 * width / 640.0
    T = se3_exp(_random_twist(rng, 0.02, 0.02))
    views = [make_view(width, height, f, T)]
    W = decoder_matrix(rng, 16, 20)
    labels = rng.integers(0, 20, size=width * height).astype(np.int32)
    tgt = perturbed_copy(np.random.default_rng(102), sc)
    tv = [make_view(width, height, f, np.eye(4))]
    wl = Workload("cfg2-640x480-200k", sc, views, 16, 20, W, MAPPING_WEIGHTS,
                  pose_only=False, pose_grad=True, target_scene=tgt, target_views=tv, seed=2)
    wl.targets = Targets(None, None, labels)
    return wl


def config3(n: int = 1_000_000, width: int = 1200, height: int = 680) -> Workload:
    """Tracking step: 1200x680, 1M room Gaussians, pose-only gradient."""
    rng = np.random.default_rng(3)
    sc = room_scene(rng, n, 16)
    f = 600.0 * width / 1200.0
    T_gt = look_from([0.0, 1.5, 0.0], [0.0, 0.0, 1.0], [0.0, -1.0, 0.0])
    T = se3_exp(_random_twist(rng, 0.02, 0.02)) @ T_gt
    W = decoder_matrix(rng, 16, 20)
    views = [make_view(width, height, f, T)]
    tv = [make_view(width, height, f, T_gt)]
    wl = Workload("cfg3-1200x680-1M-track", sc, views, 16, 20, W, TRACKING_WEIGHTS,
                  pose_only=True, pose_grad=True, target_scene=sc, target_views=tv, seed=3)
    # the analytic observation of the empty room at the true pose (throughput
    # runs); parity tests render their own targets at the true pose
    wl.targets = concat_targets([room_targets(v, 20) for v in tv])
    return wl


def config4(n: int = 1_000_000, n_views: int = 8, width: int = 1200, height: int = 680) -> Workload:
    """Batched mapping: 8 keyframes at 1200x680 drawn from a 100-pose yaw
    sweep, sharing 1M room Gaussians with F=16 (CE over 20 classes)."""
    rng = np.random.default_rng(4)
    sc = room_scene(rng, n, 16)
    W = decoder_matrix(rng, 16, 20)
    poses = trajectory_poses()
    pick = np.random.default_rng(204).choice(len(poses), size=n_views, replace=False)
    f = 600.0 * width / 1200.0
    views = [make_view(width, height, f, poses[k]) for k in pick]
    wl = Workload(f"cfg4-{n_views}x{width}x{height}-{n // 1000}k-batched", sc, views, 16, 20, W,
                  MAPPING_WEIGHTS, pose_only=False, pose_grad=False, seed=4)
    wl.targets = concat_targets([room_targets(v, 20) for v in views])
    return wl


RES5 = [(320, 240, 262.5), (640, 480, 525.0), (1200, 680, 600.0)]


def config5(n: int = 2_000_000, n_views: int = 16, res=None) -> Workload:
    """Uneven batched mapping: 16 views at mixed resolutions, 2M Gaussians,
    F=32, CE over 50 classes, pose gradients for every view."""
    rng = np.random.default_rng(5)
    sc = room_scene(rng, n, 32)
    W = decoder_matrix(rng, 32, 50)
    poses = trajectory_poses()
    krng = np.random.default_rng(205)
    pick = krng.choice(len(poses), size=n_views, replace=False)
    res = RES5 if res is None else res
    ridx = krng.integers(0, len(res), size=n_views)
    views = [make_view(res[r][0], res[r][1], res[r][2], poses[k]) for k, r in zip(pick, ridx)]
    wl = Workload(f"cfg5-{n_views}views-mixed-{n // 1000}k", sc, views, 16, 50, W, MAPPING_WEIGHTS,
                  pose_only=False, pose_grad=True, seed=5)
    wl.targets = concat_targets([room_targets(v, 50) for v in views])
    return wl


def concat_targets(ts: List[Targets]) -> Targets:
    return Targets(np.concatenate([t.rgb for t in ts], axis=1), np.concatenate([t.depth for t in ts]),
                   np.concatenate([t.labels for t in ts]))


def tiny_scene(seed: int, n: int, F: int = 8, W: int = 24, H: int = 20, f: float = 30.0,
               log_scale_mu: float = -2.2, spread: float = 0.7) -> Workload:
    """A few Gaussians in front of a small camera, for brute-force pins and
    finite differences."""
    rng = np.random.default_rng(seed)
    sc = box_scene(rng, n, (-spread, -spread, 2.0), (spread, spread, 3.5), log_scale_mu, 0.3, F)
    T = se3_exp(_random_twist(rng, 0.05, 0.05))
    views = [make_view(W, H, f, T)]
    return Workload(f"tiny-{seed}", sc, views, 8, 0, None, (0.5, 1.0, 0.0), pose_only=False,
                    pose_grad=True, seed=seed)


def get_config(idx: int, **kw) -> Workload:
    return {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}[idx](**kw)
