"""Brute-force FP64 renderer in plain PyTorch (CPU), differentiable by autograd.

TEST INFRASTRUCTURE ONLY -- an independent second implementation used to pin
the C oracle on tiny scenes.  It has no tiles and no bounding boxes: every
pixel considers every Gaussian that survives culling, in (binary32 depth,
index) order, and composites front to back (GS^3LAM Sec. 3.2.1 Eq. (4)-(7),
Sec. 3.3.1 Eq. (10)).  Gradients come from torch.autograd, not from any
hand-derived chain rule, so they pin the oracle's analytic backward.

The discrete decisions (culling, alpha_min skip, T_min stop) are taken on
detached FP64 values; with the pose entering as T(xi) = (I + xi^) T_CW, the
gradient with respect to xi at xi = 0 equals the twist gradient of the left
perturbation Exp(xi) T_CW.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def _hat(w):
    z = torch.zeros((), dtype=w.dtype)
    return torch.stack([torch.stack([z, -w[2], w[1]]), torch.stack([w[2], z, -w[0]]),
                        torch.stack([-w[1], w[0], z])])


def render(mu, log_scale, quat, logit, color, feat, view, xi=None, *, z_near=0.2, blur=0.3, guard=1.3,
           alpha_min=1.0 / 255.0, alpha_max=0.99, T_min=1e-4):
    """All tensors FP64.  mu[3][N], log_scale[3][N], quat[4][N], logit[N],
    color[3][N], feat[F][N]; view has width, height, fx, fy, cx, cy, Rt.
    Returns out[5+F][H*W] (R, G, B, depth, opacity, features) and T_final."""
    dt = torch.float64
    # the configuration crosses the C ABI as binary32: use the same values
    z_near, blur, guard, alpha_min, alpha_max, T_min = (
        float(np.float32(v)) for v in (z_near, blur, guard, alpha_min, alpha_max, T_min))
    W, H = view.width, view.height
    fx, fy, cx, cy = (float(np.float32(v)) for v in (view.fx, view.fy, view.cx, view.cy))
    Rt = torch.tensor(np.asarray(view.Rt, np.float32).astype(np.float64), dtype=dt)
    Rc, tc = Rt[:, :3], Rt[:, 3]
    if xi is not None:
        A = torch.eye(3, dtype=dt) + _hat(xi[3:])
        Rc = A @ Rc
        tc = A @ tc + xi[:3]
    # camera-space mean and depth
    p = Rc @ mu + tc[:, None]
    x, y, z = p[0], p[1], p[2]
    # covariance from quaternion and scales
    qn = quat / torch.linalg.norm(quat, dim=0, keepdim=True)
    w, qx, qy, qz = qn
    R = torch.stack([
        torch.stack([1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - w * qz), 2 * (qx * qz + w * qy)]),
        torch.stack([2 * (qx * qy + w * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - w * qx)]),
        torch.stack([2 * (qx * qz - w * qy), 2 * (qy * qz + w * qx), 1 - 2 * (qx * qx + qy * qy)]),
    ])                                                  # [3][3][N]
    s = torch.exp(log_scale)                            # [3][N]
    M = R * s[None, :, :]
    Sig = torch.einsum("ikn,jkn->ijn", M, M)
    Sc = torch.einsum("ia,abn,jb->ijn", Rc, Sig, Rc)
    zero = torch.zeros_like(z)
    J = torch.stack([torch.stack([fx / z, zero, -fx * x / z ** 2]),
                     torch.stack([zero, fy / z, -fy * y / z ** 2])])  # [2][3][N]
    S2 = torch.einsum("ian,abn,jbn->ijn", J, Sc, J)
    a = S2[0, 0] + blur
    b = S2[0, 1]
    c = S2[1, 1] + blur
    det = a * c - b * b
    cA, cB, cC = c / det, -b / det, a / det
    mx = fx * x / z + cx
    my = fy * y / z + cy
    o = torch.sigmoid(logit)
    # culling (readings: opacity, near plane, frustum guard, degenerate conic)
    with torch.no_grad():
        limx = guard * 0.5 * W / fx
        limy = guard * 0.5 * H / fy
        keep = (o > alpha_min) & (z > z_near) & ((x / z).abs() <= limx) & ((y / z).abs() <= limy) & (det > 0)
        idx = torch.nonzero(keep).flatten().tolist()
        z32 = z.detach().numpy().astype(np.float32)
        idx.sort(key=lambda i: (z32[i], i))
    F = feat.shape[0]
    P = W * H
    uu, vv = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    px = torch.tensor(uu.reshape(-1), dtype=dt)
    py = torch.tensor(vv.reshape(-1), dtype=dt)
    T = torch.ones(P, dtype=dt)
    done = torch.zeros(P, dtype=torch.bool)
    acc = [torch.zeros(P, dtype=dt) for _ in range(5 + F)]
    for i in idx:
        dx = px - mx[i]
        dy = py - my[i]
        q = cA[i] * dx * dx + 2 * cB[i] * dx * dy + cC[i] * dy * dy
        q = torch.clamp(q, min=0.0)
        al = torch.clamp(o[i] * torch.exp(-0.5 * q), max=alpha_max)
        with torch.no_grad():
            inc = (~done) & (al >= alpha_min)
            stop = inc & (T.detach() * (1 - al.detach()) < T_min)
            inc = inc & ~stop
            done = done | stop
        m = inc.to(dt)
        wgt = al * T * m
        vals = [color[0, i], color[1, i], color[2, i], z[i], None] + [feat[f, i] for f in range(F)]
        for ch in range(5 + F):
            acc[ch] = acc[ch] + (wgt if ch == 4 else wgt * vals[ch])
        T = T * (1 - al * m)
    return torch.stack(acc), T


def as_tensors(scene, requires_grad=False):
    ts = [torch.tensor(np.asarray(getattr(scene, k), np.float64)) for k in
          ("mu", "log_scale", "quat", "logit", "color", "feat")]
    for t in ts:
        t.requires_grad_(requires_grad)
    return ts
