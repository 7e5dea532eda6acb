"""FP64 CPU oracle for the semantic Gaussian-splatting rasterizer.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product library
never does, and this package never imports the product package.

The arithmetic lives in ``sgs_oracle.c`` (plain C, FP64 values, binary32
decisions); this module builds it with gcc, loads it with ctypes and
marshals numpy arrays.  ``bruteforce.py`` is a second, independent NumPy
renderer (no tiles, no boxes) used to pin the C oracle on tiny scenes.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sgs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle (gcc, -O2, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _lib.orc_bin.restype = ctypes.c_int64
        _lib.orc_total_tiles.restype = ctypes.c_int64
        _lib.orc_depth_median.restype = ctypes.c_float
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be contiguous"
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------
# configuration (readings of what the paper leaves unstated)
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Cfg:
    z_near: float = 0.2
    blur: float = 0.3
    guard: float = 1.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    tile: int = 16

    def array(self) -> np.ndarray:
        amin = float(np.float32(self.alpha_min))
        lmin = math.log(amin / (1.0 - amin))
        return np.array([self.z_near, self.blur, self.guard, self.alpha_min, self.alpha_max,
                         self.T_min, 0.0, lmin], dtype=np.float32)


def views_array(views, dtype=np.float32, poses64: Optional[List[np.ndarray]] = None) -> np.ndarray:
    """[V][18] = W, H, fx, fy, cx, cy, R (row-major), t, from the float32
    inputs (exactly upcast for dtype=float64).  `poses64` replaces [R|t] by
    FP64 3x4 matrices (finite differences of the pose)."""
    rows = []
    for i, v in enumerate(views):
        Rt = np.asarray(v.Rt, np.float32).astype(np.float64)
        if poses64 is not None:
            Rt = np.asarray(poses64[i], np.float64)[:3, :4]
        intr = np.float32([v.fx, v.fy, v.cx, v.cy]).astype(np.float64)
        rows.append(np.concatenate([[v.width, v.height], intr, Rt[:, :3].reshape(-1), Rt[:, 3]]))
    return np.ascontiguousarray(np.asarray(rows, dtype=np.float64), dtype=dtype)


def pixel_counts(views) -> np.ndarray:
    return np.array([v.width * v.height for v in views], dtype=np.int64)


def scene64(scene):
    """FP64 copy of a scene (exact upcast)."""
    return {k: np.ascontiguousarray(getattr(scene, k), dtype=np.float64)
            for k in ("mu", "log_scale", "quat", "logit", "color", "feat")}


# ----------------------------------------------------------------------------
# decisions and binning (binary32)
# ----------------------------------------------------------------------------
def decide(scene, views, cfg: Cfg):
    L = lib()
    n, V = scene.n, len(views)
    rect = np.zeros((V, n, 4), np.int32)
    touched = np.zeros((V, n), np.int32)
    dbits = np.zeros((V, n), np.uint32)
    rec32 = np.zeros((V, n, 8), np.float32)
    c = lambda a: np.ascontiguousarray(a, np.float32)
    mu, ls, q, lg = c(scene.mu), c(scene.log_scale), c(scene.quat), c(scene.logit)
    vw, ca = views_array(views), cfg.array()
    L.orc_decide(ctypes.c_int(n), _p(mu), _p(ls), _p(q), _p(lg), ctypes.c_int(V), _p(vw), _p(ca),
                 ctypes.c_int(cfg.tile), _p(rect), _p(touched), _p(dbits), _p(rec32))
    return {"rect": rect, "touched": touched, "dbits": dbits, "rec32": rec32}


def total_tiles(views, tile: int) -> int:
    return int(sum(((v.width + tile - 1) // tile) * ((v.height + tile - 1) // tile) for v in views))


def bin_instances(scene, views, cfg: Cfg, dec=None):
    """Sorted (tile, depth bits, gid) instances: keys (global tile id),
    gids, ranges[T][2] (start, end) and the count."""
    L = lib()
    dec = decide(scene, views, cfg) if dec is None else dec
    n, V = scene.n, len(views)
    count = int(dec["touched"].astype(np.int64).sum())
    T = total_tiles(views, cfg.tile)
    keys = np.zeros(max(count, 1), np.uint32)
    gids = np.zeros(max(count, 1), np.int32)
    ranges = np.zeros((T, 2), np.int32)
    got = L.orc_bin(ctypes.c_int(n), ctypes.c_int(V), _p(views_array(views)), ctypes.c_int(cfg.tile),
                    _p(dec["rect"]), _p(dec["touched"]), _p(dec["dbits"]), ctypes.c_int64(max(count, 1)),
                    _p(keys), _p(gids), _p(ranges))
    assert got == count
    return {"keys": keys[:count], "gids": gids[:count], "ranges": ranges, "count": count, "dec": dec}


# ----------------------------------------------------------------------------
# FP64 projection, render, loss, backward
# ----------------------------------------------------------------------------
def project64(scene, views, cfg: Cfg, s64=None, poses64=None) -> np.ndarray:
    L = lib()
    s64 = scene64(scene) if s64 is None else s64
    n, V = scene.n, len(views)
    proj = np.zeros((V, n, 7), np.float64)
    L.orc_project64(ctypes.c_int(n), _p(s64["mu"]), _p(s64["log_scale"]), _p(s64["quat"]), _p(s64["logit"]),
                    ctypes.c_int(V), _p(views_array(views, np.float64, poses64)), _p(cfg.array()), _p(proj))
    return proj


def project32(scene, views, cfg: Cfg, dec=None) -> np.ndarray:
    """[V][n][7] projection whose mean, conic and depth are the binary32
    decision-path values (upcast exactly) and whose opacity is FP64: the
    geometry the discrete alpha_min / T_min decisions of a binary32
    implementation are taken on."""
    dec = decide(scene, views, cfg) if dec is None else dec
    r = dec["rec32"].astype(np.float64)
    o = 1.0 / (1.0 + np.exp(-np.asarray(scene.logit, np.float32).astype(np.float64)))
    proj = np.zeros(r.shape[:2] + (7,))
    proj[..., 0:5] = r[..., 0:5]
    proj[..., 5] = o[None, :]
    proj[..., 6] = r[..., 5]
    return np.ascontiguousarray(proj)


def render(scene, views, cfg: Cfg, bins=None, pix_mask=None, s64=None, poses64=None, geometry="fp64"):
    """FP64 forward render.  Discrete decisions come from the binary32 scene
    and views; values from `s64` / `poses64` when given (finite differences).
    geometry="fp32" takes the projected mean, conic and depth from the
    binary32 decision path instead of the FP64 projection (used to compare a
    binary32 implementation away from threshold ties).
    Returns out[5+F][P] (R, G, B, depth, opacity, features), Tfinal, last,
    ncontrib, margin_a / margin_t (smallest relative distance to the
    alpha_min / T_min thresholds met at that pixel) and margin (their min)."""
    L = lib()
    bins = bin_instances(scene, views, cfg) if bins is None else bins
    s64 = scene64(scene) if s64 is None else s64
    if geometry == "fp32":
        proj = project32(scene, views, cfg, bins["dec"])
    else:
        proj = project64(scene, views, cfg, s64, poses64)
    F, n, V = scene.n_feat, scene.n, len(views)
    P = int(pixel_counts(views).sum())
    out = np.zeros((5 + F, P), np.float64)
    Tf = np.zeros(P, np.float64)
    last = np.zeros(P, np.int32)
    ncon = np.zeros(P, np.int32)
    ma = np.full(P, np.inf)
    mt = np.full(P, np.inf)
    gids = np.ascontiguousarray(bins["gids"] if bins["count"] else np.zeros(1, np.int32))
    pm = None if pix_mask is None else np.ascontiguousarray(pix_mask, np.uint8)
    L.orc_render(ctypes.c_int(n), ctypes.c_int(F), _p(s64["color"]), _p(s64["feat"]), ctypes.c_int(V),
                 _p(views_array(views, np.float64, poses64)), _p(cfg.array()), ctypes.c_int(cfg.tile),
                 _p(np.ascontiguousarray(bins["ranges"])), _p(gids), _p(proj), _p(pm), _p(out), _p(Tf),
                 _p(last), _p(ncon), _p(ma), _p(mt))
    return {"out": out, "Tfinal": Tf, "last": last, "ncontrib": ncon, "margin_a": ma, "margin_t": mt,
            "margin": np.minimum(ma, mt), "bins": bins, "proj": proj}


def loss(out: np.ndarray, views, rgb_t, depth_t, labels=None, decoder=None, weights=(0.5, 1.0, 0.0)):
    """Image-space loss and its gradient d L / d out (FP64)."""
    L = lib()
    F = out.shape[0] - 5
    K = 0 if decoder is None else int(decoder.shape[1])
    P = out.shape[1]
    g = np.zeros_like(out)
    terms = np.zeros(4, np.float64)
    lab = np.zeros(P, np.int32) if labels is None else np.ascontiguousarray(labels, np.int32)
    Wd = np.zeros((max(F, 1), 1)) if decoder is None else np.ascontiguousarray(decoder, np.float64)
    w = np.asarray(weights, np.float64)
    if K == 0:
        w = w.copy()
        w[2] = 0.0
    L.orc_loss(ctypes.c_int(F), ctypes.c_int(K), ctypes.c_int(len(views)), _p(pixel_counts(views)),
               _p(np.ascontiguousarray(out, np.float64)), _p(np.ascontiguousarray(rgb_t, np.float64)),
               _p(np.ascontiguousarray(depth_t, np.float64)), _p(lab), _p(Wd), _p(w), _p(g), _p(terms))
    return g, terms


@dataclasses.dataclass
class SlamLossOpts:
    """Weights and thresholds of the SLAM losses (Eq. 11, 15, 18, 21).

    tau_obs / tau_unobs are not stated in the paper; the defaults follow the
    silhouette thresholds of the SplaTAM work that the masks are modelled on.
    The residual factors 10 and 50 are Eq. (21)'s and Eq. (11)'s."""
    w_color: float = 0.5
    w_depth: float = 1.0
    w_sem: float = 0.01
    ssim_lambda: float = 0.2
    tau_obs: float = 0.99
    tau_unobs: float = 0.5
    obs_factor: float = 10.0
    unobs_factor: float = 50.0
    use_obs: bool = False
    bce: bool = False  # semantic term: BCE on softmax (Eq. 16) instead of CE

    def array(self) -> np.ndarray:
        # every value as the binary32 the device receives, upcast exactly
        v = [self.w_color, self.w_depth, self.w_sem, self.ssim_lambda, self.tau_obs, self.tau_unobs,
             self.obs_factor, self.unobs_factor]
        return np.array([float(np.float32(x)) for x in v] + [1.0 if self.use_obs else 0.0,
                                                              1.0 if self.bce else 0.0], np.float64)


def depth_median(depth, depth_t) -> np.float32:
    """Lower median of the binary32 residual |D - D*| over pixels with D* > 0."""
    d = np.ascontiguousarray(depth, np.float64)
    t = np.ascontiguousarray(depth_t, np.float64)
    return np.float32(lib().orc_depth_median(ctypes.c_int64(d.size), _p(d), _p(t)))


def ssim_map(x, y) -> np.ndarray:
    """Per-pixel SSIM of one H x W channel (11x11 Gaussian window, zero padding)."""
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    H, W = x.shape
    s = np.zeros_like(x)
    lib().orc_ssim_map(ctypes.c_int(W), ctypes.c_int(H), _p(x), _p(y), _p(s))
    return s


def slam_loss(out, wh, rgb_t, depth_t, labels=None, decoder=None, opts: SlamLossOpts = SlamLossOpts(),
              medians=None, norm_counts=None, bias=None, decoder_grads=False):
    """SLAM loss (Eq. 15 / 18 / 21) of views of sizes wh = [(W, H), ...].

    Returns (grad_out [5+F][P] FP64, terms[5] = colour L1, SSIM, depth,
    semantic, total; masks uint8 [P] = M_obs | M_unobs << 1; medians float32
    [V]), and with decoder_grads=True also (dL/dW [F][K], dL/db [K]).
    `medians` (float32 [V]) replaces the computed median depth errors and
    `norm_counts` the P_v of each view's means (crops of larger views);
    `bias` [K] is the decoder's bias (z = W^T f + b)."""
    L = lib()
    out = np.ascontiguousarray(out, np.float64)
    F = out.shape[0] - 5
    K = 0 if decoder is None else int(decoder.shape[1])
    P = out.shape[1]
    V = len(wh)
    whs = np.ascontiguousarray(np.asarray(wh, np.int32).reshape(V, 2))
    assert int((whs[:, 0].astype(np.int64) * whs[:, 1]).sum()) == P
    nc = (whs[:, 0].astype(np.int64) * whs[:, 1]) if norm_counts is None else np.asarray(norm_counts, np.int64)
    nc = np.ascontiguousarray(nc, np.int64)
    g = np.zeros_like(out)
    terms = np.zeros(5, np.float64)
    masks = np.zeros(P, np.uint8)
    med_out = np.zeros(V, np.float32)
    med_in = None if medians is None else np.ascontiguousarray(medians, np.float32)
    lab = np.zeros(P, np.int32) if labels is None else np.ascontiguousarray(labels, np.int32)
    Wd = np.zeros((max(F, 1), 1)) if decoder is None else np.ascontiguousarray(decoder, np.float64)
    o = opts.array()
    if K == 0:
        o[2] = 0.0
    bz = None if bias is None else np.ascontiguousarray(bias, np.float64)
    gW = np.zeros((max(F, 1), max(K, 1)))
    gb = np.zeros(max(K, 1))
    L.orc_slam_loss2(ctypes.c_int(F), ctypes.c_int(K), ctypes.c_int(V), _p(whs), _p(nc), _p(out),
                     _p(np.ascontiguousarray(rgb_t, np.float64)), _p(np.ascontiguousarray(depth_t, np.float64)),
                     _p(lab), _p(Wd), _p(bz), _p(o), _p(med_in), _p(med_out), _p(masks), _p(g), _p(terms), _p(gW),
                     _p(gb))
    if decoder_grads:
        return g, terms, masks, med_out, gW[:F, :K], gb[:K]
    return g, terms, masks, med_out


def expand(views, masks, rgb_t, depth_t, feat_init, n0: int, capacity: int, F: int):
    """Adaptive expansion (Sec. 3.3.1-3.3.2): new Gaussians at the pixels with
    M_unobs and a valid depth.  Returns (count of candidates, dict of FP64
    SoA planes with `capacity` columns; only columns [n0, n0 + count) capped
    at capacity are written)."""
    L = lib()
    va = views_array(views, np.float64)
    out = {"mu": np.zeros((3, capacity)), "log_scale": np.zeros((3, capacity)), "quat": np.zeros((4, capacity)),
           "logit": np.zeros(capacity), "color": np.zeros((3, capacity)), "feat": np.zeros((max(F, 1), capacity))}
    fi = np.ascontiguousarray(feat_init if F > 0 else np.zeros((1, 1)), np.float64)
    L.orc_expand.restype = ctypes.c_int64
    cnt = L.orc_expand(ctypes.c_int(F), ctypes.c_int(len(views)), _p(va), _p(np.ascontiguousarray(masks, np.uint8)),
                       _p(np.ascontiguousarray(rgb_t, np.float64)), _p(np.ascontiguousarray(depth_t, np.float64)),
                       _p(fi), ctypes.c_int64(n0), ctypes.c_int64(capacity), _p(out["mu"]), _p(out["log_scale"]),
                       _p(out["quat"]), _p(out["logit"]), _p(out["color"]), _p(out["feat"]))
    return int(cnt), out


def dsr(log_scale, w_big: float = 0.01, w_small: float = 0.001):
    """Depth-adaptive scale regularisation, Eq. (12), over the 3n per-axis
    scales; returns (dict of L_big, L_small, loss, mu, sigma, n_big, n_small;
    gradient with respect to log_scale, FP64 [3][n])."""
    ls = np.ascontiguousarray(log_scale, np.float32)
    g = np.zeros(ls.shape, np.float64)
    o = np.zeros(7)
    lib().orc_dsr(ctypes.c_int64(ls.size // 3), _p(ls), ctypes.c_double(w_big), ctypes.c_double(w_small), _p(g),
                  _p(o))
    keys = ("L_big", "L_small", "loss", "mu", "sigma", "n_big", "n_small")
    return dict(zip(keys, o.tolist())), g


def adam(p, g, m, v, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place on FP64 arrays (bias-corrected at step t >= 1)."""
    arrs = [np.ascontiguousarray(a, np.float64) for a in (p, g, m, v)]
    lib().orc_adam(ctypes.c_int64(arrs[0].size), _p(arrs[0]), _p(arrs[1]), _p(arrs[2]), _p(arrs[3]),
                   ctypes.c_double(lr), ctypes.c_double(b1), ctypes.c_double(b2), ctypes.c_double(eps), ctypes.c_int(t))
    return arrs[0], arrs[2], arrs[3]


def se3_exp(xi) -> np.ndarray:
    """3x4 [R|t] = Exp(xi), xi = (rho, phi)."""
    x = np.ascontiguousarray(xi, np.float64)
    out = np.zeros(12)
    lib().orc_se3_exp(_p(x), _p(out))
    return out.reshape(3, 4)


def pose_step(Rt, grad, m, v, lr_rho, lr_phi, t, b1=0.9, b2=0.999, eps=1e-8):
    """Tracking pose step for V views: Adam on the twist, then T <- Exp(dxi) T."""
    R = np.ascontiguousarray(Rt, np.float64).reshape(-1, 12).copy()
    gg = np.ascontiguousarray(grad, np.float64).reshape(-1, 6)
    mm = np.ascontiguousarray(m, np.float64).reshape(-1, 6).copy()
    vv = np.ascontiguousarray(v, np.float64).reshape(-1, 6).copy()
    lib().orc_pose_step(ctypes.c_int(R.shape[0]), _p(R), _p(gg), _p(mm), _p(vv), ctypes.c_double(lr_rho),
                        ctypes.c_double(lr_phi), ctypes.c_double(b1), ctypes.c_double(b2), ctypes.c_double(eps),
                        ctypes.c_int(t))
    return R.reshape(-1, 3, 4), mm, vv


GRAD_PARAMS = 1
GRAD_POSE = 2


def backward(scene, views, cfg: Cfg, grad_out: np.ndarray, bins=None, flags=GRAD_PARAMS | GRAD_POSE,
             tile_mask=None, s64=None, poses64=None, decisions="fp64"):
    """FP64 backward of <grad_out, render> to every parameter and the pose.
    decisions="fp32" takes each pixel's contributor set and stop (the
    alpha_min / T_min decisions) on the binary32 decision geometry, as
    render(geometry="fp32") does, while every value and derivative stays on
    the FP64 projection."""
    L = lib()
    bins = bin_instances(scene, views, cfg) if bins is None else bins
    s64 = scene64(scene) if s64 is None else s64
    proj = project64(scene, views, cfg, s64, poses64)
    dproj = project32(scene, views, cfg, bins["dec"]) if decisions == "fp32" else None
    F, n, V = scene.n_feat, scene.n, len(views)
    vis = np.ascontiguousarray((bins["dec"]["touched"] > 0).astype(np.uint8))
    r = {
        "grad2d": np.zeros((V, n, 6)), "gapp": np.zeros((n, 4 + F)),
        "mu": np.zeros((3, n)), "log_scale": np.zeros((3, n)), "quat": np.zeros((4, n)),
        "logit": np.zeros(n), "color": np.zeros((3, n)), "feat": np.zeros((F, n)),
        "gcam": np.zeros((V, n, 3)), "Gcam": np.zeros((V, n, 6)), "twist": np.zeros((V, 6)),
    }
    gids = np.ascontiguousarray(bins["gids"] if bins["count"] else np.zeros(1, np.int32))
    tm = None if tile_mask is None else np.ascontiguousarray(tile_mask, np.uint8)
    L.orc_backward(ctypes.c_int(n), ctypes.c_int(F), _p(s64["mu"]), _p(s64["log_scale"]), _p(s64["quat"]),
                   _p(s64["logit"]), _p(s64["color"]), _p(s64["feat"]), ctypes.c_int(V),
                   _p(views_array(views, np.float64, poses64)), _p(cfg.array()), ctypes.c_int(cfg.tile),
                   _p(np.ascontiguousarray(bins["ranges"])), _p(gids), _p(proj), _p(dproj),
                   _p(np.ascontiguousarray(grad_out, np.float64)), _p(tm), _p(vis), ctypes.c_int(flags),
                   _p(r["grad2d"]), _p(r["gapp"]), _p(r["mu"]), _p(r["log_scale"]), _p(r["quat"]),
                   _p(r["logit"]), _p(r["color"]), _p(r["feat"]), _p(r["gcam"]), _p(r["Gcam"]),
                   _p(r["twist"]))
    return r


def geom(mu, ls, q, logit, view, cfg: Cfg):
    """FP64 geometry of one pair: dict(p, Sigma, Sigma_c, Sigma2D, R, o)."""
    L = lib()
    out = np.zeros(34)
    vw = views_array([view], np.float64)[0].copy()
    L.orc_geom(_p(np.asarray(mu, np.float64).copy()), _p(np.asarray(ls, np.float64).copy()),
               _p(np.asarray(q, np.float64).copy()), ctypes.c_double(float(logit)), _p(vw),
               _p(cfg.array()), _p(out))
    return {"p": out[:3], "Sigma": out[3:12].reshape(3, 3), "Sigma_c": out[12:21].reshape(3, 3),
            "Sigma2D": out[21:24], "R": out[24:33].reshape(3, 3), "o": out[33]}


def dec_exp(x: np.ndarray) -> np.ndarray:
    L = lib()
    x = np.ascontiguousarray(x, np.float32)
    y = np.zeros_like(x)
    L.orc_dec_exp(ctypes.c_int(x.size), _p(x), _p(y))
    return y


def dec_log(x: np.ndarray) -> np.ndarray:
    """The decision path's binary32 natural logarithm (positive normal x)."""
    x = np.ascontiguousarray(x, np.float32)
    y = np.zeros_like(x)
    lib().orc_dec_log(ctypes.c_int(x.size), _p(x), _p(y))
    return y


def box_k(logit: np.ndarray, alpha_min: float = 1.0 / 255.0) -> np.ndarray:
    """Squared box radius (in standard deviations) of each opacity logit on
    the decision path, 2 ln(o / alpha_min) + 2^-8; 0 where o <= alpha_min."""
    x = np.ascontiguousarray(logit, np.float32)
    k = np.zeros_like(x)
    lib().orc_box_k(ctypes.c_int(x.size), _p(x), ctypes.c_float(float(np.float32(alpha_min))), _p(k))
    return k


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on."""
    lib().orc_set_num_threads(ctypes.c_int(int(n)))
