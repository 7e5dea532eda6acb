"""Shared helpers of the GPU parity tests (HIP path through the C ABI versus
the FP64 CPU oracle on the same seeded inputs)."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2603_27781_amd import workloads as wl

# tolerances (stated for the path): RGB and opacity max-abs 1e-5; depth and
# features 1e-4 of the channel's max |oracle|; gradients 1e-3 of the
# tensor's max |oracle|.
TOL_RGB = 1e-5
TOL_REL_DF = 1e-4
TOL_GRAD = 1e-3
# Binary32 and FP64 may take a pixel's alpha_min / T_min decisions
# differently only where a decision lies within the binary32 evaluation
# error of its threshold.  Every pixel is held to the tolerances above; a
# pixel that misses them (or whose last contributor differs) is excused only
# if the oracle shows a decision within these relative margins of its
# threshold and the deviation stays within what flipped decisions can cause.
#  - against the oracle on the binary32 projected geometry (mean, conic,
#    depth as the decision path computes them): only the kernel's binary32
#    alpha (hardware exp2, a few ulp) and transmittance products differ,
MARGIN_A32, MARGIN_T32 = 1e-5, 1e-4
#  - against the oracle on the FP64 geometry: the binary32 mean alone is
#    off by up to half an ulp of ~1e3 px, i.e. ~3e-5 px, so alpha can differ
#    by ~1e-4 relatively near the box edge.
MARGIN_A64, MARGIN_T64 = 1e-3, 1e-3
MARGIN = MARGIN_A64


def gpu_setup(scene, views, cfg_kw=None, capacity=None):
    import torch
    from paper_2603_27781_amd import raster
    cfg = raster.Config(**(cfg_kw or {}))
    V = raster.Views(views, cfg.tile)
    g = raster.Gaussians.from_numpy(scene)
    r = raster.Rasterizer(scene.n, scene.n_feat, V, cfg, capacity=capacity)
    return r, g, cfg


def oracle_cfg(cfg) -> oracle.Cfg:
    return oracle.Cfg(z_near=cfg.z_near, blur=cfg.blur, guard=cfg.guard, alpha_min=cfg.alpha_min,
                      alpha_max=cfg.alpha_max, T_min=cfg.T_min, tile=cfg.tile)


def chan_scales(scene, proj_depth_max):
    """max |x| per output channel over the scene (colour, depth, opacity 1,
    features): the size of one Gaussian's contribution to a channel."""
    c = float(np.max(np.abs(scene.color))) if scene.n else 1.0
    f = np.max(np.abs(scene.feat), axis=1) if scene.n_feat else np.zeros(0)
    return np.concatenate([[c, c, c, proj_depth_max, 1.0], f])


def compare_render(out_gpu, T_gpu, last_gpu, ref, sel=None, geometry="fp32", scales=None, cfg=None,
                   max_flipped=None):
    """Holds every pixel of `sel` (default all) to the tolerances: RGB,
    opacity and T_final within 1e-5 max-abs, depth and features within 1e-4
    of the channel's max |oracle|, the last contributor equal.  A pixel that
    misses them is excused only as a flipped threshold decision: the oracle
    must show one of its alpha_min / T_min decisions within the margin of
    its threshold, and its deviation must stay within the flipped-decision
    bound (one flipped alpha_min decision moves a channel by at most
    2 alpha_min max|x|, its own weight and the (1 - alpha) it puts on
    everything behind it; a flipped T_min stop by T_min max|x|; the bound
    taken is (4 alpha_min + T_min) max|x| per channel).  The excused pixels
    are counted and must number at most `max_flipped` (default 1e-5 of the
    pixels compared on the binary32 geometry, 5e-3 on the FP64 geometry,
    whose threshold margins are 100x wider).  Returns (n_excused, report)."""
    P = ref["out"].shape[1]
    sel = np.ones(P, bool) if sel is None else np.asarray(sel, bool)
    n_sel = int(sel.sum())
    ma, mt = (MARGIN_A32, MARGIN_T32) if geometry == "fp32" else (MARGIN_A64, MARGIN_T64)
    if max_flipped is None:
        max_flipped = int((1e-5 if geometry == "fp32" else 5e-3) * n_sel)
    o = ref["out"]
    g = np.asarray(out_gpu, np.float64)
    C = o.shape[0]
    tol = np.full(C, TOL_RGB)
    for ch in [3] + list(range(5, C)):
        tol[ch] = TOL_REL_DF * max(float(np.max(np.abs(o[ch][sel]), initial=0.0)), 1e-30)
    dev = np.abs(g - o)
    bad_val = np.any(dev > tol[:, None], axis=0)
    bad_T = np.abs(np.asarray(T_gpu, np.float64) - ref["Tfinal"]) > TOL_RGB
    bad_last = np.asarray(last_gpu) != ref["last"]
    bad = sel & (bad_val | bad_T | bad_last)
    good = sel & ~bad
    rep = {"pixels": n_sel}
    rep["rgb"] = float(np.max(dev[0:3][:, good], initial=0.0))
    rep["opacity"] = float(np.max(dev[4][good], initial=0.0))
    for ch in [3] + list(range(5, C)):
        rep[f"ch{ch}"] = float(np.max(dev[ch][good], initial=0.0)) / (tol[ch] / TOL_REL_DF)
    n_bad = int(bad.sum())
    rep["excused"] = n_bad
    rep["_excused_mask"] = bad
    if n_bad:
        near = (ref["margin_a"] < ma) | (ref["margin_t"] < mt)
        assert np.all(near[bad]), ("pixel off tolerance with no decision near a threshold",
                                   np.nonzero(bad & ~near)[0][:10], rep)
        assert scales is not None, "excused pixels need the channel scales for the flipped-decision bound"
        amin = 1.0 / 255.0 if cfg is None else cfg.alpha_min
        tmin = 1e-4 if cfg is None else cfg.T_min
        bound = (4.0 * amin + tmin) * np.asarray(scales)[:, None]
        d = dev[:, bad]
        rep["excused_max_over_bound"] = float(np.max(d / bound))
        assert np.all(d <= bound), rep
        assert n_bad <= max_flipped, (n_bad, max_flipped, rep)
    return n_bad, rep


def rel_err(a, b):
    scale = max(float(np.max(np.abs(b))), 1e-30)
    return float(np.max(np.abs(np.asarray(a, np.float64) - b))) / scale


# ----------------------------------------------------------------------------
# seeded parity cases (scene, views)
# ----------------------------------------------------------------------------
def _multi_view_tiny(seed=61, n=300, F=16):
    w = wl.tiny_scene(seed, n, F=F, W=53, H=37, f=40.0)
    v2 = wl.make_view(29, 21, 25.0, wl.se3_exp(np.array([0.02, -0.01, 0.03, 0.01, 0.03, -0.02])))
    v3 = wl.make_view(64, 48, 50.0, wl.se3_exp(np.array([-0.05, 0.02, 0.0, -0.02, 0.01, 0.04])))
    return w.scene, w.views + [v2, v3]


def _stacked():
    """600 large Gaussians in a small region: every tile list spans several
    LDS batches and most pixels stop at T_min."""
    w = wl.tiny_scene(65, 600, F=16, W=48, H=40, f=40.0, log_scale_mu=-1.6, spread=0.15)
    return w.scene, w.views


def _stacked_long():
    """3000 large Gaussians over a 32x32 image: tile lists of thousands of
    instances, longer than the per-tile depth sort holds in LDS."""
    w = wl.tiny_scene(69, 3000, F=8, W=32, H=32, f=30.0, log_scale_mu=-1.6, spread=0.15)
    return w.scene, w.views


def _stacked_longest():
    """5000 large Gaussians over a 32x32 image: tile lists longer than the
    per-tile depth sort merges in LDS (global-memory counting passes)."""
    w = wl.tiny_scene(70, 5000, F=8, W=32, H=32, f=30.0, log_scale_mu=-1.6, spread=0.12)
    return w.scene, w.views


def _with_empty_view():
    """A batch whose second view faces away from every Gaussian."""
    w = wl.tiny_scene(66, 250, F=8, W=36, H=28, f=30.0)
    away = wl.make_view(32, 24, 30.0, wl.se3_exp(np.array([0.0, 0.0, 0.0, 0.0, np.pi, 0.0])))
    return w.scene, w.views + [away]


def _many_views(seed=67, n=300, F=8, V=40):
    """40 small views of mixed sizes and poses (some seeing little): more
    views than lanes of a wavefront's projection queue drains at once, view
    masks past bit 31 in the projection backward, and the record
    reduction's cross-lane sum over 64 lanes per Gaussian."""
    w = wl.tiny_scene(seed, n, F=F, W=24, H=20, f=25.0)
    rng = np.random.default_rng(seed)
    views = list(w.views)
    for _ in range(V - 1):
        xi = rng.normal(size=6) * np.array([0.05, 0.05, 0.05, 0.2, 0.2, 0.1])
        views.append(wl.make_view(int(rng.integers(12, 33)), int(rng.integers(10, 25)),
                                  float(rng.uniform(18.0, 35.0)), wl.se3_exp(xi)))
    return w.scene, views


CASES = {
    "tiny3views-F16": lambda: _multi_view_tiny(),
    "cfg1-64x64-2k": lambda: (wl.config1().scene, wl.config1().views),
    "cfg2-160x120-20k-F16": lambda: (lambda w: (w.scene, w.views))(wl.config2(n=20_000, width=160, height=120)),
    "tiny-F8": lambda: (lambda w: (w.scene, w.views))(wl.tiny_scene(62, 200, F=8, W=40, H=40, f=35.0)),
    "tiny-F32": lambda: (lambda w: (w.scene, w.views))(wl.tiny_scene(63, 200, F=32, W=40, H=24, f=35.0)),
    "tiny-F0": lambda: (lambda w: (w.scene, w.views))(wl.tiny_scene(64, 200, F=0, W=40, H=40, f=35.0)),
    "stacked600-F16": _stacked,
    "empty-view-F8": _with_empty_view,
    "40views-F8": _many_views,
    "64views-F8": lambda: _many_views(seed=68, V=64),  # the most views a batch may hold (mask bit 63)
    "stacked3000-F8": _stacked_long,
    "stacked5000-F8": _stacked_longest,
}


# ----------------------------------------------------------------------------
# a whole mapping / tracking step against the oracle
# ----------------------------------------------------------------------------
def _log(*a):
    import time
    print(f"[{time.strftime('%H:%M:%S')}]", *a, flush=True)


def step_snapshot(step):
    """Host copies of everything a step produces."""
    import torch
    torch.cuda.synchronize()
    r = step.r
    snap = {"out": r.out.cpu().numpy().copy(), "T": r.T_final.cpu().numpy().copy(),
            "last": r.last.cpu().numpy().copy(), "grad_out": r.grad_out.cpu().numpy().copy(),
            "loss": r.loss.cpu().numpy().copy(), "geo": r.grad_geo.cpu().numpy().copy(),
            "counts": r.instance_counts()}
    if step.grads is not None:
        snap["grads"] = {nm: t.cpu().numpy().copy() for nm, t in
                         zip(("mu", "log_scale", "quat", "logit", "color", "feat"), step.grads.tensors())}
        snap["app"] = r.grad_app.cpu().numpy().copy()
    if step.flags & 2:
        snap["twist"] = r.twist.cpu().numpy().copy()
    return snap


def assert_same_step(a, b, tol=1e-5):
    """Two runs of the same step on the same inputs: forward, loss and loss
    gradient bit for bit; the backward up to the last bits (the order in
    which a tile's wavefronts add into LDS is not fixed)."""
    assert a["counts"] == b["counts"]
    for k in ("out", "T", "last", "grad_out", "loss"):
        assert np.array_equal(a[k], b[k]), k
    assert rel_err(a["geo"], b["geo"].astype(np.float64)) <= tol
    if "grads" in a:
        for nm in a["grads"]:
            assert rel_err(a["grads"][nm], b["grads"][nm].astype(np.float64)) <= tol, nm
    if "twist" in a:
        for v in range(a["twist"].shape[0]):
            assert rel_err(a["twist"][v], b["twist"][v].astype(np.float64)) <= tol, v


def tie_free_targets(ref_out, seed):
    """Colour and depth targets a seeded margin away from the oracle's render
    (each value moved up or down by U[0.01, 0.1], depth by U[0.02, 0.2] m),
    so that no L1 residual sits within the binary32 render's rounding of
    zero, where the subgradient sign(render - target) of Eq. (15) / (17)
    could legitimately differ between binary32 and FP64."""
    rng = np.random.default_rng(seed)
    P = ref_out.shape[1]
    s = rng.choice([-1.0, 1.0], size=(4, P))
    rgb = ref_out[0:3] + s[0:3] * rng.uniform(0.01, 0.1, (3, P))
    dep = ref_out[3] + s[3] * rng.uniform(0.02, 0.2, P)
    return np.ascontiguousarray(rgb, np.float32), np.ascontiguousarray(dep, np.float32)


def gpu_backward_of(step):
    """The step's own backward entry points (same rasterizer buffers, same
    launch configuration) on a given upstream gradient [5+F][P]: returns the
    2D gradients, the parameter gradients and the twists it produces."""
    import torch

    def run(grad_out):
        r = step.r
        go = torch.from_numpy(np.ascontiguousarray(grad_out, np.float32)).cuda()
        grads = step.g.zeros_like() if step.grads is not None else None
        r.render_bwd(step.g, go, step.flags, grads, write=True)
        res = {"geo": r.grad_geo.cpu().numpy().copy()}
        if grads is not None:
            res["grads"] = {nm: t.cpu().numpy().copy() for nm, t in
                            zip(("mu", "log_scale", "quat", "logit", "color", "feat"), grads.tensors())}
        if step.flags & 2:
            r.pose_grad(step.g)
            res["twist"] = r.twist.cpu().numpy().copy()
        torch.cuda.synchronize()
        return res
    return run


def tiles_of_pixels(views, tile, pix):
    """Tile mask [T_total] of the tiles holding the given pixel indices."""
    T = sum(((v.width + tile - 1) // tile) * ((v.height + tile - 1) // tile) for v in views)
    mask = np.zeros(T, np.uint8)
    poff, toff = 0, 0
    for v in views:
        P = v.width * v.height
        tx = (v.width + tile - 1) // tile
        sel = pix[(pix >= poff) & (pix < poff + P)] - poff
        mask[toff + (sel // v.width // tile) * tx + (sel % v.width) // tile] = 1
        poff += P
        toff += tx * ((v.height + tile - 1) // tile)
    return mask


def step_oracle_parity(snap, r, scene, views, cfg, rgb_t, dep_t, lab, W, weights, flags, max_flipped=None,
                       bins=None, ref=None, gpu_backward=None):
    """The oracle, from the seeded inputs alone, against a step's snapshot on
    every pixel and every Gaussian: binning and order bit for bit; the render
    at the stated tolerances (compare_render); the loss value within 1e-4
    and its gradient (from the oracle's own render); the 2D gradients of
    every visible (view, Gaussian) pair, every parameter gradient of every
    Gaussian and every view's twist within 1e-3 of the tensor's max (the
    oracle's backward runs on the oracle's own loss gradient and takes its
    contributor decisions on the binary32 decision geometry, as the render
    comparison does; the contributions of the counted, excused pixels are
    taken out on both sides through `gpu_backward`, the step's own backward
    entry points, since the backward is linear in its upstream gradient)."""
    ocfg = oracle_cfg(cfg)
    V, n = len(views), scene.n
    # binning, bit for bit
    if bins is None:
        bins = oracle.bin_instances(scene, views, ocfg)
    dec = bins["dec"]
    touched = r.touched.view(V, n).cpu().numpy()
    assert np.array_equal(touched, dec["touched"])
    inst, nvis, over, gave_up = snap["counts"]
    assert not over and not gave_up and inst == bins["count"] and nvis == int((touched > 0).sum())
    assert np.array_equal(r.keys[:inst].cpu().numpy().view(np.uint32), bins["keys"])
    assert np.array_equal(r.sorted_gids(inst).cpu().numpy(), bins["gids"])
    assert np.array_equal(r.ranges.view(-1, 2).cpu().numpy(), bins["ranges"])
    _log("binning bit-exact:", inst, "instances,", nvis, "visible pairs")
    # forward, every pixel
    if ref is None:
        ref = oracle.render(scene, views, ocfg, bins=bins, geometry="fp32")
    excused, rep = compare_render(snap["out"], snap["T"], snap["last"], ref,
                                  scales=chan_scales(scene, float(ref["proj"][..., 6].max())), cfg=cfg,
                                  max_flipped=max_flipped)
    flipped = rep.pop("_excused_mask")
    _log("forward, every pixel:", rep)
    # the loss and its gradient on the oracle's own render (binary32 decision
    # geometry, FP64 values); compared on every pixel but the excused ones,
    # whose render legitimately differs
    Wd = W.astype(np.float64) if W is not None else None
    gout, terms = oracle.loss(ref["out"], views, rgb_t, dep_t, lab, Wd, weights)
    assert abs(float(snap["loss"][3]) - terms[3]) <= 1e-4 * abs(terms[3]), (snap["loss"], terms)
    keep = ~flipped
    go = snap["grad_out"][:, keep]
    gk = gout[:, keep]
    same_sign = np.sign(go[0:4]) == np.sign(gk[0:4])
    assert np.mean(same_sign) > 0.9999
    assert np.max(np.abs(go[0:4][same_sign] - gk[0:4][same_sign])) <= 1e-6 * np.max(np.abs(gk[0:4]))
    if go.shape[0] > 5:
        assert rel_err(go[5:], gk[5:]) <= 1e-3, rel_err(go[5:], gk[5:])
    _log("loss", float(snap["loss"][3]), "oracle", terms[3])
    # backward, every Gaussian.  The backward is linear in the upstream
    # gradient, so the contributions of the excused pixels (whose contributor
    # sets legitimately differ) are separated on both sides: the GPU's own
    # backward entry points on the excused pixels' upstream gradient alone,
    # the oracle's on the oracle's, and what remains -- the contributions of
    # every other pixel -- is held to the tolerance.
    b = oracle.backward(scene, views, ocfg, gout, bins=bins, flags=flags, decisions="fp32")
    gpu = {"geo": snap["geo"], "grads": snap.get("grads"), "twist": snap.get("twist")}
    orc = {"geo": b["grad2d"], "grads": {nm: b[nm] for nm in ("mu", "log_scale", "quat", "logit", "color", "feat")},
           "twist": b["twist"]}
    if excused:
        assert gpu_backward is not None, "excused pixels need the GPU backward to separate their contributions"
        pix = np.nonzero(flipped)[0]
        ge = np.zeros_like(snap["grad_out"])
        ge[:, pix] = snap["grad_out"][:, pix]
        GE = gpu_backward(ge)
        oe = np.zeros_like(gout)
        oe[:, pix] = gout[:, pix]
        OE = oracle.backward(scene, views, ocfg, oe, bins=bins, flags=flags, decisions="fp32",
                             tile_mask=tiles_of_pixels(views, cfg.tile, pix))
        gpu = {"geo": gpu["geo"].astype(np.float64) - GE["geo"],
               "grads": {nm: a.astype(np.float64) - GE["grads"][nm] for nm, a in gpu["grads"].items()}
               if gpu["grads"] is not None else None,
               "twist": gpu["twist"].astype(np.float64) - GE["twist"] if gpu["twist"] is not None else None}
        orc = {"geo": orc["geo"] - OE["grad2d"], "grads": {nm: a - OE[nm] for nm, a in orc["grads"].items()},
               "twist": orc["twist"] - OE["twist"]}
        _log(f"contributions of the {excused} excused pixels separated")
    errs = {}
    for k, nm in enumerate(["mx", "my", "A", "B", "C", "d"]):
        errs["2d_" + nm] = rel_err(gpu["geo"][..., k], orc["geo"][..., k])
    if flags & 1:
        for nm in ("mu", "log_scale", "quat", "logit", "color", "feat"):
            if nm == "feat" and scene.n_feat == 0:
                continue
            errs[nm] = rel_err(gpu["grads"][nm], orc["grads"][nm])
    if flags & 2:
        for v in range(V):
            errs[f"twist{v}"] = rel_err(gpu["twist"][v], orc["twist"][v])
    _log("gradients, every Gaussian:", {k: float(f"{e:.2e}") for k, e in errs.items()})
    bad = {k: e for k, e in errs.items() if e > TOL_GRAD}
    assert not bad, bad
    return errs
