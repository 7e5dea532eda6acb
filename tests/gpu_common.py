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
# A pixel whose alpha_min / T_min decisions lie within these relative
# margins of the threshold may legitimately decide differently in binary32
# and FP64; it is left out of the value comparison and counted.
#  - against the oracle on the binary32 projected geometry (mean, conic,
#    depth as the decision path computes them): only the kernel's binary32
#    alpha and transmittance arithmetic differs,
MARGIN_A32, MARGIN_T32 = 2e-5, 2e-4
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


def compare_render(out_gpu, T_gpu, last_gpu, ref, sel=None, geometry="fp32", scales=None, cfg=None):
    """Asserts the tolerances on the pixels of `sel` (default all) whose
    alpha_min / T_min decisions are unambiguous; returns (n_flagged, report).
    Flagged pixels (a decision within the margin of its threshold) may differ
    by flipped decisions only: one flipped alpha_min decision moves a channel
    by at most 2 alpha_min max|x| (its own weight and the (1 - alpha) it puts
    on everything behind it) and a flipped T_min stop by T_min max|x|; the
    flagged pixels are checked against 4 alpha_min + T_min times the
    channel's max |x| and must stay under 1% of the pixels compared (5%
    against the FP64 geometry, whose margins are 50x wider)."""
    P = ref["out"].shape[1]
    sel = np.ones(P, bool) if sel is None else sel
    ma, mt = (MARGIN_A32, MARGIN_T32) if geometry == "fp32" else (MARGIN_A64, MARGIN_T64)
    ok = sel & (ref["margin_a"] >= ma) & (ref["margin_t"] >= mt)
    flagged_mask = sel & ~ok
    flagged = int(flagged_mask.sum())
    o, g = ref["out"][:, ok], out_gpu[:, ok].astype(np.float64)
    rep = {}
    rep["rgb"] = float(np.max(np.abs(g[0:3] - o[0:3]))) if ok.any() else 0.0
    rep["opacity"] = float(np.max(np.abs(g[4] - o[4]))) if ok.any() else 0.0
    assert rep["rgb"] <= TOL_RGB, rep
    assert rep["opacity"] <= TOL_RGB, rep
    for ch in [3] + list(range(5, o.shape[0])):
        scale = max(np.max(np.abs(ref["out"][ch][sel])), 1e-30)
        err = float(np.max(np.abs(g[ch] - o[ch]))) if ok.any() else 0.0
        rep[f"ch{ch}"] = err / scale
        assert err <= TOL_REL_DF * scale, (ch, err, scale)
    assert np.max(np.abs(T_gpu[ok] - ref["Tfinal"][ok]), initial=0.0) <= TOL_RGB
    assert np.array_equal(last_gpu[ok], ref["last"][ok])
    if flagged:
        frac = 0.01 if geometry == "fp32" else 0.05
        assert flagged <= frac * max(int(sel.sum()), 1), flagged
        if scales is not None:
            amin = 1.0 / 255.0 if cfg is None else cfg.alpha_min
            tmin = 1e-4 if cfg is None else cfg.T_min
            bound = (4.0 * amin + tmin) * np.asarray(scales)[:, None]
            d = np.abs(out_gpu[:, flagged_mask].astype(np.float64) - ref["out"][:, flagged_mask])
            rep["flagged_max_over_bound"] = float(np.max(d / bound))
            assert np.all(d <= bound), rep
    return flagged, rep


def rel_err(a, b):
    scale = max(float(np.max(np.abs(b))), 1e-30)
    return float(np.max(np.abs(np.asarray(a, np.float64) - b))) / scale
