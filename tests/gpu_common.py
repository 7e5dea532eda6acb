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


def compare_render(out_gpu, T_gpu, last_gpu, ref, sel=None, geometry="fp32"):
    """Returns (n_flagged, report dict); asserts the tolerances on the
    unflagged pixels of `sel` (a boolean pixel mask, default all)."""
    P = ref["out"].shape[1]
    sel = np.ones(P, bool) if sel is None else sel
    ma, mt = (MARGIN_A32, MARGIN_T32) if geometry == "fp32" else (MARGIN_A64, MARGIN_T64)
    ok = sel & (ref["margin_a"] >= ma) & (ref["margin_t"] >= mt)
    flagged = int((sel & ~ok).sum())
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
    assert np.max(np.abs(T_gpu[ok] - ref["Tfinal"][ok])) <= TOL_RGB
    assert np.array_equal(last_gpu[ok], ref["last"][ok])
    return flagged, rep


def rel_err(a, b):
    scale = max(float(np.max(np.abs(b))), 1e-30)
    return float(np.max(np.abs(np.asarray(a, np.float64) - b))) / scale
