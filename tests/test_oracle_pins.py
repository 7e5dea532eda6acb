"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics (closed forms, invariants, brute force, finite differences).

Paper: GS^3LAM, Sec. 3.2 (Eq. 1-7), Sec. 3.3.1 (Eq. 10), Supp. B.1.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg
import torch

from paper_2603_27781_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _scene_from(gs, F=2):
    n = len(gs)
    mu = np.array([g["mu"] for g in gs], np.float32).T
    ls = np.array([[g.get("log_scale", -3.0)] * 3 for g in gs], np.float32).T
    quat = np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, n))
    logit = np.array([g.get("logit", 0.0) for g in gs], np.float32)
    color = np.array([g.get("color", [0.5, 0.5, 0.5]) for g in gs], np.float32).T
    feat = np.array([g.get("feat", [0.0] * F) for g in gs], np.float32).T
    return wl.Scene(*(np.ascontiguousarray(a) for a in (mu, ls, quat, logit, color, feat)))


def _cam(gold=None):
    gold = gold or json.load(open(os.path.join(GOLD, "closed_forms.json")))
    c = gold["camera"]
    return wl.View(c["width"], c["height"], c["fx"], c["fy"], c["cx"], c["cy"],
                   np.eye(4, dtype=np.float32)[:3].copy())


def _sig(x):
    return 1.0 / (1.0 + math.exp(-float(np.float32(x))))


# ----------------------------------------------------------------------------
# decision-path exponential and geometry (Eq. 2, 3)
# ----------------------------------------------------------------------------
def test_dec_exp_accuracy(orc):
    x = np.linspace(-20.0, 5.0, 20001).astype(np.float32)
    y = orc.dec_exp(x).astype(np.float64)
    ref = np.exp(x.astype(np.float64))
    assert np.max(np.abs(y / ref - 1.0)) < 4e-7


def test_quaternion_is_textbook_rotation(orc):
    cam = _cam()
    for th in (0.3, 1.1, -2.5):
        q = [math.cos(th / 2), 0.0, 0.0, math.sin(th / 2)]
        g = orc.geom([0, 0, 3], [-3, -3, -3], q, 0.0, cam, orc.Cfg())
        Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
        assert np.allclose(g["R"], Rz, atol=1e-14)
        # non-unit quaternion is normalised (Eq. 2 needs a rotation)
        g2 = orc.geom([0, 0, 3], [-3, -3, -3], [3 * v for v in q], 0.0, cam, orc.Cfg())
        assert np.allclose(g2["R"], Rz, atol=1e-14)


def test_covariance_eigenvalues_are_squared_scales(orc):
    cam = _cam()
    rng = np.random.default_rng(0)
    for _ in range(5):
        q = rng.normal(size=4)
        ls = rng.normal(-2, 0.5, size=3)
        g = orc.geom([0.1, 0.2, 3], ls, q, 0.0, cam, orc.Cfg())
        ev = np.sort(np.linalg.eigvalsh(g["Sigma"]))
        assert np.allclose(ev, np.sort(np.exp(2 * ls)), rtol=1e-12)
    g = orc.geom([0, 0, 3], [-2.0] * 3, [1, 0, 0, 0], 0.0, cam, orc.Cfg())
    assert np.allclose(g["Sigma"], math.exp(-4.0) * np.eye(3), atol=1e-16)


def test_on_axis_isotropic_sigma2d(orc):
    cam = _cam()
    cfg = orc.Cfg()
    b = float(np.float32(cfg.blur))
    for z, ls in ((2.0, -3.0), (3.5, -2.0)):
        g = orc.geom([0, 0, z], [ls] * 3, [0.3, 0.1, -0.7, 0.2], 0.0, cam, cfg)
        s = math.exp(ls)
        expect = (cam.fx * s / z) ** 2 + b
        assert g["Sigma2D"][0] == pytest.approx(expect, rel=1e-13)
        assert g["Sigma2D"][2] == pytest.approx(expect, rel=1e-13)
        assert abs(g["Sigma2D"][1]) < 1e-13


def test_projection_lands_on_pixel_centre(orc):
    """x = (u + 1/2 - cx) z / fx projects exactly onto the centre of pixel u."""
    cam = wl.View(40, 30, 50.0, 45.0, 20.0, 15.0, np.eye(4, dtype=np.float32)[:3].copy())
    z = 2.5
    us, vs = np.array([3, 17, 30]), np.array([2, 9, 21])
    xs = (us + 0.5 - 20.0) * z / 50.0
    ys = (vs + 0.5 - 15.0) * z / 45.0
    sc = _scene_from([{"mu": [x, y, z]} for x, y in zip(xs, ys)])
    proj = orc.project64(sc, [cam], orc.Cfg(), s64={k: np.ascontiguousarray(v, np.float64) for k, v in
                                                     {"mu": np.array([xs, ys, [z] * 3]), "log_scale": sc.log_scale,
                                                      "quat": sc.quat, "logit": sc.logit, "color": sc.color,
                                                      "feat": sc.feat}.items()})
    assert np.allclose(proj[0, :, 0], us + 0.5, atol=1e-12)
    assert np.allclose(proj[0, :, 1], vs + 0.5, atol=1e-12)


def test_jacobian_matches_finite_difference_of_projection(orc):
    """The EWA Jacobian J = d pi / d p (Eq. 3), checked through Sigma2D of an
    isotropic Gaussian of tiny scale: Sigma2D - bI = s^2 J J^T."""
    cam = wl.View(64, 64, 60.0, 55.0, 31.0, 29.0, np.eye(4, dtype=np.float32)[:3].copy())
    cfg = orc.Cfg()
    p = np.array([0.4, -0.3, 2.7])
    s = 1e-3
    g = orc.geom(p, [math.log(s)] * 3, [1, 0, 0, 0], 0.0, cam, cfg)

    def pi(pp):
        return np.array([cam.fx * pp[0] / pp[2] + cam.cx, cam.fy * pp[1] / pp[2] + cam.cy])

    J = np.zeros((2, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1e-6
        J[:, k] = (pi(p + e) - pi(p - e)) / 2e-6
    S = s * s * J @ J.T
    b = float(np.float32(cfg.blur))
    got = np.array([[g["Sigma2D"][0] - b, g["Sigma2D"][1]], [g["Sigma2D"][1], g["Sigma2D"][2] - b]])
    assert np.allclose(got, S, rtol=1e-6, atol=1e-14)


def test_dec_log_accuracy(orc):
    """The decision path's binary32 logarithm against the FP64 library log:
    within 2 ulp of the result everywhere, exact at 1."""
    rng = np.random.default_rng(5)
    x = np.concatenate([1.0 + rng.uniform(0, 1e-3, 4000), rng.uniform(1.0, 300.0, 40000),
                        np.exp(rng.uniform(-80, 80, 40000)), [1.0, 2.0, 255.0, 0.5, 1e-30, 1e30]]).astype(np.float32)
    y = orc.dec_log(x).astype(np.float64)
    ref = np.log(x.astype(np.float64))
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(y - ref) <= 2.0 * ulp), float(np.max(np.abs(y - ref) / ulp))
    assert y[x == 1.0].tolist() == [0.0] * int(np.sum(x == 1.0))


def test_box_k_is_twice_log_opacity_over_alpha_min(orc):
    """The opacity-aware box: its squared radius is 2 ln(o / alpha_min)
    (+ 2^-8), from the opacity o = sigmoid(logit); 0 (culled) where
    o <= alpha_min."""
    rng = np.random.default_rng(6)
    amin = float(np.float32(1.0 / 255.0))
    lmin = math.log(amin / (1 - amin))
    logit = np.concatenate([rng.normal(0, 3, 20000), lmin + rng.normal(0, 1e-3, 2000), [60.0, -60.0, 0.0]])
    logit = logit.astype(np.float32)
    k = orc.box_k(logit).astype(np.float64)
    o = 1.0 / (1.0 + np.exp(-logit.astype(np.float64)))
    ref = 2.0 * np.log(o / amin) + 2.0 ** -8
    clear_in = o > amin * (1 + 1e-5)
    clear_out = o < amin * (1 - 1e-5)
    assert np.all(np.abs(k[clear_in] - ref[clear_in]) <= 1e-6 * np.maximum(1.0, ref[clear_in]))
    assert np.all(k[clear_out] == 0.0)
    # an opaque Gaussian's box: 2 ln(1/alpha_min) = 2 ln 255
    assert k[-3] == pytest.approx(2 * math.log(255.0) + 2.0 ** -8, rel=1e-6)


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_tile_rectangle_edges_follow_the_opacity_aware_box(orc, tile):
    """Both edges of every visible pair's tile rectangle are where the
    opacity-aware box puts them, from FP64 quantities: the box [m - r, m + r]
    with r = sqrt(k Sigma2D_xx) (1 + 2^-10), k = 2 ln(o / alpha_min)
    (+ 2^-8), mean, Sigma2D and o from the FP64 projection, touches tiles
    floor((m - r)/tile) .. floor((m + r)/tile), clamped to the grid.  The FP64 box is bracketed (r without the padding,
    less 1e-3 px, and with it, plus 1e-3 px) to absorb binary32 rounding; a
    rectangle even one tile too wide or too narrow on either side fails."""
    w = wl.config1(scale=0.5)
    views = w.views + [wl.make_view(53, 37, 40.0, wl.se3_exp(np.array([0.1, -0.05, 0.2, 0.05, 0.1, -0.03])))]
    cfg = orc.Cfg(tile=tile)
    dec = orc.decide(w.scene, views, cfg)
    proj = orc.project64(w.scene, views, cfg)
    amin = float(np.float32(cfg.alpha_min))
    checked = 0
    for vi, v in enumerate(views):
        vis = dec["touched"][vi] > 0
        mx, my, A, B, C, o = (proj[vi][vis][:, k] for k in range(6))
        det = A * C - B * B
        sxx, syy = C / det, A / det
        kk = 2.0 * np.log(o / amin)
        ntx, nty = (v.width + tile - 1) // tile, (v.height + tile - 1) // tile
        rect = dec["rect"][vi][vis]
        for m, sig, lim, lo_col, hi_col in ((mx, sxx, ntx, 0, 2), (my, syy, nty, 1, 3)):
            r_lo = np.sqrt(kk * sig) - 1e-3
            r_hi = np.sqrt((kk + 2.0 ** -8) * sig) * (1 + 2.0 ** -10) + 1e-3
            cl = lambda t: np.clip(t, 0, lim - 1)
            lo0, lo1 = cl(np.floor((m - r_hi) / tile)), cl(np.floor((m - r_lo) / tile))
            hi0, hi1 = cl(np.floor((m + r_lo) / tile)), cl(np.floor((m + r_hi) / tile))
            assert np.all((rect[:, lo_col] >= lo0) & (rect[:, lo_col] <= lo1))
            assert np.all((rect[:, hi_col] >= hi0) & (rect[:, hi_col] <= hi1))
            # the bracket is narrow: it leaves a choice for few pairs
            assert np.mean(lo0 != lo1) < 0.01 and np.mean(hi0 != hi1) < 0.01
        checked += int(vis.sum())
        # opacity cull: o <= alpha_min is never visible
        o_all = 1.0 / (1.0 + np.exp(-w.scene.logit.astype(np.float64)))
        assert not np.any(dec["touched"][vi][o_all <= amin])
    assert checked > 500


def test_culls_follow_the_near_plane_guard_and_opacity_rules(orc):
    """Which pairs survive the culls, against the rules evaluated in FP64:
    camera depth > z_near; |x/z| <= guard (W/2)/fx and |y/z| <= guard
    (H/2)/fy; opacity o > alpha_min.  Each Gaussian sits a relative 1e-4
    (1e-3 in the logit) inside or outside one boundary; the scales are large
    (0.5 m), so every Gaussian reaches the image and only a cull can drop
    it."""
    W, H, f = 64, 48, 40.0
    view = wl.make_view(W, H, f, np.eye(4))
    cfg = orc.Cfg()
    limx, limy = cfg.guard * (W / 2) / f, cfg.guard * (H / 2) / f
    amin = float(np.float32(cfg.alpha_min))
    lmin = math.log(amin / (1.0 - amin))
    eps = 1e-4
    pts, logit = [], []
    for z in (cfg.z_near * (1 + eps), cfg.z_near * (1 - eps), 0.5, 3.0):
        pts.append((0.0, 0.0, z))
        logit.append(0.0)
    for sgn in (1.0, -1.0):
        for fac in (1 - eps, 1 + eps):
            pts.append((sgn * limx * fac * 3.0, 0.0, 3.0))
            pts.append((0.0, sgn * limy * fac * 3.0, 3.0))
            logit += [0.0, 0.0]
    for dl in (1e-3, -1e-3, 0.5, -0.5):
        pts.append((0.1, -0.1, 2.0))
        logit.append(lmin + dl)
    n = len(pts)
    mu = np.array(pts, np.float64).T
    logit = np.array(logit, np.float64)
    sc = wl.Scene(mu.astype(np.float32), np.full((3, n), math.log(0.5), np.float32),
                  np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, n)),
                  logit.astype(np.float32), np.full((3, n), 0.5, np.float32), np.zeros((2, n), np.float32))
    # the rules, in FP64, on the binary32 inputs
    m = sc.mu.astype(np.float64)
    z = m[2]
    o = 1.0 / (1.0 + np.exp(-sc.logit.astype(np.float64)))
    with np.errstate(divide="ignore", invalid="ignore"):
        expect = (z > cfg.z_near) & (np.abs(m[0] / z) <= limx) & (np.abs(m[1] / z) <= limy) & (o > amin)
    dec = orc.decide(sc, [view], cfg)
    got = dec["touched"][0] > 0
    assert expect.sum() >= 8 and (~expect).sum() >= 7
    assert np.array_equal(got, expect), (np.nonzero(got != expect)[0], got, expect)


def test_decision_path_agrees_with_fp64(orc):
    w = wl.config1(scale=0.25)
    cfg = orc.Cfg()
    dec = orc.decide(w.scene, w.views, cfg)
    proj = orc.project64(w.scene, w.views, cfg)
    vis = dec["touched"][0] > 0
    r32, p64 = dec["rec32"][0][vis], proj[0][vis]
    assert np.allclose(r32[:, 0:2], p64[:, 0:2], rtol=0, atol=2e-4)
    for k in (2, 3, 4):
        assert np.max(np.abs(r32[:, k] - p64[:, k])) <= 2e-5 * np.max(np.abs(p64[:, k]))
    assert np.allclose(r32[:, 5], p64[:, 6], rtol=1e-6)
    # depth key is the binary32 depth
    assert np.array_equal(dec["dbits"][0][vis], r32[:, 5].view(np.uint32))


# ----------------------------------------------------------------------------
# closed forms of the compositing (Eq. 4-7, 9), from tests/golden
# ----------------------------------------------------------------------------
def test_closed_form_single_gaussian(orc):
    gold = json.load(open(os.path.join(GOLD, "closed_forms.json")))
    case = gold["cases"][0]
    g = case["gaussians"][0]
    sc = _scene_from([g])
    cam = _cam(gold)
    r = orc.render(sc, [cam], orc.Cfg())
    u, v = case["pixel"]
    p = v * cam.width + u
    o = _sig(g["logit"])
    c = np.float32(g["color"]).astype(np.float64)
    f = np.float32(g["feat"]).astype(np.float64)
    assert np.allclose(r["out"][0:3, p], c * o, rtol=1e-14)
    assert r["out"][3, p] == pytest.approx(3.0 * o, rel=1e-14)
    assert r["out"][4, p] == pytest.approx(o, rel=1e-14)
    assert np.allclose(r["out"][5:, p], f * o, rtol=1e-14)
    assert r["Tfinal"][p] == pytest.approx(1.0 - o, rel=1e-14)
    # one pixel to the right: alpha = o exp(-conic_xx / 2), conic_xx = 1/((fx s/z)^2 + b)
    s = math.exp(float(np.float32(g["log_scale"])))
    b = float(np.float32(0.3))
    conic_xx = 1.0 / ((cam.fx * s / 3.0) ** 2 + b)
    a1 = o * math.exp(-0.5 * conic_xx)
    assert r["out"][4, p + 1] == pytest.approx(a1, rel=1e-12)


def test_closed_form_two_stacked(orc):
    gold = json.load(open(os.path.join(GOLD, "closed_forms.json")))
    case = gold["cases"][1]
    far, near = case["gaussians"]
    sc = _scene_from(case["gaussians"])
    cam = _cam(gold)
    r = orc.render(sc, [cam], orc.Cfg())
    u, v = case["pixel"]
    p = v * cam.width + u
    o1, o2 = _sig(near["logit"]), _sig(far["logit"])
    c1, c2 = (np.float32(near["color"]).astype(np.float64), np.float32(far["color"]).astype(np.float64))
    assert np.allclose(r["out"][0:3, p], c1 * o1 + c2 * o2 * (1 - o1), rtol=1e-13)
    d_expect = 2.0 * o1 + 3.0 * o2 * (1 - o1)
    assert r["out"][3, p] == pytest.approx(d_expect, rel=1e-13)


def test_closed_form_thirteen_contributors(orc):
    gold = json.load(open(os.path.join(GOLD, "closed_forms.json")))
    case = gold["cases"][2]
    n = case["n"]
    sc = _scene_from([{"mu": [0.0, 0.0, 3.0], "logit": 0.0} for _ in range(n)])
    cam = _cam(gold)
    r = orc.render(sc, [cam], orc.Cfg())
    u, v = case["pixel"]
    p = v * cam.width + u
    assert r["ncontrib"][p] == case["expect"]["contributors"]
    assert r["out"][4, p] == case["expect"]["opacity"]
    assert r["Tfinal"][p] == 2.0 ** -13


def test_equal_depth_composites_in_index_order(orc):
    sc = _scene_from([{"mu": [0.0, 0.0, 3.0], "logit": 0.2, "color": [1, 0, 0]},
                      {"mu": [0.0, 0.0, 3.0], "logit": 0.2, "color": [0, 1, 0]}])
    cam = _cam()
    r = orc.render(sc, [cam], orc.Cfg())
    p = 32 * 64 + 32
    o = _sig(0.2)
    assert r["out"][0, p] == pytest.approx(o, rel=1e-14)
    assert r["out"][1, p] == pytest.approx(o * (1 - o), rel=1e-14)


# ----------------------------------------------------------------------------
# invariants
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [3, 4])
def test_opacity_plus_transmittance_is_one(orc, seed):
    w = wl.tiny_scene(seed, 60, F=4)
    r = orc.render(w.scene, w.views, orc.Cfg(tile=8))
    assert np.max(np.abs(r["out"][4] + r["Tfinal"] - 1.0)) < 1e-14


def test_tile_size_does_not_change_the_render(orc):
    w = wl.config1(scale=0.5)
    outs = [orc.render(w.scene, w.views, orc.Cfg(tile=t))["out"] for t in (8, 16, 32)]
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])


def test_linear_in_colour_and_feature(orc):
    w = wl.tiny_scene(5, 50, F=3)
    cfg = orc.Cfg(tile=8)
    a, b = w.scene.copy(), w.scene.copy()
    rng = np.random.default_rng(1)
    b.color = rng.uniform(0, 1, size=a.color.shape).astype(np.float32)
    b.feat = rng.normal(size=a.feat.shape).astype(np.float32)
    s = w.scene.copy()
    s.color = (a.color.astype(np.float64) + b.color).astype(np.float32)
    s.feat = (a.feat.astype(np.float64) + b.feat).astype(np.float32)
    ra, rb, rs = (orc.render(x, w.views, cfg)["out"] for x in (a, b, s))
    chans = [0, 1, 2] + list(range(5, 5 + 3))
    assert np.allclose(rs[chans], ra[chans] + rb[chans], atol=1e-12)


def test_bins_cover_every_contributing_pair(orc):
    """The tile rectangle only prunes: every pixel a Gaussian reaches with
    alpha >= alpha_min lies in a tile whose list holds that Gaussian."""
    w = wl.tiny_scene(11, 80, F=2, W=40, H=32)
    cfg = orc.Cfg(tile=8)
    bins = orc.bin_instances(w.scene, w.views, cfg)
    proj = orc.project64(w.scene, w.views, cfg)[0]
    vis = bins["dec"]["touched"][0] > 0
    v = w.views[0]
    tx = (v.width + 7) // 8
    lists = {t: set(bins["gids"][bins["ranges"][t, 0]:bins["ranges"][t, 1]].tolist())
             for t in range(bins["ranges"].shape[0])}
    amin = float(np.float32(cfg.alpha_min))
    uu, vv = np.meshgrid(np.arange(v.width) + 0.5, np.arange(v.height) + 0.5)
    for i in np.nonzero(vis)[0]:
        mx, my, A, B, C, o, d = proj[i]
        dx, dy = uu - mx, vv - my
        al = o * np.exp(-0.5 * np.maximum(A * dx * dx + 2 * B * dx * dy + C * dy * dy, 0))
        ys, xs = np.nonzero(al >= amin * 0.999)
        for x, y in zip(xs, ys):
            assert i in lists[(y // 8) * tx + x // 8]


def test_binning_matches_enumeration(orc):
    w = wl.tiny_scene(12, 70, F=2, W=40, H=32)
    views = w.views + [wl.make_view(24, 16, 20.0, np.eye(4))]
    cfg = orc.Cfg(tile=8)
    bins = orc.bin_instances(w.scene, views, cfg)
    dec = bins["dec"]
    items = []
    base = 0
    for vi, v in enumerate(views):
        tx, ty = (v.width + 7) // 8, (v.height + 7) // 8
        for i in range(w.scene.n):
            r = dec["rect"][vi, i]
            if dec["touched"][vi, i] == 0:
                continue
            for y in range(r[1], r[3] + 1):
                for x in range(r[0], r[2] + 1):
                    items.append((base + y * tx + x, int(dec["dbits"][vi, i]), i))
        base += tx * ty
    items.sort()
    assert bins["count"] == len(items)
    assert np.array_equal(bins["keys"], np.array([t for t, _, _ in items], np.uint32))
    assert np.array_equal(bins["gids"], np.array([g for _, _, g in items], np.int32))
    for t in range(base):
        sel = [k for k, it in enumerate(items) if it[0] == t]
        lo, hi = bins["ranges"][t]
        if sel:
            assert (lo, hi) == (sel[0], sel[-1] + 1)
        else:
            assert lo == hi


# ----------------------------------------------------------------------------
# brute force (independent PyTorch renderer, autograd gradients)
# ----------------------------------------------------------------------------
NAMES = ["mu", "log_scale", "quat", "logit", "color", "feat"]


@pytest.mark.parametrize("seed,n,F", [(21, 30, 4), (22, 64, 8)])
def test_oracle_matches_bruteforce_forward_and_gradients(orc, seed, n, F):
    from oracle import bruteforce as bf
    w = wl.tiny_scene(seed, n, F=F)
    cfg = orc.Cfg(tile=8)
    r = orc.render(w.scene, w.views, cfg)
    g = np.random.default_rng(seed).normal(size=r["out"].shape)
    b = orc.backward(w.scene, w.views, cfg, g, bins=r["bins"])
    ts = bf.as_tensors(w.scene, True)
    xi = torch.zeros(6, dtype=torch.float64, requires_grad=True)
    out, T = bf.render(*ts, w.views[0], xi=xi)
    assert np.max(np.abs(out.detach().numpy() - r["out"])) < 1e-12
    assert np.max(np.abs(T.detach().numpy() - r["Tfinal"])) < 1e-12
    (out * torch.tensor(g)).sum().backward()
    for nm, t in zip(NAMES, ts):
        e = t.grad.numpy()
        assert np.max(np.abs(b[nm] - e)) <= 1e-10 * max(1.0, np.max(np.abs(e))), nm
    assert np.max(np.abs(b["twist"][0] - xi.grad.numpy())) <= 1e-10 * np.max(np.abs(xi.grad.numpy()))


def test_oracle_matches_bruteforce_config1(orc):
    """64x64, 2,000 Gaussians (the small workload) against brute force."""
    from oracle import bruteforce as bf
    w = wl.config1()
    cfg = orc.Cfg(tile=16)
    r = orc.render(w.scene, w.views, cfg)
    ts = bf.as_tensors(w.scene, False)
    out, T = bf.render(*ts, w.views[0])
    assert np.max(np.abs(out.numpy() - r["out"])) < 1e-11


# ----------------------------------------------------------------------------
# central finite differences in FP64 (decision-set guarded)
# ----------------------------------------------------------------------------
def _lin_loss(orc, w, cfg, bins, g, s64=None, poses64=None):
    r = orc.render(w.scene, w.views, cfg, bins=bins, s64=s64, poses64=poses64)
    return float(np.sum(g * r["out"])), (r["last"].copy(), r["ncontrib"].copy())


def test_oracle_gradients_match_central_differences(orc):
    w = wl.tiny_scene(31, 40, F=3)
    cfg = orc.Cfg(tile=8)
    bins = orc.bin_instances(w.scene, w.views, cfg)
    base = orc.render(w.scene, w.views, cfg, bins=bins)
    g = np.random.default_rng(3).normal(size=base["out"].shape)
    b = orc.backward(w.scene, w.views, cfg, g, bins=bins)
    s0 = orc.scene64(w.scene)
    key0 = (base["last"], base["ncontrib"])
    rng = np.random.default_rng(4)
    vis = np.nonzero(bins["dec"]["touched"][0] > 0)[0]
    checked = 0
    for nm in NAMES:
        for _ in range(4):
            i = int(rng.choice(vis))
            k = int(rng.integers(0, s0[nm].shape[0])) if s0[nm].ndim == 2 else None
            idx = (k, i) if k is not None else (i,)
            x = s0[nm][idx]
            h = 1e-6 * max(1.0, abs(x))
            ok = False
            while h > 1e-9:
                sp = {kk: vv.copy() for kk, vv in s0.items()}
                sm = {kk: vv.copy() for kk, vv in s0.items()}
                sp[nm][idx] = x + h
                sm[nm][idx] = x - h
                lp, kp = _lin_loss(orc, w, cfg, bins, g, s64=sp)
                lm, km = _lin_loss(orc, w, cfg, bins, g, s64=sm)
                if all(np.array_equal(a, c) for a, c in zip(kp, key0)) and \
                        all(np.array_equal(a, c) for a, c in zip(km, key0)):
                    ok = True
                    break
                h *= 0.5
            if not ok:
                continue
            fd = (lp - lm) / (2 * h)
            an = b[nm][idx]
            assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (nm, idx, fd, an)
            checked += 1
    assert checked >= 18


def test_twist_gradient_matches_central_differences(orc):
    """Left perturbation T(xi) = Exp(xi) T_CW (Supp. B.1 written as a twist),
    Exp by the matrix exponential of the 4x4 twist matrix."""
    w = wl.tiny_scene(41, 40, F=3)
    cfg = orc.Cfg(tile=8)
    bins = orc.bin_instances(w.scene, w.views, cfg)
    base = orc.render(w.scene, w.views, cfg, bins=bins)
    g = np.random.default_rng(5).normal(size=base["out"].shape)
    b = orc.backward(w.scene, w.views, cfg, g, bins=bins)
    T0 = np.eye(4)
    T0[:3] = np.asarray(w.views[0].Rt, np.float32).astype(np.float64)

    def twist_mat(xi):
        M = np.zeros((4, 4))
        M[:3, :3] = np.array([[0, -xi[5], xi[4]], [xi[5], 0, -xi[3]], [-xi[4], xi[3], 0]])
        M[:3, 3] = xi[:3]
        return M

    h = 1e-6
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        Tp = scipy.linalg.expm(twist_mat(e)) @ T0
        Tm = scipy.linalg.expm(twist_mat(-e)) @ T0
        lp, kp = _lin_loss(orc, w, cfg, bins, g, poses64=[Tp])
        lm, km = _lin_loss(orc, w, cfg, bins, g, poses64=[Tm])
        assert np.array_equal(kp[0], base["last"]) and np.array_equal(km[0], base["last"])
        fd = (lp - lm) / (2 * h)
        assert abs(fd - b["twist"][0, k]) <= 1e-5 * max(1.0, np.max(np.abs(b["twist"][0]))), k


def test_twist_translation_equals_rotated_mean_gradient(orc):
    """dL/drho = R_CW^-T sum_i dL/dmu_i (= R_CW sum_i dL/dmu_i for an exactly
    orthogonal R_CW; the binary32 pose is orthogonal only to ~1e-8): translating
    the camera by rho moves every camera-space mean by rho, as does moving every
    mean by R_CW^-1 rho."""
    w = wl.tiny_scene(51, 60, F=3)
    cfg = orc.Cfg(tile=8)
    r = orc.render(w.scene, w.views, cfg)
    g = np.random.default_rng(6).normal(size=r["out"].shape)
    b = orc.backward(w.scene, w.views, cfg, g, bins=r["bins"])
    R = np.asarray(w.views[0].Rt, np.float32).astype(np.float64)[:, :3]
    assert np.allclose(b["twist"][0, :3], np.linalg.solve(R.T, b["mu"].sum(axis=1)), rtol=1e-10, atol=1e-10)


# ----------------------------------------------------------------------------
# image-space losses (Sec. 3.3.4, 3.4)
# ----------------------------------------------------------------------------
def test_loss_gradient_matches_torch_cross_entropy(orc):
    rng = np.random.default_rng(7)
    F, K = 6, 9
    views = [wl.make_view(5, 4, 10.0, np.eye(4)), wl.make_view(3, 3, 10.0, np.eye(4))]
    P = 29
    out = rng.normal(size=(5 + F, P))
    rgb = rng.uniform(size=(3, P))
    dep = rng.uniform(1, 3, size=P)
    lab = rng.integers(0, K, size=P).astype(np.int32)
    Wd = rng.normal(size=(F, K))
    wts = (0.5, 1.0, 0.01)
    g, terms = orc.loss(out, views, rgb, dep, lab, Wd, wts)
    # torch reference per view (library cross entropy, mean reduction)
    o = torch.tensor(out, requires_grad=True)
    tot = 0.0
    base = 0
    for v in views:
        Pv = v.width * v.height
        sl = slice(base, base + Pv)
        tot = tot + wts[0] * (o[0:3, sl] - torch.tensor(rgb[:, sl])).abs().mean()
        tot = tot + wts[1] * (o[3, sl] - torch.tensor(dep[sl])).abs().mean()
        logits = o[5:, sl].T @ torch.tensor(Wd)
        tot = tot + wts[2] * torch.nn.functional.cross_entropy(logits, torch.tensor(lab[sl]).long())
        base += Pv
    tot.backward()
    assert terms[3] == pytest.approx(float(tot), rel=1e-12)
    assert np.max(np.abs(g - o.grad.numpy())) < 1e-15
    assert np.all(g[4] == 0)


def test_backward_decision_geometry_changes_only_decisions(orc):
    """Taking the alpha_min / T_min decisions on the binary32 decision
    geometry leaves every value on the FP64 projection: where both
    geometries give every pixel the same contributors and stop (the 64x64,
    2,000-Gaussian workload), the gradients are the same bits."""
    w = wl.config1()
    cfg = orc.Cfg(tile=16)
    bins = orc.bin_instances(w.scene, w.views, cfg)
    r64 = orc.render(w.scene, w.views, cfg, bins=bins)
    r32 = orc.render(w.scene, w.views, cfg, bins=bins, geometry="fp32")
    assert np.array_equal(r64["ncontrib"], r32["ncontrib"]) and np.array_equal(r64["last"], r32["last"])
    go = np.random.default_rng(3).normal(size=r64["out"].shape) * 1e-2
    a = orc.backward(w.scene, w.views, cfg, go, bins=bins)
    b = orc.backward(w.scene, w.views, cfg, go, bins=bins, decisions="fp32")
    for k in ("grad2d", "mu", "log_scale", "quat", "logit", "color", "feat", "twist"):
        assert np.array_equal(a[k], b[k]), k
