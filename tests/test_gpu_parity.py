"""GPU parity: every C-ABI entry point against the FP64 CPU oracle on the
same seeded inputs.  Bit-exact for the integer work (culling, tile
rectangles, instance lists, sorted order, ranges); stated tolerances for
floating point."""
import numpy as np
import pytest

import oracle
from paper_2603_27781_amd import workloads as wl
from gpu_common import (CASES, MARGIN, TOL_GRAD, chan_scales, compare_render, gpu_setup, oracle_cfg, rel_err)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _project(name, tile):
    scene, views = CASES[name]()
    r, g, cfg = gpu_setup(scene, views, {"tile": tile})
    r.project(g)
    torch.cuda.synchronize()
    dec = oracle.decide(scene, views, oracle_cfg(cfg))
    return scene, views, r, g, cfg, dec


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("tile", [8, 16])
def test_project_bit_exact(name, tile):
    scene, views, r, g, cfg, dec = _project(name, tile)
    V, n = len(views), scene.n
    rec = r.rec.view(V, n, 8).cpu().numpy()
    touched = r.touched.view(V, n).cpu().numpy()
    rect = r.rect.view(V, n, 4).cpu().numpy().view(np.uint32)
    assert np.array_equal(touched, dec["touched"])
    vis = touched > 0
    assert vis.sum() > 0
    r32 = dec["rec32"]
    # mean, conic, depth: the binary32 decision path, bit for bit
    for k_gpu, k_orc in ((0, 0), (1, 1), (2, 2), (3, 3), (4, 4), (6, 5)):
        assert np.array_equal(rec[..., k_gpu][vis].view(np.uint32), r32[..., k_orc][vis].view(np.uint32)), k_gpu
    # rectangles
    ro = dec["rect"]
    x0 = (rect[..., 0] & 0xFFFF).astype(np.int32)
    y0 = (rect[..., 0] >> 16).astype(np.int32)
    x1 = (rect[..., 1] & 0xFFFF).astype(np.int32)
    y1 = (rect[..., 1] >> 16).astype(np.int32)
    for a, k in ((x0, 0), (y0, 1), (x1, 2), (y1, 3)):
        assert np.array_equal(a[vis], ro[..., k][vis])
    # opacity (value path) and the conservative binary16 radii
    proj = oracle.project64(scene, views, oracle_cfg(cfg))
    assert np.max(np.abs(rec[..., 5][vis] - proj[..., 5][vis])) < 1e-6
    bits = rec[..., 7].view(np.uint32)
    rx = (bits & 0xFFFF).astype(np.uint16).view(np.float16).astype(np.float32)
    ry = (bits >> 16).astype(np.uint16).view(np.float16).astype(np.float32)
    assert np.all(rx[vis] >= r32[..., 6][vis]) and np.all(ry[vis] >= r32[..., 7][vis])


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_bin_sort_bit_exact(name, tile):
    scene, views, r, g, cfg, dec = _project(name, tile)
    r.bin_sort()
    inst, nvis, over, gave_up = r.instance_counts()
    ref = oracle.bin_instances(scene, views, oracle_cfg(cfg), dec=dec)
    assert not over and not gave_up
    assert inst == ref["count"]
    assert nvis == int((dec["touched"] > 0).sum())
    assert np.array_equal(r.keys[:inst].cpu().numpy().view(np.uint32), ref["keys"])
    assert np.array_equal(r.sorted_gids(inst).cpu().numpy(), ref["gids"])
    # emission layout: each visible pair's instances are contiguous from pair_first
    touched = r.touched.cpu().numpy()
    first = r.pair_first.cpu().numpy()
    inst_gid = r.inst_gid[:inst].cpu().numpy()
    n = scene.n
    vis = np.nonzero(touched > 0)[0]
    for pair in vis[:: max(1, len(vis) // 200)]:
        e0 = first[pair]
        assert np.all(inst_gid[e0:e0 + touched[pair]] == pair % n)
    assert np.array_equal(np.sort(r.inst[:inst].cpu().numpy()), np.arange(inst))
    assert np.array_equal(r.ranges.view(-1, 2).cpu().numpy(), ref["ranges"])


def test_bin_sort_capacity_overflow_is_reported():
    scene, views = CASES["cfg1-64x64-2k"]()
    r, g, cfg = gpu_setup(scene, views, {"tile": 16}, capacity=1000)
    r.project(g)
    r.bin_sort()
    inst, _, over, _ = r.instance_counts()
    assert over and inst > 1000
    assert r.ensure_capacity(g) == inst
    r.bin_sort()
    assert r.instance_counts()[2] is False


def _render(name, tile, lds_batch=256, persistent=0, lds_batch_bwd=0):
    scene, views = CASES[name]()
    r, g, cfg = gpu_setup(scene, views, {"tile": tile, "lds_batch": lds_batch, "persistent": persistent,
                                         "lds_batch_bwd": lds_batch_bwd})
    r.ensure_capacity(g)
    r.forward(g)
    torch.cuda.synchronize()
    return scene, views, r, g, cfg


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("tile,lds_batch,persistent", [(16, 256, 0), (8, 64, 0), (32, 128, 1)])
def test_render_fwd_parity(name, tile, lds_batch, persistent):
    """Against the oracle on the binary32 projected geometry, every pixel:
    RGB, opacity, T within 1e-5, depth and features within 1e-4 of the
    channel max, the last contributor equal.  A pixel off tolerance is
    excused only as a flipped threshold decision (a decision within 1e-5
    (alpha) / 1e-4 (T) of its threshold, the deviation within the flip
    bound), at most 1e-5 P of them: none at these sizes."""
    scene, views, r, g, cfg = _render(name, tile, lds_batch, persistent)
    ref = oracle.render(scene, views, oracle_cfg(cfg), geometry="fp32")
    excused, rep = compare_render(r.out.cpu().numpy(), r.T_final.cpu().numpy(), r.last.cpu().numpy(), ref,
                                  scales=chan_scales(scene, float(ref["proj"][..., 6].max())), cfg=cfg)
    rep.pop("_excused_mask")
    print(name, tile, "excused", excused, rep)


# stacked3000, stacked5000: thousands of Gaussians at nearly equal depths,
# whose binary32 depth order differs from the FP64 one for many pairs (a
# different but equally valid composite); the binary32-geometry parity above
# covers them
@pytest.mark.parametrize("name", [c for c in CASES if c not in ("stacked3000-F8", "stacked5000-F8")])
def test_render_fwd_parity_fp64_geometry(name):
    """Against the all-FP64 oracle: the same tolerances on every pixel; the
    threshold margins that can excuse a pixel are 1e-3 (the binary32 mean is
    ~3e-5 px off the FP64 one), and at most 5e-3 P pixels may be excused."""
    scene, views, r, g, cfg = _render(name, 16)
    ref = oracle.render(scene, views, oracle_cfg(cfg), geometry="fp64")
    excused, rep = compare_render(r.out.cpu().numpy(), r.T_final.cpu().numpy(), r.last.cpu().numpy(), ref,
                                  geometry="fp64", scales=chan_scales(scene, float(ref["proj"][..., 6].max())),
                                  cfg=cfg)
    rep.pop("_excused_mask")
    print(name, "excused", excused, rep)


@pytest.mark.parametrize("name", ["cfg1-64x64-2k", "tiny3views-F16"])
def test_render_is_tile_size_invariant(name):
    outs = []
    for tile, lb in ((8, 64), (16, 256), (32, 128)):
        _, _, r, _, _ = _render(name, tile, lb)
        outs.append(r.out.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])


def test_persistent_forward_is_bit_identical():
    _, _, r0, _, _ = _render("tiny3views-F16", 16, 256, 0)
    _, _, r1, _, _ = _render("tiny3views-F16", 16, 256, 1)
    assert np.array_equal(r0.out.cpu().numpy(), r1.out.cpu().numpy())
    assert np.array_equal(r0.last.cpu().numpy(), r1.last.cpu().numpy())


@pytest.mark.parametrize("name", ["tiny3views-F16", "cfg2-160x120-20k-F16", "tiny-F32"])
def test_loss_grad_parity(name):
    _loss_case(name, K=20)


@pytest.mark.parametrize("K", [1, 32, 33, 64, 65, 200])
def test_loss_grad_class_counts(K):
    """Class counts around the register-cached limits (32, 64): cached logits and
    the recomputing path give the oracle's loss and gradient alike."""
    _loss_case("tiny-F8", K=K)


@pytest.mark.parametrize("name,K", [("tiny3views-F16", 1), ("tiny3views-F16", 16), ("tiny3views-F16", 17),
                                    ("cfg2-160x120-20k-F16", 20), ("tiny3views-F16", 33), ("tiny-F32", 16),
                                    ("tiny-F32", 32)])
def test_loss_grad_class_counts_wide_features(name, K):
    """Class counts with 16 and 32 feature channels (one class: the gradient
    is exactly zero), on views whose pixel counts leave partial wavefronts and
    workgroups that straddle two views."""
    _loss_case(name, K=K)


def _loss_case(name, K):
    """The loss of a synthetic render (seeded; not the GPU's render, so that
    no oracle input comes from the device) on the case's views."""
    scene, views, r, g, cfg = _render(name, 16)
    F = scene.n_feat
    rng = np.random.default_rng(7)
    P = r.views.total_pixels
    li = wl.loss_images(rng, [(v.width, v.height) for v in views], F, K)
    out32 = li.out
    rgb_t = rng.uniform(0, 1, size=(3, P)).astype(np.float32)
    dep_t = rng.uniform(1, 4, size=P).astype(np.float32)
    lab = rng.integers(0, K, size=P).astype(np.int32)
    W = wl.decoder_matrix(rng, F, K)
    wts = (0.5, 1.0, 0.01)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    r.loss_grad(dev(rgb_t), dev(dep_t), dev(lab), dev(W), wts, out=dev(out32))
    go = r.grad_out.cpu().numpy()
    gref, terms = oracle.loss(out32.astype(np.float64), views, rgb_t, dep_t, lab, W.astype(np.float64), wts)
    assert np.array_equal(np.sign(go[0:4]), np.sign(gref[0:4]))
    assert np.max(np.abs(go[0:4] - gref[0:4])) <= 1e-6 * np.max(np.abs(gref[0:4]))
    assert rel_err(go[5:], gref[5:]) <= 1e-5
    assert np.all(go[4] == 0)
    loss = r.loss.cpu().numpy()
    assert loss[3] == pytest.approx(terms[3], rel=1e-5)


def _backward_case(name, tile=16, flags=3, persistent=0, lds_batch=256, seed=11, lds_batch_bwd=0):
    scene, views, r, g, cfg = _render(name, tile, lds_batch, persistent, lds_batch_bwd)
    rng = np.random.default_rng(seed)
    go = rng.normal(size=r.out.shape).astype(np.float32) * 1e-2
    grads = g.zeros_like()
    r.render_bwd(g, torch.from_numpy(go).cuda(), flags, grads if flags & 1 else None)
    tw = r.pose_grad(g).cpu().numpy() if flags & 2 else None
    torch.cuda.synchronize()
    ref = oracle.backward(scene, views, oracle_cfg(cfg), go.astype(np.float64), flags=flags)
    return scene, views, r, grads, tw, ref


def _check_grads(scene, views, r, grads, tw, ref, flags):
    V, n, F = len(views), scene.n, scene.n_feat
    geo = r.grad_geo.cpu().numpy()
    errs = {}
    for k, nm in enumerate(["mx", "my", "A", "B", "C", "d"]):
        errs[nm] = rel_err(geo[..., k], ref["grad2d"][..., k])
    if flags & 1:
        app = r.grad_app.cpu().numpy()
        errs["o"] = rel_err(app[:, 0], ref["gapp"][:, 0])
        errs["c"] = rel_err(app[:, 1:4], ref["gapp"][:, 1:4])
        if F:
            errs["f"] = rel_err(app[:, 4:], ref["gapp"][:, 4:])
        for nm in ["mu", "log_scale", "quat", "logit", "color", "feat"]:
            if nm == "feat" and F == 0:
                continue
            errs["d" + nm] = rel_err(getattr(grads, "logit" if nm == "logit" else nm).cpu().numpy(), ref[nm])
    if flags & 2:
        for v in range(V):
            errs[f"twist{v}"] = rel_err(tw[v], ref["twist"][v])
    print(errs)
    bad = {k: e for k, e in errs.items() if e > TOL_GRAD}
    assert not bad, bad


@pytest.mark.parametrize("name", list(CASES))
def test_render_bwd_and_pose_parity(name):
    out = _backward_case(name)
    _check_grads(*out, flags=3)


@pytest.mark.parametrize("tile,lds_batch,persistent,lds_batch_bwd",
                         [(8, 64, 1, 0), (32, 128, 0, 0), (16, 256, 1, 64), (16, 64, 0, 256)])
def test_backward_launch_shapes(tile, lds_batch, persistent, lds_batch_bwd):
    out = _backward_case("tiny3views-F16", tile=tile, persistent=persistent, lds_batch=lds_batch,
                         lds_batch_bwd=lds_batch_bwd)
    _check_grads(*out, flags=3)


@pytest.mark.parametrize("name", ["tiny3views-F16", "tiny-F32"])
def test_project_without_appearance_records(name):
    """gs_project with a null appearance buffer writes the same records,
    rectangles and tile counts, and leaves the appearance records alone."""
    scene, views, r, g, cfg = _render(name, 16)
    rec, rect, touched, app = (t.clone() for t in (r.rec, r.rect, r.touched, r.app))
    r.app.fill_(7.0)
    r.rec.zero_()
    r.project(g, write_app=False)
    torch.cuda.synchronize()
    assert torch.all(r.app == 7.0)
    vis = (touched > 0).cpu().numpy()
    assert np.array_equal(r.touched.cpu().numpy(), touched.cpu().numpy())
    assert np.array_equal(r.rec.view(len(views) * scene.n, 8).cpu().numpy()[vis],
                          rec.view(len(views) * scene.n, 8).cpu().numpy()[vis])
    assert np.array_equal(r.rect.view(len(views) * scene.n, -1).cpu().numpy()[vis],
                          rect.view(len(views) * scene.n, -1).cpu().numpy()[vis])


@pytest.mark.parametrize("name", ["tiny3views-F16", "cfg1-64x64-2k", "tiny-F32"])
def test_project_bwd_write_equals_add_on_cleared(name):
    """gs_project_bwd_write into planes full of garbage gives, bit for bit,
    what gs_project_bwd adds to cleared planes, zeros included for Gaussians
    no view touches (ten moved far behind every camera)."""
    from paper_2603_27781_amd import _lib
    scene, views, r, g, cfg = _render(name, 16)
    g.mu[:, :10] = torch.tensor([0.0, 0.0, -1e3], device="cuda")[:, None]
    r.project(g)
    r.bin_sort()
    r.render_fwd()
    rng = np.random.default_rng(5)
    go = torch.from_numpy(rng.normal(size=r.out.shape).astype(np.float32) * 1e-2).cuda()
    r.render_bwd_2d(g, go, _lib.GS_GRAD_PARAMS)
    added = g.zeros_like()
    r.project_bwd(g, added)
    written = g.zeros_like()
    for t in written.tensors():
        t.copy_(torch.from_numpy(rng.normal(size=tuple(t.shape)).astype(np.float32) * 1e3))
    r.project_bwd(g, written, write=True)
    torch.cuda.synchronize()
    untouched = (r.touched.view(len(views), -1) == 0).all(dim=0).cpu().numpy()
    assert untouched.any()
    for a, b in zip(added.tensors(), written.tensors()):
        assert np.array_equal(a.cpu().numpy().view(np.uint32), b.cpu().numpy().view(np.uint32))
    assert np.all(written.mu.cpu().numpy()[:, untouched] == 0)


@pytest.mark.parametrize("flags", [3, 2])
def test_backward_split_entry_points(flags):
    """gs_render_bwd_records followed by gs_reduce_records gives the grad2d of
    gs_render_bwd (same kernels; only the order of the wavefront additions
    into LDS may differ between runs, a last-bits effect)."""
    scene, views, r, g, cfg = _render("tiny3views-F16", 16, 128, 1)
    rng = np.random.default_rng(5)
    go = torch.from_numpy(rng.normal(size=r.out.shape).astype(np.float32) * 1e-2).cuda()
    r.render_bwd_2d(g, go, flags)
    torch.cuda.synchronize()
    geo1, app1 = r.grad_geo.clone(), r.grad_app.clone()
    r.grad2d.fill_(float("nan"))
    r.render_bwd_records(g, go, flags)
    r.reduce_records(flags)
    torch.cuda.synchronize()
    assert not torch.isnan(r.grad_geo).any()
    assert rel_err(r.grad_geo.cpu().numpy(), geo1.cpu().numpy()) <= 1e-5
    if flags & 1:
        assert rel_err(r.grad_app.cpu().numpy(), app1.cpu().numpy()) <= 1e-5


def test_pose_only_backward():
    """Tracking mode (GS_GRAD_POSE only): the field is frozen, only the 2D
    geometric gradients and the twist are produced."""
    out = _backward_case("cfg1-64x64-2k", flags=2)
    _check_grads(*out, flags=2)


def test_batched_equals_sum_of_single_views():
    scene, views = CASES["tiny3views-F16"]()
    rng = np.random.default_rng(3)
    P = sum(v.width * v.height for v in views)
    go = (rng.normal(size=(5 + scene.n_feat, P)) * 1e-2).astype(np.float32)
    r, g, cfg = gpu_setup(scene, views, {"tile": 16})
    r.ensure_capacity(g)
    r.forward(g)
    gb = g.zeros_like()
    r.render_bwd(g, torch.from_numpy(go).cuda(), 3, gb)
    twb = r.pose_grad(g).cpu().numpy()
    outb = r.out.cpu().numpy()
    acc = g.zeros_like()
    off = 0
    for vi, v in enumerate(views):
        rv, gv, _ = gpu_setup(scene, [v], {"tile": 16})
        rv.ensure_capacity(gv)
        rv.forward(gv)
        Pv = v.width * v.height
        assert np.array_equal(rv.out.cpu().numpy(), outb[:, off:off + Pv])
        rv.render_bwd(gv, torch.from_numpy(np.ascontiguousarray(go[:, off:off + Pv])).cuda(), 3, acc)
        twv = rv.pose_grad(gv).cpu().numpy()
        assert rel_err(twv[0], twb[vi]) <= 1e-4
        off += Pv
    for a, b in zip(acc.tensors(), gb.tensors()):
        assert rel_err(a.cpu().numpy(), b.cpu().numpy().astype(np.float64)) <= 1e-4


def test_autograd_function_matches_direct_calls():
    from paper_2603_27781_amd import raster
    scene, views = CASES["tiny3views-F16"]()
    r, g, cfg = gpu_setup(scene, views, {"tile": 16})
    r.ensure_capacity(g)
    params = [t.clone().requires_grad_(True) for t in g.tensors()]
    xi = torch.zeros(len(views), 6, device="cuda", requires_grad=True)
    out = raster.rasterize(r, xi, *params)
    wgt = torch.randn_like(out)
    (out * wgt).sum().backward()
    direct = g.zeros_like()
    r.forward(g)
    r.render_bwd(g, wgt.contiguous(), 3, direct)
    tw = r.pose_grad(g)
    for p, d in zip(params, direct.tensors()):
        assert torch.allclose(p.grad, d, rtol=1e-4, atol=1e-6 * float(d.abs().max()))
    assert torch.allclose(xi.grad, tw, rtol=1e-4, atol=1e-6 * float(tw.abs().max()))


def test_parameter_gradients_match_fp64_central_differences():
    """The backward behind torch.autograd (raster.rasterize) against FP64
    central finite differences of the oracle's forward render, for four
    coordinates of every parameter tensor (means, log-scales, quaternions,
    opacity logits, colours, features) of visible Gaussians and all six
    twist components, on L = sum(wgt * out) with seeded weights.  The
    binary32 decisions are held: a step counts only if no pixel's contributor
    set or last contributor moves, else it is halved.  Tolerance: 1e-3 of
    the tensor's largest |gradient|."""
    import scipy.linalg
    from paper_2603_27781_amd import raster
    w = wl.tiny_scene(31, 40, F=8)
    r, g, cfg = gpu_setup(w.scene, w.views, {"tile": 16})
    r.ensure_capacity(g)
    params = [t.clone().requires_grad_(True) for t in g.tensors()]
    xi = torch.zeros(1, 6, device="cuda", requires_grad=True)
    out = raster.rasterize(r, xi, *params)
    wgt = np.random.default_rng(3).normal(size=tuple(out.shape))
    (out * torch.from_numpy(wgt.astype(np.float32)).cuda()).sum().backward()
    ocfg = oracle_cfg(cfg)
    bins = oracle.bin_instances(w.scene, w.views, ocfg)

    def lin(s64=None, poses64=None):
        ro = oracle.render(w.scene, w.views, ocfg, bins=bins, s64=s64, poses64=poses64)
        return float(np.sum(wgt * ro["out"])), (ro["last"].copy(), ro["ncontrib"].copy())

    _, key0 = lin()
    s0 = oracle.scene64(w.scene)
    rng = np.random.default_rng(4)
    vis = np.nonzero(bins["dec"]["touched"][0] > 0)[0]
    checked = 0
    for nm, p in zip(("mu", "log_scale", "quat", "logit", "color", "feat"), params):
        grad = p.grad.cpu().numpy().astype(np.float64)
        scale = max(float(np.max(np.abs(grad))), 1e-30)
        for _ in range(4):
            i = int(rng.choice(vis))
            idx = (int(rng.integers(0, s0[nm].shape[0])), i) if s0[nm].ndim == 2 else (i,)
            x = s0[nm][idx]
            h = 1e-6 * max(1.0, abs(x))
            fd = None
            while h > 1e-9:
                sp = {k: v.copy() for k, v in s0.items()}
                sm = {k: v.copy() for k, v in s0.items()}
                sp[nm][idx] = x + h
                sm[nm][idx] = x - h
                lp, kp = lin(s64=sp)
                lm, km = lin(s64=sm)
                if all(np.array_equal(a, c) for a, c in zip(kp + km, key0 + key0)):
                    fd = (lp - lm) / (2 * h)
                    break
                h *= 0.5
            if fd is None:
                continue
            assert abs(grad[idx] - fd) <= 1e-3 * scale, (nm, idx, grad[idx], fd, scale)
            checked += 1
    assert checked >= 20
    # the twist: left perturbation Exp(xi) T_CW
    T0 = np.eye(4)
    T0[:3] = np.asarray(w.views[0].Rt, np.float32).astype(np.float64)

    def hat(v):
        M = np.zeros((4, 4))
        M[:3, :3] = np.array([[0, -v[5], v[4]], [v[5], 0, -v[3]], [-v[4], v[3], 0]])
        M[:3, 3] = v[:3]
        return M

    tw = xi.grad.cpu().numpy()[0].astype(np.float64)
    fd6 = np.zeros(6)
    for k in range(6):
        e6 = np.zeros(6)
        e6[k] = 1e-6
        lp, kp = lin(poses64=[scipy.linalg.expm(hat(e6)) @ T0])
        lm, km = lin(poses64=[scipy.linalg.expm(hat(-e6)) @ T0])
        assert all(np.array_equal(a, c) for a, c in zip(kp + km, key0 + key0))
        fd6[k] = (lp - lm) / 2e-6
    assert rel_err(tw, fd6) <= 1e-3, (tw, fd6)


def test_edge_cases_empty_and_single():
    # every Gaussian behind the camera: nothing visible, background 0, T = 1
    w = wl.tiny_scene(71, 50, F=8)
    sc = w.scene.copy()
    sc.mu[2] = -5.0
    r, g, cfg = gpu_setup(sc, w.views, {"tile": 16})
    r.forward(g)
    torch.cuda.synchronize()
    assert r.instance_counts()[0] == 0
    assert float(r.out.abs().max()) == 0.0 and float(r.T_final.min()) == 1.0
    grads = g.zeros_like()
    r.render_bwd(g, torch.ones_like(r.out), 3, grads)
    assert all(float(t.abs().max()) == 0.0 for t in grads.tensors())
    # a single Gaussian
    s1 = w.scene.subset(np.array([3]))
    out = _single(s1, w.views)
    assert out


def _single(scene, views):
    r, g, cfg = gpu_setup(scene, views, {"tile": 8, "lds_batch": 64})
    r.ensure_capacity(g)
    r.forward(g)
    ref = oracle.render(scene, views, oracle_cfg(cfg), geometry="fp32")
    excused, _ = compare_render(r.out.cpu().numpy(), r.T_final.cpu().numpy(), r.last.cpu().numpy(), ref,
                                scales=chan_scales(scene, float(ref["proj"][..., 6].max())), cfg=cfg)
    return excused == 0


def test_abi_rejects_bad_arguments_without_launching():
    from paper_2603_27781_amd import _lib, raster
    scene, views = CASES["tiny-F8"]()
    r, g, cfg = gpu_setup(scene, views, {"tile": 16})
    L = _lib.load()
    bad = raster.Config(tile=12).c()
    import ctypes
    st = L.gs_project(ctypes.byref(g.c()), r.views.host, r.views.dev_ptr(), 1, ctypes.byref(bad), r.rec.data_ptr(),
                      r.rect.data_ptr(), r.touched.data_ptr(), r.app.data_ptr(), None)
    assert st == _lib.GS_EUNSUPPORTED
    st = L.gs_project(ctypes.byref(g.c()), r.views.host, r.views.dev_ptr(), 1, ctypes.byref(r.cc), None,
                      r.rect.data_ptr(), r.touched.data_ptr(), r.app.data_ptr(), None)
    assert st == _lib.GS_EINVAL
    st = L.gs_bin_sort(r.rect.data_ptr(), r.touched.data_ptr(), r.n, r.views.host,
                       r.views.dev_ptr(), 1, ctypes.byref(r.cc), r.ws_view.data_ptr(), 16, r.capacity,
                       r.keys.data_ptr(), r.inst.data_ptr(), r.inst_gid.data_ptr(), r.pair_first.data_ptr(),
                       r.ranges.data_ptr(), r.counts.data_ptr(), None)
    assert st == _lib.GS_ECAPACITY


def test_views_check_counts_the_views_whose_copies_differ():
    """gs_views_check: 0 when the device copy equals the host array, 0 after
    the poses change on the device only (the poses are not compared), and
    one per view whose size, offset or intrinsics differ."""
    _scene, views = CASES["tiny3views-F16"]()
    from paper_2603_27781_amd import raster
    vw = raster.Views(views, 16)
    assert vw.check() == 0
    Rts = torch.from_numpy(np.stack([np.asarray(v.Rt, np.float32) for v in views]) * 1.01).cuda()
    vw.set_poses(Rts)
    assert vw.check() == 0
    words = vw.dev.view(torch.int32)
    words[1, 0] += 1  # width of view 1
    assert vw.check() == 1
    words[1, 0] -= 1
    vw.dev.view(torch.float32)[2, 4] += 0.5  # cx of view 2
    assert vw.check() == 1
    words[0, 1] += 3  # height of view 0
    assert vw.check() == 2


def test_lookback_give_up_is_reported_and_the_binning_stands_down(monkeypatch):
    """A wait of the sort's single-pass scan that gives up -- forced from the
    host with SGS_LOOKBACK_SPIN=0, so a block never waits for a predecessor
    that has not published yet, and every kernel still exits normally -- is
    reported in counts[3] and in the sticky counts[4]; the later binning
    kernels then stand down and leave every tile list empty (the render is
    background).  Without the override the next call bins bit-exactly."""
    scene, views = CASES["cfg2-160x120-20k-F16"]()
    # a large capacity: 1024 radix blocks, so each digit scan runs over 128 tiles
    r, g, cfg = gpu_setup(scene, views, {"tile": 16}, capacity=8_000_000)
    r.project(g)
    monkeypatch.setenv("SGS_LOOKBACK_SPIN", "0")
    seen = []
    for _ in range(5):
        r.clear_trouble()
        r.bin_sort()
        c = r.instance_counts()
        seen.append(c.lookback_gave_up)
        if c.lookback_gave_up:
            assert r.trouble() and not c.overflow
            assert not r.ranges.any()
            r.render_fwd()
            torch.cuda.synchronize()
            assert float(r.out.abs().max()) == 0.0 and float(r.T_final.min()) == 1.0
    assert any(seen), "no wait gave up in five calls with a spin limit of 0"
    monkeypatch.delenv("SGS_LOOKBACK_SPIN")
    r.clear_trouble()
    r.bin_sort()
    c = r.instance_counts()
    assert not c.lookback_gave_up and not c.overflow and not r.trouble()
    ref = oracle.bin_instances(scene, views, oracle_cfg(cfg))
    assert c.instances == ref["count"]
    assert np.array_equal(r.keys[:c.instances].cpu().numpy().view(np.uint32), ref["keys"])
    assert np.array_equal(r.sorted_gids(c.instances).cpu().numpy(), ref["gids"])
    assert np.array_equal(r.ranges.view(-1, 2).cpu().numpy(), ref["ranges"])
