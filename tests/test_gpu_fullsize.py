"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times, with nothing sampled: integer work (culling, rectangles,
instance lists, sorted order, ranges) bit for bit; every pixel of every
view, every visible pair's 2D gradient, every Gaussian's parameter gradients
and every view's twist against the FP64 oracle.

Tolerances: RGB and opacity 1e-5 max-abs; depth and features 1e-4 of the
channel's max; gradients and twists 1e-3 of the tensor's max."""
import time

import numpy as np
import pytest

import oracle
from paper_2603_27781_amd import workloads as wl
from gpu_common import (assert_same_step, chan_scales, compare_render, gpu_backward_of, gpu_setup, oracle_cfg,
                        rel_err, step_oracle_parity, step_snapshot, tie_free_targets)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _log(*a):
    print(f"[{time.strftime('%H:%M:%S')}]", *a, flush=True)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _bench_cfg():
    from paper_2603_27781_amd.batched import BENCH_CONFIG
    return dict(BENCH_CONFIG)


def _check_binning(scene, views, r, cfg):
    dec = oracle.decide(scene, views, oracle_cfg(cfg))
    V, n = len(views), scene.n
    touched = r.touched.view(V, n).cpu().numpy()
    assert np.array_equal(touched, dec["touched"])
    rec = r.rec.view(V, n, 8).cpu().numpy()
    vis = touched > 0
    for k_gpu, k_orc in ((0, 0), (1, 1), (6, 5)):
        assert np.array_equal(rec[..., k_gpu][vis].view(np.uint32), dec["rec32"][..., k_orc][vis].view(np.uint32))
    ref = oracle.bin_instances(scene, views, oracle_cfg(cfg), dec=dec)
    inst, nvis, over, gave_up = r.instance_counts()
    assert not over and not gave_up and inst == ref["count"] and nvis == int(vis.sum())
    assert np.array_equal(r.keys[:inst].cpu().numpy().view(np.uint32), ref["keys"])
    assert np.array_equal(r.sorted_gids(inst).cpu().numpy(), ref["gids"])
    assert np.array_equal(r.ranges.view(-1, 2).cpu().numpy(), ref["ranges"])
    _log("binning bit-exact:", inst, "instances,", nvis, "visible pairs")
    return ref


def _run_step(w, cfg_kw, targets, flags):
    from paper_2603_27781_amd import raster
    r, g, cfg = gpu_setup(w.scene, w.views, cfg_kw)
    r.ensure_capacity(g)
    r.forward(g)
    rgb, dep, lab = targets
    W = _dev(w.decoder) if w.decoder is not None else None
    go = r.loss_grad(_dev(rgb), _dev(dep), _dev(lab) if lab is not None else None, W, w.weights)
    grads = g.zeros_like() if flags & 1 else None
    r.render_bwd(g, go, flags, grads)
    tw = r.pose_grad(g).cpu().numpy() if flags & 2 else None
    torch.cuda.synchronize()
    return r, g, cfg, grads, tw


def test_config2_full_image_parity():
    """640x480, 200k Gaussians, F=16, CE over 20 classes; targets are the
    oracle's render of the seed-perturbed copy at the identity pose."""
    w = wl.config2()
    ocfg = oracle.Cfg(tile=16)
    tgt = oracle.render(w.target_scene, w.target_views, ocfg)
    rgb_t = tgt["out"][0:3].astype(np.float32)
    dep_t = tgt["out"][3].astype(np.float32)
    lab = w.targets.labels
    _log("targets rendered")
    r, g, cfg, grads, tw = _run_step(w, {"tile": 16}, (rgb_t, dep_t, lab), 3)
    _check_binning(w.scene, w.views, r, cfg)
    ref = oracle.render(w.scene, w.views, oracle_cfg(cfg), geometry="fp32")
    excused, rep = compare_render(r.out.cpu().numpy(), r.T_final.cpu().numpy(), r.last.cpu().numpy(), ref,
                                  scales=chan_scales(w.scene, float(ref["proj"][..., 6].max())), cfg=cfg,
                                  max_flipped=0)
    rep.pop("_excused_mask")
    _log("forward", rep)
    ref64 = oracle.render(w.scene, w.views, oracle_cfg(cfg), bins=ref["bins"])
    gout, terms = oracle.loss(ref64["out"], w.views, rgb_t, dep_t, lab, w.decoder.astype(np.float64), w.weights)
    assert float(r.loss[3]) == pytest.approx(terms[3], rel=1e-4)
    b = oracle.backward(w.scene, w.views, oracle_cfg(cfg), gout, bins=ref["bins"], flags=3)
    errs = {nm: rel_err(getattr(grads, nm).cpu().numpy(), b[nm]) for nm in
            ("mu", "log_scale", "quat", "logit", "color", "feat")}
    errs["twist"] = rel_err(tw[0], b["twist"][0])
    _log("gradients", errs)
    assert max(errs.values()) <= 1e-3, errs


@pytest.mark.timeout(300)
def test_config3_tracking_twist_and_finite_differences():
    """1200x680, 1M room Gaussians, pose-only (tracking).  GPU twist vs the
    oracle's analytic twist, and the oracle's twist vs FP64 central finite
    differences of Exp(xi) T_CW on the pixels whose alpha_min / T_min
    decisions sit at least 1e-3 (relative) from their thresholds."""
    import scipy.linalg
    w = wl.config3()
    ocfg = oracle.Cfg(tile=16)
    tgt = oracle.render(w.target_scene, w.target_views, ocfg)
    rgb_t = tgt["out"][0:3].astype(np.float32)
    dep_t = tgt["out"][3].astype(np.float32)
    logits = tgt["out"][5:].T @ w.decoder.astype(np.float64)
    lab = logits.argmax(axis=1).astype(np.int32)
    _log("targets rendered")
    r, g, cfg, _, tw = _run_step(w, _bench_cfg(), (rgb_t, dep_t, lab), 2)
    ref = oracle.render(w.scene, w.views, oracle_cfg(cfg))
    gout, _ = oracle.loss(ref["out"], w.views, rgb_t, dep_t, lab, w.decoder.astype(np.float64), w.weights)
    b = oracle.backward(w.scene, w.views, oracle_cfg(cfg), gout, bins=ref["bins"], flags=2)
    e = rel_err(tw[0], b["twist"][0])
    _log("twist gpu", tw[0], "oracle", b["twist"][0], "rel", e)
    assert e <= 1e-3
    # finite differences on the well-separated pixels (decisions at least 1e-2
    # from their thresholds; a 1e-7 step moves a mean by ~6e-5 px, far too
    # little to flip them, which the decision-set guard below confirms)
    S = (ref["margin_a"] > 1e-2) & (ref["margin_t"] > 1e-2)
    gS = gout * S[None, :]
    bS = oracle.backward(w.scene, w.views, oracle_cfg(cfg), gS, bins=ref["bins"], flags=2)
    T0 = np.eye(4)
    T0[:3] = np.asarray(w.views[0].Rt, np.float32).astype(np.float64)

    def hat(xi):
        M = np.zeros((4, 4))
        M[:3, :3] = np.array([[0, -xi[5], xi[4]], [xi[5], 0, -xi[3]], [-xi[4], xi[3], 0]])
        M[:3, 3] = xi[:3]
        return M

    h = 1e-7
    fd = np.zeros(6)
    for k in range(6):
        e6 = np.zeros(6)
        e6[k] = h
        lp = oracle.render(w.scene, w.views, oracle_cfg(cfg), bins=ref["bins"],
                           poses64=[scipy.linalg.expm(hat(e6)) @ T0])
        lm = oracle.render(w.scene, w.views, oracle_cfg(cfg), bins=ref["bins"],
                           poses64=[scipy.linalg.expm(hat(-e6)) @ T0])
        assert np.array_equal(lp["ncontrib"][S], ref["ncontrib"][S])
        assert np.array_equal(lm["ncontrib"][S], ref["ncontrib"][S])
        fd[k] = (np.sum(gS * lp["out"]) - np.sum(gS * lm["out"])) / (2 * h)
    _log("fd", fd, "analytic", bS["twist"][0])
    assert rel_err(bS["twist"][0], fd) <= 1e-5
    # and the GPU on the same pixel set
    r.render_bwd(g, _dev((r.grad_out.cpu().numpy() * S[None, :]).astype(np.float32)), 2, None)
    twS = r.pose_grad(g).cpu().numpy()
    assert rel_err(twS[0], fd) <= 1e-3


def _bench_step(w, cfg_kw, params, pose, rgb_t, dep_t):
    """The step bench.py times: MappingStep in the given launch
    configuration, capacity sized, captured, replayed twice."""
    from paper_2603_27781_amd import batched, raster
    cfg = raster.Config(**cfg_kw)
    g = raster.Gaussians.from_numpy(w.scene)
    W = _dev(w.decoder) if w.decoder is not None else None
    step = batched.MappingStep(g, w.views, cfg, _dev(rgb_t), _dev(dep_t), _dev(w.targets.labels),
                               W, w.weights, params=params, pose=pose)
    step.ensure_capacity()
    step.capture(warmup=1)
    step.replay()
    step.replay()
    return step, cfg


def _oracle_first(w):
    """The oracle's binning and render of the workload (binary32 decision
    geometry), and colour / depth targets a seeded margin away from that
    render (the workload's own analytic targets can equal the render to
    within rounding at some pixels, where the L1 subgradient's sign is not
    defined by either precision); labels stay the workload's."""
    from paper_2603_27781_amd import raster
    ocfg = oracle_cfg(raster.Config(**_bench_cfg()))
    bins = oracle.bin_instances(w.scene, w.views, ocfg)
    ref = oracle.render(w.scene, w.views, ocfg, bins=bins, geometry="fp32")
    rgb_t, dep_t = tie_free_targets(ref["out"], w.seed + 300)
    _log("oracle render and targets")
    return bins, ref, rgb_t, dep_t


@pytest.mark.timeout(900)
def test_config4_benchmarked_step_full_parity():
    """8 x 1200x680 keyframes, 1M room Gaussians, F=16, CE over 20 classes,
    parameter gradients: the graph-captured step in the benchmark's launch
    configuration, after two replays.  Replay equals an eager run, and the
    oracle agrees on every one of the 6.5M pixels, every visible (view,
    Gaussian) pair's 2D gradient and every Gaussian's parameter gradients."""
    w = wl.config4()
    bins, ref, rgb_t, dep_t = _oracle_first(w)
    step, cfg = _bench_step(w, _bench_cfg(), params=True, pose=False, rgb_t=rgb_t, dep_t=dep_t)
    a = step_snapshot(step)
    step.run()
    assert_same_step(a, step_snapshot(step))
    _log("replay equals eager")
    step_oracle_parity(a, step.r, w.scene, w.views, cfg, rgb_t, dep_t, w.targets.labels, w.decoder, w.weights,
                       flags=1, bins=bins, ref=ref, gpu_backward=gpu_backward_of(step))


@pytest.mark.timeout(900)
def test_config5_uneven_batched_step_full_parity_and_vs_per_view():
    """16 views at mixed resolutions, 2M Gaussians, F=32, CE over 50
    classes, parameter gradients and a twist for every view: the captured
    step (benchmark configuration) against the oracle on every pixel, every
    Gaussian and all 16 twists; the persistent launch mode gives the same
    step; 16 plain per-view passes give the same images, gradients and
    twists."""
    from paper_2603_27781_amd import batched
    w = wl.config5()
    bins, ref, rgb_t, dep_t = _oracle_first(w)
    step, cfg = _bench_step(w, _bench_cfg(), params=True, pose=True, rgb_t=rgb_t, dep_t=dep_t)
    a = step_snapshot(step)
    step.run()
    assert_same_step(a, step_snapshot(step))
    _log("replay equals eager")
    step_oracle_parity(a, step.r, w.scene, w.views, cfg, rgb_t, dep_t, w.targets.labels, w.decoder, w.weights,
                       flags=3, bins=bins, ref=ref, gpu_backward=gpu_backward_of(step))
    # the persistent launch mode of the same step
    pst, _ = _bench_step(w, dict(_bench_cfg(), persistent=1), params=True, pose=True, rgb_t=rgb_t, dep_t=dep_t)
    assert_same_step(a, step_snapshot(pst))
    del pst
    _log("persistent mode equals")
    # 16 plain per-view passes
    pv = batched.PerViewStep(step.g, w.views, cfg, step.rgb_t, step.depth_t, step.labels, step.decoder, w.weights,
                             params=True, pose=True)
    pv.ensure_capacity()
    pv.run()
    torch.cuda.synchronize()
    off = 0
    for v, st in zip(w.views, pv.steps):
        Pv = v.width * v.height
        assert np.array_equal(st.r.out.cpu().numpy(), a["out"][:, off:off + Pv])
        off += Pv
    for nm, t in zip(("mu", "log_scale", "quat", "logit", "color", "feat"), pv.grads.tensors()):
        assert rel_err(t.cpu().numpy(), a["grads"][nm].astype(np.float64)) <= 1e-5, nm
    twv = np.array([st.r.twist.cpu().numpy()[0] for st in pv.steps])
    assert rel_err(twv, a["twist"].astype(np.float64)) <= 1e-5
