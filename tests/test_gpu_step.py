"""The batched step as the benchmark runs it: `batched.MappingStep` captured
once in a HIP graph and replayed, in the benchmark's launch configuration.

Each replay is compared with an eager run of the same step (forward, loss
and loss gradient bit for bit, gradients up to the last bits) and with the
FP64 oracle on every pixel and every Gaussian; between the two replays every
camera moves (through the device pose records the captured kernels read).
`PerViewStep`, the plain per-view alternative the benchmark compares
against, must give the batched step's images, losses, gradients and twists.
Paper: Sec. 3.3.3-3.3.4, Eq. (13)-(14) (mapping over sampled keyframes)."""
import numpy as np
import pytest

from paper_2603_27781_amd import workloads as wl
from gpu_common import (CASES, _log, assert_same_step, gpu_backward_of, rel_err, step_oracle_parity,
                        step_snapshot)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WEIGHTS = (0.5, 1.0, 0.01)


def _dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _targets(views, F, K, seed):
    """Seeded targets of the views' sizes (data, never a render of this path)."""
    rng = np.random.default_rng(seed)
    P = sum(v.width * v.height for v in views)
    rgb = rng.uniform(0, 1, (3, P)).astype(np.float32)
    dep = rng.uniform(1, 4, P).astype(np.float32)
    lab = rng.integers(0, K, P).astype(np.int32) if K else None
    W = wl.decoder_matrix(rng, F, K) if K else None
    return rgb, dep, lab, W


def _step(name, persistent=0, pose=True):
    from paper_2603_27781_amd import batched, raster
    scene, views = CASES[name]()
    F = scene.n_feat
    K = 20 if F else 0
    rgb, dep, lab, W = _targets(views, F, K, 17)
    cfg = raster.Config(**dict(batched.BENCH_CONFIG, persistent=persistent))
    g = raster.Gaussians.from_numpy(scene)
    step = batched.MappingStep(g, views, cfg, _dev(rgb), _dev(dep), _dev(lab), _dev(W), WEIGHTS, params=True,
                               pose=pose)
    step.ensure_capacity(slack=1.5)
    return step, scene, views, cfg, (rgb, dep, lab, W)


def _moved(views, rng):
    out = []
    for v in views:
        xi = rng.normal(size=6) * np.array([0.01, 0.01, 0.01, 0.01, 0.01, 0.01])
        T = np.eye(4)
        T[:3] = np.asarray(v.Rt, np.float64)
        out.append(wl.make_view(v.width, v.height, v.fx, wl.se3_exp(xi) @ T, v.cx, v.cy))
    return out


@pytest.mark.parametrize("name,persistent", [("tiny3views-F16", 0), ("tiny3views-F16", 1), ("40views-F8", 0),
                                             ("cfg2-160x120-20k-F16", 0), ("empty-view-F8", 1)])
def test_mapping_step_replays_match_eager_and_oracle(name, persistent):
    step, scene, views, cfg, (rgb, dep, lab, W) = _step(name, persistent)
    step.capture()
    rng = np.random.default_rng(23)
    cur = list(views)
    for it in range(2):
        if it == 1:
            cur = _moved(views, rng)
            step.views.set_poses(torch.from_numpy(np.stack([v.Rt for v in cur]).astype(np.float32)).cuda())
        _log(name, "replay", it)
        step.replay()
        a = step_snapshot(step)
        step.run()
        b = step_snapshot(step)
        assert_same_step(a, b)
        step_oracle_parity(a, step.r, scene, cur, cfg, rgb, dep, lab, W, WEIGHTS, flags=3,
                           gpu_backward=gpu_backward_of(step))


@pytest.mark.parametrize("name", ["tiny3views-F16", "40views-F8", "empty-view-F8"])
def test_per_view_step_equals_batched_step(name):
    """V plain single-view passes (no graph) give the batched step's images
    bit for bit, the same per-view losses, and gradients and twists equal up
    to the order in which the views' contributions are added."""
    from paper_2603_27781_amd import batched, raster
    step, scene, views, cfg, (rgb, dep, lab, W) = _step(name)
    step.run()
    a = step_snapshot(step)
    g = step.g
    pv = batched.PerViewStep(g, views, cfg, _dev(rgb), _dev(dep), _dev(lab), _dev(W), WEIGHTS, params=True,
                             pose=True)
    pv.ensure_capacity()
    pv.run()
    torch.cuda.synchronize()
    off = 0
    loss = 0.0
    for v, st in zip(views, pv.steps):
        P = v.width * v.height
        assert np.array_equal(st.r.out.cpu().numpy(), a["out"][:, off:off + P])
        loss += float(st.r.loss[3])
        off += P
    assert loss == pytest.approx(float(a["loss"][3]), rel=1e-6)
    for nm, t in zip(("mu", "log_scale", "quat", "logit", "color", "feat"), pv.grads.tensors()):
        assert rel_err(t.cpu().numpy(), a["grads"][nm].astype(np.float64)) <= 1e-5, nm
    for vi, st in enumerate(pv.steps):
        assert rel_err(st.r.twist.cpu().numpy()[0], a["twist"][vi].astype(np.float64)) <= 1e-5, vi


@pytest.mark.parametrize("name,persistent,tile,weights", [
    ("tiny3views-F16", 0, 16, WEIGHTS), ("tiny3views-F16", 1, 16, WEIGHTS), ("40views-F8", 0, 8, WEIGHTS),
    ("cfg2-160x120-20k-F16", 0, 32, WEIGHTS), ("empty-view-F8", 1, 16, WEIGHTS), ("tiny-F0", 0, 16, WEIGHTS),
    ("tiny3views-F16", 0, 16, (0.5, 1.0, 0.0))])
def test_fused_forward_loss_equals_separate_calls(name, persistent, tile, weights):
    """gs_render_fwd_loss (the loss in the forward kernel's epilogue, what the
    batched step runs) writes what gs_render_fwd followed by gs_loss_grad
    writes: the render, T_final and last bit for bit, the loss gradient bit
    for bit (the same per-pixel arithmetic on the same binary32 values), and
    the loss terms up to the grouping of their FP64 sums (per tile against
    per block of pixels).  Paper: Sec. 3.2.1-3.2.2 Eq. (4)-(8), Sec. 3.3.4."""
    from paper_2603_27781_amd import batched, raster
    scene, views = CASES[name]()
    F = scene.n_feat
    K = 20 if F else 0
    rgb, dep, lab, W = _targets(views, F, K, 29)
    cfg = raster.Config(**dict(batched.BENCH_CONFIG, tile=tile, persistent=persistent))
    g = raster.Gaussians.from_numpy(scene)
    step = batched.MappingStep(g, views, cfg, _dev(rgb), _dev(dep), _dev(lab), _dev(W), weights, params=True)
    assert step.fuse_loss
    step.ensure_capacity(slack=1.5)
    r = step.r
    _log(name, "tile", tile, "persistent", persistent, "weights", weights)
    r.project(g)
    r.bin_sort()
    args = (step.rgb_t, step.depth_t, step.labels, step.decoder, weights)
    r.out.fill_(float("nan"))
    r.grad_out.fill_(float("nan"))
    r.render_fwd_loss(*args)
    torch.cuda.synchronize()
    fused = {k: t.cpu().numpy().copy() for k, t in
             (("out", r.out), ("T", r.T_final), ("last", r.last), ("grad_out", r.grad_out), ("loss", r.loss))}
    r.out.fill_(float("nan"))
    r.grad_out.fill_(float("nan"))
    r.render_fwd()
    r.loss_grad(*args)
    torch.cuda.synchronize()
    sep = {k: t.cpu().numpy().copy() for k, t in
           (("out", r.out), ("T", r.T_final), ("last", r.last), ("grad_out", r.grad_out), ("loss", r.loss))}
    for k in ("out", "T", "last", "grad_out"):
        assert np.array_equal(fused[k], sep[k]), k
    assert np.all(np.isfinite(fused["grad_out"]))
    np.testing.assert_allclose(fused["loss"], sep["loss"], rtol=1e-12, atol=1e-300)
    if weights[2] == 0.0 or K == 0:
        assert fused["loss"][2] == 0.0


def test_mapping_step_falls_back_beyond_the_fused_class_count():
    """With more classes than the fused forward keeps in registers the step
    makes the two separate calls, and its replay still matches the eager run
    and the oracle."""
    from paper_2603_27781_amd import batched, raster
    scene, views = CASES["tiny3views-F16"]()
    rgb, dep, lab, W = _targets(views, scene.n_feat, 21, 31)
    cfg = raster.Config(**batched.BENCH_CONFIG)
    g = raster.Gaussians.from_numpy(scene)
    step = batched.MappingStep(g, views, cfg, _dev(rgb), _dev(dep), _dev(lab), _dev(W), WEIGHTS, params=True,
                               pose=True)
    assert not step.fuse_loss
    step.ensure_capacity(slack=1.5)
    step.capture()
    step.replay()
    a = step_snapshot(step)
    step.run()
    assert_same_step(a, step_snapshot(step))
    step_oracle_parity(a, step.r, scene, views, cfg, rgb, dep, lab, W, WEIGHTS, flags=3,
                       gpu_backward=gpu_backward_of(step))
