"""GPU parity of gs_slam_loss (the SLAM losses with masks and the SSIM
colour term) against the FP64 oracle, on seeded synthetic renders and
targets (workloads.loss_images; none of the inputs comes from the GPU).

  - median depth errors and masks: bit-exact (both sides decide in binary32);
  - gradients: within 1e-3 of the tensor's max |oracle| (the L1 signs exact
    where the SSIM term is off);
  - loss terms: 1e-5 relative (SSIM term 1e-4: it sums 1 - s, which loses
    digits to cancellation in binary32).
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2603_27781_amd import workloads as wl
from gpu_common import TOL_GRAD, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MODES = {
    # mapping loss of Eq. (18) without the scale terms: L1 + SSIM colour (lambda 0.2), depth, semantic
    "mapping": dict(ssim_lambda=0.2, use_obs=False, w_sem=0.01),
    # tracking loss of Eq. (21): every term under M_obs, L1 colour only
    "tracking": dict(ssim_lambda=0.0, use_obs=True, w_sem=0.001),
    # both at once (the mask also weights the per-pixel SSIM)
    "masked-ssim": dict(ssim_lambda=0.2, use_obs=True, w_sem=0.01),
}

SIZES = {
    "3views-ragged": [(61, 37), (40, 52), (17, 9)],
    "degenerate": [(1, 1), (3, 2), (33, 17), (32, 16)],
}


def _rasterizer(sizes, F):
    from paper_2603_27781_amd import raster
    views = [wl.make_view(W, H, 0.8 * max(W, H), np.eye(4)) for (W, H) in sizes]
    cfg = raster.Config()
    return raster.Rasterizer(1, F, raster.Views(views, cfg.tile), cfg, capacity=1024)


def _opts(mode):
    from paper_2603_27781_amd import _lib
    m = MODES[mode]
    L = _lib.load()
    o = _lib.GsSlamLossOpts()
    L.gs_default_slam_loss_opts(ctypes.byref(o))
    o.ssim_lambda = m["ssim_lambda"]
    o.w_sem = m["w_sem"]
    o.flags = _lib.GS_LOSS_OBS_MASK if m["use_obs"] else 0
    oo = oracle.SlamLossOpts(w_color=o.w_color, w_depth=o.w_depth, w_sem=o.w_sem, ssim_lambda=o.ssim_lambda,
                             tau_obs=o.tau_obs, tau_unobs=o.tau_unobs, obs_factor=o.obs_factor,
                             unobs_factor=o.unobs_factor, use_obs=m["use_obs"])
    return o, oo


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run(r, li, W, o):
    out = _dev(li.out)
    r.slam_loss(_dev(li.rgb_t), _dev(li.depth_t), _dev(li.labels), _dev(W) if W is not None else None, o, out=out)
    torch.cuda.synchronize()
    return (r.grad_out.cpu().numpy(), r.slam_terms.cpu().numpy(), r.masks.cpu().numpy(),
            r.median.cpu().numpy())


def _check(go, terms, masks, med, ref, lam):
    gref, tref, mref, medref = ref
    assert np.array_equal(med.view(np.uint32), medref.view(np.uint32)), (med, medref)
    assert np.array_equal(masks, mref), int(np.sum(masks != mref))
    assert np.all(go[4] == 0)
    # depth: L1 only, exact signs
    assert np.array_equal(np.sign(go[3]), np.sign(gref[3]))
    assert rel_err(go[3], gref[3]) <= 1e-6
    if lam == 0.0:
        assert np.array_equal(np.sign(go[:3]), np.sign(gref[:3]))
    assert rel_err(go[:3], gref[:3]) <= TOL_GRAD, rel_err(go[:3], gref[:3])
    if go.shape[0] > 5:
        assert rel_err(go[5:], gref[5:]) <= 1e-5
    for k, tol in zip(range(5), (1e-5, 1e-4, 1e-5, 1e-5, 1e-5)):
        assert terms[k] == pytest.approx(tref[k], rel=tol, abs=1e-12), (k, terms, tref)


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("F,K", [(16, 20), (8, 40), (0, 0)])
@pytest.mark.parametrize("sizes", list(SIZES))
def test_slam_loss_parity(sizes, F, K, mode):
    sz = SIZES[sizes]
    rng = np.random.default_rng(21 + F)
    li = wl.loss_images(rng, sz, F, K)
    if sizes == "degenerate":
        off = sz[0][0] * sz[0][1] + sz[1][0] * sz[1][1]
        li.depth_t[off:off + sz[2][0] * sz[2][1]] = 0.0  # a view without valid depth
    W = wl.decoder_matrix(rng, F, K) if K > 0 and F > 0 else None
    o, oo = _opts(mode)
    r = _rasterizer(sz, F)
    got = _run(r, li, W, o)
    ref = oracle.slam_loss(li.out, sz, li.rgb_t, li.depth_t, li.labels if W is not None else None,
                           None if W is None else W.astype(np.float64), oo)
    _check(*got, ref, oo.ssim_lambda)
    if sizes == "degenerate":
        assert got[3][2] == 0.0 and not np.any(got[2][off:off + 33 * 17] & 1)


def test_slam_loss_deterministic_and_graph_replay():
    sz = SIZES["3views-ragged"]
    rng = np.random.default_rng(5)
    li = wl.loss_images(rng, sz, 16, 20)
    W = _dev(wl.decoder_matrix(rng, 16, 20))
    o, _ = _opts("masked-ssim")
    r = _rasterizer(sz, 16)
    out, rgb, dep, lab = _dev(li.out), _dev(li.rgb_t), _dev(li.depth_t), _dev(li.labels)
    r.slam_loss(rgb, dep, lab, W, o, out=out)  # allocates the workspace
    torch.cuda.synchronize()
    g0, t0, m0 = r.grad_out.clone(), r.slam_terms.clone(), r.masks.clone()
    r.slam_loss(rgb, dep, lab, W, o, out=out)
    torch.cuda.synchronize()
    assert torch.equal(r.slam_terms, t0) and torch.equal(r.grad_out, g0) and torch.equal(r.masks, m0)
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            r.slam_loss(rgb, dep, lab, W, o, out=out)
    torch.cuda.current_stream().wait_stream(s)
    for k in range(3):
        r.grad_out.fill_(7.0)
        r.slam_terms.fill_(-1.0)
        r.masks.fill_(255)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(r.slam_terms, t0), k
        assert torch.equal(r.grad_out, g0), k
        assert torch.equal(r.masks, m0), k


def _crop_ref(li, sizes, view, q, med, W, oo, F):
    """Oracle gradient at pixel q = (row, col) of `view`, from the crop
    q +- 10 (clipped to the view): every windowed sum that reaches q lies in
    it, and the means divide by the full view's pixel count."""
    Wv, Hv = sizes[view]
    base = sum(w * h for (w, h) in sizes[:view])
    r0, r1 = max(q[0] - 10, 0), min(q[0] + 11, Hv)
    c0, c1 = max(q[1] - 10, 0), min(q[1] + 11, Wv)
    rows = np.arange(r0, r1)[:, None] * Wv + np.arange(c0, c1)[None, :] + base
    idx = rows.reshape(-1)
    out = li.out[:, idx].astype(np.float64)
    g, _, m, _ = oracle.slam_loss(out, [(c1 - c0, r1 - r0)], li.rgb_t[:, idx], li.depth_t[idx],
                                  li.labels[idx], W, oo, medians=np.float32([med]), norm_counts=[Wv * Hv])
    k = (q[0] - r0) * (c1 - c0) + (q[1] - c0)
    return g[:, k], m[k], base + q[0] * Wv + q[1]


def test_slam_loss_full_size_sampled():
    """Eight 1200x680 views, F = 16, 20 classes, mapping loss with the
    observed mask: medians and masks of every pixel bit-exact, the L1 and
    depth terms against the full oracle, the gradient of 96 sampled pixels
    (corners, edges, interior) against oracle crops."""
    F, K = 16, 20
    sz = [(1200, 680)] * 8
    rng = np.random.default_rng(77)
    li = wl.loss_images(rng, sz, F, K)
    W = wl.decoder_matrix(rng, F, K).astype(np.float64)
    o, oo = _opts("masked-ssim")
    r = _rasterizer(sz, F)
    go, terms, masks, med = _run(r, li, W.astype(np.float32), o)
    # medians and masks of every pixel (no SSIM, no CE: linear time)
    oo_plain = oracle.SlamLossOpts(**{**oo.__dict__, "ssim_lambda": 0.0, "w_sem": 0.0})
    _, tref, mref, medref = oracle.slam_loss(li.out, sz, li.rgb_t, li.depth_t, None, None, oo_plain)
    assert np.array_equal(med.view(np.uint32), medref.view(np.uint32))
    assert np.array_equal(masks, mref)
    assert terms[0] / (1.0 - np.float32(0.2)) == pytest.approx(tref[0], rel=1e-5)
    assert terms[2] == pytest.approx(tref[2], rel=1e-5)
    pts = [(0, 0), (0, 1199), (679, 0), (679, 1199), (0, 600), (679, 3), (340, 0), (5, 1194)]
    for v in range(8):
        qs = pts[:4] + [(int(rng.integers(0, 680)), int(rng.integers(0, 1200))) for _ in range(8)]
        for q in qs:
            gref, mk, p = _crop_ref(li, sz, v, q, med[v], W, oo, F)
            assert masks[p] == mk
            scale = max(np.abs(gref[:3]).max(), 1e-30)
            assert np.max(np.abs(go[:3, p] - gref[:3])) <= TOL_GRAD * scale, (v, q)
            assert np.array_equal(np.sign(go[3, p]), np.sign(gref[3]))
            assert np.max(np.abs(go[5:, p] - gref[5:])) <= 1e-5 * max(np.abs(gref[5:]).max(), 1e-30), (v, q)


DEC_CASES = [(8, 5, True, False), (16, 20, False, True), (16, 20, True, True), (32, 40, True, False),
             (16, 64, False, False), (32, 64, True, True), (16, 33, True, False)]


@pytest.mark.parametrize("F,K,bce,use_obs", DEC_CASES)
def test_slam_loss_decoder_gradients(F, K, bce, use_obs):
    """Learned decoder z = W^T f + b (bias on), CE or BCE (Eq. 16), with the
    decoder gradients dL/dW, dL/db (MFMA contraction over the pixels, fixed
    order sums) against the oracle; the rest of the loss as in mapping."""
    from paper_2603_27781_amd import _lib
    sz = SIZES["3views-ragged"]
    rng = np.random.default_rng(50 + F + K)
    li = wl.loss_images(rng, sz, F, K)
    W = wl.decoder_matrix(rng, F, K)
    b = (rng.normal(0, 0.3, K)).astype(np.float32)
    o, oo = _opts("masked-ssim" if use_obs else "mapping")
    if bce:
        o.flags |= _lib.GS_LOSS_BCE
        oo.bce = True
    r = _rasterizer(sz, F)
    r.slam_loss(_dev(li.rgb_t), _dev(li.depth_t), _dev(li.labels), _dev(W), o, out=_dev(li.out), bias=_dev(b),
                decoder_grads=True)
    torch.cuda.synchronize()
    go, terms = r.grad_out.cpu().numpy(), r.slam_terms.cpu().numpy()
    gw, gb = r.grad_decoder_w.cpu().numpy(), r.grad_decoder_b.cpu().numpy()
    gref, tref, mref, medref, gwr, gbr = oracle.slam_loss(li.out, sz, li.rgb_t, li.depth_t, li.labels,
                                                          W.astype(np.float64), oo, bias=b.astype(np.float64),
                                                          decoder_grads=True)
    assert np.array_equal(r.masks.cpu().numpy(), mref)
    assert rel_err(go[5:], gref[5:]) <= 1e-5, rel_err(go[5:], gref[5:])
    assert rel_err(go[:3], gref[:3]) <= TOL_GRAD
    assert terms[3] == pytest.approx(tref[3], rel=1e-5)
    assert rel_err(gw, gwr) <= 1e-5, rel_err(gw, gwr)
    assert rel_err(gb, gbr) <= 1e-5, rel_err(gb, gbr)
    # run-to-run identical (fixed-order sums)
    w0, b0 = r.grad_decoder_w.clone(), r.grad_decoder_b.clone()
    r.slam_loss(_dev(li.rgb_t), _dev(li.depth_t), _dev(li.labels), _dev(W), o, out=_dev(li.out), bias=_dev(b),
                decoder_grads=True)
    torch.cuda.synchronize()
    assert torch.equal(r.grad_decoder_w, w0) and torch.equal(r.grad_decoder_b, b0)


def test_slam_loss_decoder_full_size():
    """Eight 1200x680 views, F = 16, 20 classes, BCE under M_obs, no SSIM:
    the decoder gradients (sums over 6.5 M pixels) and the semantic term
    against the full FP64 oracle."""
    from paper_2603_27781_amd import _lib
    F, K = 16, 20
    sz = [(1200, 680)] * 8
    rng = np.random.default_rng(79)
    li = wl.loss_images(rng, sz, F, K)
    W = wl.decoder_matrix(rng, F, K)
    b = (rng.normal(0, 0.3, K)).astype(np.float32)
    o, oo = _opts("tracking")
    o.flags |= _lib.GS_LOSS_BCE
    oo.bce = True
    r = _rasterizer(sz, F)
    r.slam_loss(_dev(li.rgb_t), _dev(li.depth_t), _dev(li.labels), _dev(W), o, out=_dev(li.out), bias=_dev(b),
                decoder_grads=True)
    torch.cuda.synchronize()
    gref, tref, mref, _, gwr, gbr = oracle.slam_loss(li.out, sz, li.rgb_t, li.depth_t, li.labels,
                                                     W.astype(np.float64), oo, bias=b.astype(np.float64),
                                                     decoder_grads=True)
    assert np.array_equal(r.masks.cpu().numpy(), mref)
    terms = r.slam_terms.cpu().numpy()
    assert terms[3] == pytest.approx(tref[3], rel=1e-5)
    assert rel_err(r.grad_decoder_w.cpu().numpy(), gwr) <= 1e-5
    assert rel_err(r.grad_decoder_b.cpu().numpy(), gbr) <= 1e-5
    go = r.grad_out.cpu().numpy()
    assert rel_err(go[5:], gref[5:]) <= 1e-5
