"""Pins of the oracle's SLAM-loss extensions (no GPU).

What is pinned, and against what:
  - the median depth error (Eq. 11 / 21's median of the L1 depth error):
    a brute-force sort of the binary32 residuals;
  - the masks M_obs (Eq. 21) and M_unobs (Eq. 11): hand-built pixels on
    either side of every threshold;
  - the SSIM map of Eq. (15) (Wang et al. 2004, 11x11 Gaussian window of
    standard deviation 1.5, zero padding): closed forms for identical
    images, constant images (inside and at a corner, where only part of
    the window lies on the image) and a point impulse on a constant field,
    which exercises the means, variances and covariance;
  - the loss gradient: central finite differences of the oracle's own
    FP64 loss (colour with the SSIM term, depth, semantic, under M_obs);
  - special cases: lambda = 0 without a mask is the plain loss (itself
    pinned in test_oracle_pins.py); an empty mask gives zero.
"""
import math

import numpy as np
import pytest

import oracle

C1 = 0.01 ** 2
C2 = 0.03 ** 2


def gauss1d():
    g = np.array([math.exp(-((k - 5) ** 2) / (2 * 1.5 ** 2)) for k in range(11)])
    return g / g.sum()


# --------------------------------------------------------------------------
# median depth error
# --------------------------------------------------------------------------
def brute_median(d, t):
    d32, t32 = np.float32(d), np.float32(t)
    valid = t32 > 0
    r = np.abs(d32[valid] - t32[valid])  # binary32 subtraction, as the oracle
    if r.size == 0:
        return np.float32(0)
    return np.sort(r)[(r.size - 1) // 2]


@pytest.mark.parametrize("n", [1, 2, 7, 64, 1001])
def test_median_matches_sort(n):
    rng = np.random.default_rng(n)
    d = rng.uniform(0.5, 4.0, n).astype(np.float32)
    t = (d + rng.normal(0, 0.05, n)).astype(np.float32)
    t[rng.random(n) < 0.2] = 0.0  # missing depth
    if n > 10:
        t[:5] = d[:5] + 0.25  # ties
    assert oracle.depth_median(d, t) == brute_median(d, t)


def test_median_empty_and_even():
    assert oracle.depth_median(np.ones(5), np.zeros(5)) == 0.0
    assert oracle.depth_median(np.float32([1, 1, 1, 1]), np.float32([2, 4, 1.5, 1.25])) == np.float32(0.5)


# --------------------------------------------------------------------------
# masks
# --------------------------------------------------------------------------
def test_masks_at_thresholds():
    # one view of 10 pixels with median residual exactly 1: residuals
    # 1,1,1,1,1,1 (six), then the probes
    D_t = np.full(10, 2.0)
    r = np.array([1, 1, 1, 1, 1, 1, 9.5, 10.0, 50.0, 60.0])
    sign = np.array([1, 1, 1, 1, 1, 1, 1, 1, 1, 1.0])
    sign[9] = -1.0  # rendered depth in front of the observed: never "unobserved" by depth
    D = D_t + sign * r
    O = np.full(10, 0.995)
    O[0] = 0.99   # not > tau_obs (0.99 as binary32 both sides)
    O[1] = 0.4    # < tau_unobs
    F = 0
    out = np.zeros((5 + F, 10))
    out[3] = D
    out[4] = O
    rgb = np.zeros((3, 10))
    _, _, m, med = oracle.slam_loss(out, [(10, 1)], rgb, D_t)
    assert med[0] == 1.0
    obs = m & 1
    unobs = m >> 1
    assert list(obs) == [0, 0, 1, 1, 1, 1, 1, 0, 0, 0]
    assert list(unobs) == [0, 1, 0, 0, 0, 0, 0, 0, 0, 0]
    # residual just above 50 medians, behind the observed depth
    out[3, 8] = 2.0 + 50.5
    _, _, m, _ = oracle.slam_loss(out, [(10, 1)], rgb, D_t)
    assert (m[8] >> 1) == 1


# --------------------------------------------------------------------------
# SSIM closed forms
# --------------------------------------------------------------------------
def test_ssim_identical_is_one():
    rng = np.random.default_rng(1)
    x = rng.random((17, 23))
    assert np.allclose(oracle.ssim_map(x, x), 1.0, atol=1e-14, rtol=0)


def test_ssim_constant_images():
    a, b = 0.3, 0.7
    H, W = 16, 18
    s = oracle.ssim_map(np.full((H, W), a), np.full((H, W), b))
    inner = s[5:H - 5, 5:W - 5]
    assert np.allclose(inner, (2 * a * b + C1) / (a * a + b * b + C1), rtol=1e-12, atol=0)
    # corner: window mass m = (sum of the 1-D weights at offsets 0..5)^2
    m = gauss1d()[5:].sum() ** 2
    mx, my = a * m, b * m
    vx, vy, cxy = a * a * m - mx * mx, b * b * m - my * my, a * b * m - mx * my
    want = (2 * mx * my + C1) * (2 * cxy + C2) / ((mx * mx + my * my + C1) * (vx + vy + C2))
    assert s[0, 0] == pytest.approx(want, rel=1e-12)
    assert s[H - 1, W - 1] == pytest.approx(want, rel=1e-12)


def test_ssim_impulse():
    a, b, dl, ka = 0.4, 0.55, 0.3, -0.2
    H, W = 31, 33
    q0 = (15, 16)
    x = np.full((H, W), a)
    y = np.full((H, W), b)
    x[q0] += dl
    y[q0] += ka
    s = oracle.ssim_map(x, y)
    g = gauss1d()
    for i in range(q0[0] - 7, q0[0] + 8):
        for j in range(q0[1] - 7, q0[1] + 8):
            di, dj = q0[0] - i, q0[1] - j
            w = g[di + 5] * g[dj + 5] if abs(di) <= 5 and abs(dj) <= 5 else 0.0
            mx, my = a + dl * w, b + ka * w
            v = w * (1 - w)
            want = (2 * mx * my + C1) * (2 * dl * ka * v + C2) / ((mx * mx + my * my + C1) * ((dl * dl + ka * ka) * v + C2))
            assert s[i, j] == pytest.approx(want, rel=1e-11, abs=1e-13), (i, j)


def test_ssim_symmetric():
    rng = np.random.default_rng(5)
    x, y = rng.random((12, 15)), rng.random((12, 15))
    assert np.allclose(oracle.ssim_map(x, y), oracle.ssim_map(y, x), rtol=1e-13, atol=0)


# --------------------------------------------------------------------------
# the loss: reductions and gradient
# --------------------------------------------------------------------------
def _case(seed, wh, F=4, K=5):
    rng = np.random.default_rng(seed)
    P = sum(w * h for w, h in wh)
    out = np.zeros((5 + F, P))
    out[:3] = rng.random((3, P))
    out[3] = rng.uniform(1.0, 3.0, P)
    out[4] = rng.uniform(0.9, 1.0, P)
    out[5:] = rng.normal(0, 1, (F, P))
    rgb = np.clip(out[:3] + rng.normal(0, 0.1, (3, P)), 0, 1)
    dt = out[3] + rng.normal(0, 0.05, P)
    dt[rng.random(P) < 0.05] += 1.0  # a few outliers in depth
    lab = rng.integers(0, K, P).astype(np.int32)
    W = rng.normal(0, 0.5, (F, K))
    # exact binary32 values, as the device receives
    out, rgb, dt = (np.float32(a).astype(np.float64) for a in (out, rgb, dt))
    return out, rgb, dt, lab, W


def test_reduces_to_plain_loss():
    wh = [(9, 7), (5, 6)]
    out, rgb, dt, lab, W = _case(3, wh)
    o = oracle.SlamLossOpts(ssim_lambda=0.0, use_obs=False, w_sem=0.01)
    g, t, _, _ = oracle.slam_loss(out, wh, rgb, dt, lab, W, o)

    class V:
        def __init__(self, w, h):
            self.width, self.height = w, h

    w32 = tuple(float(np.float32(x)) for x in (0.5, 1.0, 0.01))  # the weights as the options pass them
    g0, t0 = oracle.loss(out, [V(*x) for x in wh], rgb, dt, lab, W, weights=w32)
    assert np.allclose(g, g0, rtol=1e-13, atol=0)
    assert t[0] == pytest.approx(t0[0], rel=1e-13) and t[1] == 0.0
    assert t[2] == pytest.approx(t0[1], rel=1e-13) and t[3] == pytest.approx(t0[2], rel=1e-13)


def test_empty_mask_gives_zero():
    wh = [(8, 8)]
    out, rgb, dt, lab, W = _case(4, wh)
    o = oracle.SlamLossOpts(tau_obs=2.0, use_obs=True)
    g, t, m, _ = oracle.slam_loss(out, wh, rgb, dt, lab, W, o)
    assert not (m & 1).any()
    assert np.all(g == 0) and np.all(t == 0)


def test_full_mask_equals_unmasked():
    wh = [(10, 9)]
    out, rgb, dt, lab, W = _case(6, wh)
    med = np.float32([1e30])  # every residual below 10 medians
    o = oracle.SlamLossOpts(tau_obs=-1.0, use_obs=True)
    g1, t1, m, _ = oracle.slam_loss(out, wh, rgb, dt, lab, W, o, medians=med)
    assert (m & 1).all()
    o.use_obs = False
    g2, t2, _, _ = oracle.slam_loss(out, wh, rgb, dt, lab, W, o, medians=med)
    assert np.array_equal(g1, g2) and np.array_equal(t1, t2)


@pytest.mark.parametrize("use_obs", [False, True])
def test_gradient_matches_finite_differences(use_obs):
    wh = [(13, 11), (7, 9)]
    out, rgb, dt, lab, W = _case(8 + use_obs, wh)
    o = oracle.SlamLossOpts(use_obs=use_obs, tau_obs=0.95, w_sem=0.05)
    _, _, _, med = oracle.slam_loss(out, wh, rgb, dt, lab, W, o)
    g, t, m, _ = oracle.slam_loss(out, wh, rgb, dt, lab, W, o, medians=med)
    if use_obs:
        assert 0 < (m & 1).sum() < m.size  # a real mask
    rng = np.random.default_rng(11)
    P = out.shape[1]
    h = 1e-6
    chans = [0, 1, 2, 3, 5, 6, 8]
    for _ in range(60):
        c = int(rng.choice(chans))
        p = int(rng.integers(0, P))
        up, dn = out.copy(), out.copy()
        up[c, p] += h
        dn[c, p] -= h
        lu = oracle.slam_loss(up, wh, rgb, dt, lab, W, o, medians=med)[1][4]
        ld = oracle.slam_loss(dn, wh, rgb, dt, lab, W, o, medians=med)[1][4]
        fd = (lu - ld) / (2 * h)
        assert fd == pytest.approx(g[c, p], rel=1e-5, abs=1e-9), (c, p)
    assert np.all(g[4] == 0)


def test_ssim_term_value():
    wh = [(12, 10)]
    out, rgb, dt, lab, W = _case(12, wh)
    o = oracle.SlamLossOpts(ssim_lambda=0.2, use_obs=False)
    _, t, _, _ = oracle.slam_loss(out, wh, rgb, dt, lab, W, o)
    s = sum(oracle.ssim_map(out[c].reshape(10, 12), rgb[c].reshape(10, 12)).sum() for c in range(3))
    want = 0.2 * np.float32(0.5) * (3 * 120 - s) / (3 * 120)
    assert t[1] == pytest.approx(want, rel=1e-12)


def test_crop_reproduces_full_view_gradient():
    """The full-size GPU check takes the oracle's gradient at a pixel q from
    the crop q +- 10 of its view (with the view's median and pixel count):
    every windowed sum that reaches q lies inside that crop, so the result
    equals the full view's."""
    from paper_2603_27781_amd import workloads as wl
    sz = [(47, 33)]
    li = wl.loss_images(np.random.default_rng(9), sz, 8, 6)
    W = wl.decoder_matrix(np.random.default_rng(10), 8, 6).astype(np.float64)
    o = oracle.SlamLossOpts(use_obs=True)
    gf, _, mf, med = oracle.slam_loss(li.out, sz, li.rgb_t, li.depth_t, li.labels, W, o)
    Wv, Hv = sz[0]
    for q in [(0, 0), (32, 46), (16, 23), (3, 40), (29, 10)]:
        r0, r1 = max(q[0] - 10, 0), min(q[0] + 11, Hv)
        c0, c1 = max(q[1] - 10, 0), min(q[1] + 11, Wv)
        idx = (np.arange(r0, r1)[:, None] * Wv + np.arange(c0, c1)[None, :]).reshape(-1)
        g, _, m, _ = oracle.slam_loss(li.out[:, idx].astype(np.float64), [(c1 - c0, r1 - r0)], li.rgb_t[:, idx],
                                      li.depth_t[idx], li.labels[idx], W, o, medians=med, norm_counts=[Wv * Hv])
        k = (q[0] - r0) * (c1 - c0) + (q[1] - c0)
        p = q[0] * Wv + q[1]
        assert m[k] == mf[p]
        assert np.allclose(g[:, k], gf[:, p], rtol=1e-12, atol=1e-18), q


# --------------------------------------------------------------------------
# learned decoder (z = W^T f + b), CE and BCE (Eq. 16), decoder gradients
# --------------------------------------------------------------------------
@pytest.mark.parametrize("bce", [False, True])
def test_semantic_term_and_decoder_grads_match_torch(bce):
    """The semantic term, its feature gradient and the decoder gradients
    against torch autograd through torch's own cross_entropy /
    binary_cross_entropy (FP64; binary_cross_entropy clamps its logs at -100
    as the reading does)."""
    torch = pytest.importorskip("torch")
    import torch.nn.functional as tf
    from paper_2603_27781_amd import workloads as wl
    sz = [(9, 7), (6, 5)]
    F, K = 8, 6
    li = wl.loss_images(np.random.default_rng(31), sz, F, K)
    rng = np.random.default_rng(32)
    W = rng.normal(0, 0.7, (F, K))
    b = rng.normal(0, 0.5, K)
    o = oracle.SlamLossOpts(ssim_lambda=0.0, w_color=0.0, w_depth=0.0, w_sem=0.3, bce=bce)
    g, t, _, _, gW, gb = oracle.slam_loss(li.out, sz, li.rgb_t, li.depth_t, li.labels, W, o, bias=b,
                                          decoder_grads=True)
    f = torch.tensor(li.out[5:].astype(np.float64).T, requires_grad=True)  # [P][F]
    Wt = torch.tensor(W, requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    lab = torch.tensor(li.labels.astype(np.int64))
    z = f @ Wt + bt
    per = (tf.cross_entropy(z, lab, reduction="none") if not bce else
           tf.binary_cross_entropy(torch.softmax(z, 1), tf.one_hot(lab, K).double(), reduction="none").sum(1))
    w = torch.cat([torch.full((w_ * h_,), float(np.float32(0.3)) / (w_ * h_), dtype=torch.float64) for w_, h_ in sz])
    loss = (w * per).sum()
    loss.backward()
    assert t[3] == pytest.approx(loss.item(), rel=1e-12)
    assert np.allclose(g[5:].T, f.grad.numpy(), rtol=1e-10, atol=1e-15)
    assert np.allclose(gW, Wt.grad.numpy(), rtol=1e-10, atol=1e-15)
    assert np.allclose(gb, bt.grad.numpy(), rtol=1e-10, atol=1e-15)


def test_bce_log_clamp():
    """A pixel whose softmax saturates: the clamped logs (at -100) give the
    torch value and no gradient through the clamped terms."""
    torch = pytest.importorskip("torch")
    import torch.nn.functional as tf
    F, K = 2, 3
    out = np.zeros((5 + F, 1))
    out[5:, 0] = [400.0, -400.0]
    W = np.array([[1.0, 0.0, -1.0], [0.0, 1.0, 0.0]])
    lab = np.array([2], np.int32)
    o = oracle.SlamLossOpts(ssim_lambda=0.0, w_color=0.0, w_depth=0.0, w_sem=1.0, bce=True)
    g, t, _, _, gW, gb = oracle.slam_loss(out, [(1, 1)], np.zeros((3, 1)), np.ones(1), lab, W, o, decoder_grads=True)
    z = torch.tensor(out[5:, 0]) @ torch.tensor(W)
    want = tf.binary_cross_entropy(torch.softmax(z, 0), tf.one_hot(torch.tensor(2), K).double(), reduction="sum")
    assert t[3] == pytest.approx(want.item(), rel=1e-12)
    assert np.all(np.isfinite(g)) and np.all(np.isfinite(gW)) and np.all(np.isfinite(gb))


@pytest.mark.parametrize("bce", [False, True])
def test_decoder_gradient_finite_differences(bce):
    """dL/dW and dL/db of the whole loss (SSIM colour, masks, semantic term)
    against central differences of the oracle's own FP64 loss."""
    from paper_2603_27781_amd import workloads as wl
    sz = [(11, 9), (7, 6)]
    F, K = 8, 5
    li = wl.loss_images(np.random.default_rng(41 + bce), sz, F, K)
    rng = np.random.default_rng(42)
    W = rng.normal(0, 0.6, (F, K))
    b = rng.normal(0, 0.4, K)
    o = oracle.SlamLossOpts(use_obs=True, tau_obs=0.95, w_sem=0.05, bce=bce)
    _, _, _, med = oracle.slam_loss(li.out, sz, li.rgb_t, li.depth_t, li.labels, W, o, bias=b)
    _, _, _, _, gW, gb = oracle.slam_loss(li.out, sz, li.rgb_t, li.depth_t, li.labels, W, o, medians=med, bias=b,
                                          decoder_grads=True)
    h = 1e-6

    def L(Wx, bx):
        return oracle.slam_loss(li.out, sz, li.rgb_t, li.depth_t, li.labels, Wx, o, medians=med, bias=bx)[1][4]

    for (i, k) in [(0, 0), (3, 2), (7, 4), (5, 1)]:
        Wp, Wm = W.copy(), W.copy()
        Wp[i, k] += h
        Wm[i, k] -= h
        assert (L(Wp, b) - L(Wm, b)) / (2 * h) == pytest.approx(gW[i, k], rel=1e-5, abs=1e-10), (i, k)
    for k in range(K):
        bp, bm = b.copy(), b.copy()
        bp[k] += h
        bm[k] -= h
        assert (L(W, bp) - L(W, bm)) / (2 * h) == pytest.approx(gb[k], rel=1e-5, abs=1e-10), k
