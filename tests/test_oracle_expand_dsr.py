"""Pins of the oracle's map growth and scale regularisation (no GPU):
  - adaptive expansion (Sec. 3.3.1-3.3.2): every new mean, projected back
    through its view (a projection written here), lands on its pixel centre
    at the observed depth; scales are D*/fx, opacity 0.5, identity rotation,
    colour and features from the pixel; candidates are exactly the pixels
    with M_unobs and D* > 0, in (view, row, column) order; a full capacity
    truncates;
  - DSR (Eq. 12): thresholds and sets against numpy's mean and (population)
    standard deviation of the same binary32 samples, hand-made outliers on
    either side, the gradient against central differences, empty sets.
"""
import numpy as np
import pytest

import oracle
from paper_2603_27781_amd import workloads as wl


def _views():
    v1 = wl.make_view(23, 17, 20.0, wl.se3_exp(np.array([0.1, -0.2, 0.05, 0.03, 0.2, -0.1])))
    v2 = wl.make_view(11, 9, 14.0, wl.se3_exp(np.array([-0.3, 0.1, 0.2, -0.1, 0.05, 0.3])))
    return [v1, v2]


def test_expansion_unprojects_onto_pixel_centres():
    views = _views()
    rng = np.random.default_rng(3)
    P = sum(v.width * v.height for v in views)
    masks = (rng.random(P) < 0.3).astype(np.uint8) * 2 | (rng.random(P) < 0.5).astype(np.uint8)
    dep = rng.uniform(0.5, 4.0, P)
    dep[rng.random(P) < 0.1] = 0.0
    dep = np.float32(dep).astype(np.float64)
    rgb = rng.random((3, P))
    F = 4
    fi = rng.normal(size=(F, P))
    cand = np.flatnonzero(((masks >> 1) & 1).astype(bool) & (np.float32(dep) > 0))
    cap = 7 + len(cand)
    cnt, g = oracle.expand(views, masks, rgb, dep, fi, 7, cap, F)
    assert cnt == len(cand)
    off = np.cumsum([0] + [v.width * v.height for v in views])
    for j, p in enumerate(cand):
        i = 7 + j
        v = int(np.searchsorted(off, p, side="right") - 1)
        vw = views[v]
        q = p - off[v]
        y, x = divmod(q, vw.width)
        Rt = np.asarray(vw.Rt, np.float32).astype(np.float64)
        pc = Rt[:, :3] @ g["mu"][:, i] + Rt[:, 3]
        fx, fy, cx, cy = (float(np.float32(a)) for a in (vw.fx, vw.fy, vw.cx, vw.cy))
        # R is binary32, orthonormal to ~1e-7 only, and R^T stands in for its
        # inverse: the round trip is exact to that, far below any mistake's
        assert pc[2] == pytest.approx(dep[p], rel=1e-6)
        assert fx * pc[0] / pc[2] + cx == pytest.approx(x + 0.5, abs=1e-4)
        assert fy * pc[1] / pc[2] + cy == pytest.approx(y + 0.5, abs=1e-4)
        assert np.allclose(g["log_scale"][:, i], np.log(dep[p] / fx), rtol=0, atol=1e-14)
        assert g["logit"][i] == 0.0 and list(g["quat"][:, i]) == [1, 0, 0, 0]
        assert np.array_equal(g["color"][:, i], rgb[:, p]) and np.array_equal(g["feat"][:, i], fi[:, p])
    assert not g["mu"][:, :7].any()
    # a capacity that cuts the list keeps its first entries
    cnt2, g2 = oracle.expand(views, masks, rgb, dep, fi, 7, 10, F)
    assert cnt2 == cnt and np.array_equal(g2["mu"][:, 7:10], g["mu"][:, 7:10])


def _dec_exp(x):
    y = np.zeros_like(x, dtype=np.float32)
    oracle.lib().orc_dec_exp(oracle.ctypes.c_int(x.size), oracle._p(np.ascontiguousarray(x, np.float32)),
                             oracle._p(y))
    return y


def test_dsr_against_numpy():
    rng = np.random.default_rng(5)
    ls = rng.normal(-4.0, 0.4, (3, 5000)).astype(np.float32)
    ls[0, :12] = -1.5   # large outliers
    ls[1, :9] = -9.0    # small outliers
    out, _ = oracle.dsr(ls, 0.01, 0.001)
    s = _dec_exp(ls.reshape(-1)).astype(np.float64)
    # the decision-path exp is the exponential to a few ulps
    assert np.allclose(s, np.exp(ls.reshape(-1).astype(np.float64)), rtol=1e-6, atol=0)
    mu, sd = s.mean(), s.std()
    assert out["mu"] == pytest.approx(mu, rel=1e-12) and out["sigma"] == pytest.approx(sd, rel=1e-10)
    big, small = s > mu + 2 * sd, s < mu - 2 * sd
    assert out["n_big"] == big.sum() >= 12 and out["n_small"] == small.sum()
    assert out["L_big"] == pytest.approx(s[big].mean(), rel=1e-12)
    Ls = (-np.log(s[small])).mean() if small.any() else 0.0
    assert out["L_small"] == pytest.approx(Ls, rel=1e-12)
    assert out["loss"] == pytest.approx(0.01 * out["L_big"] + 0.001 * Ls, rel=1e-12)


def test_dsr_small_set_and_empty_sets():
    # log-normal scales are skewed to the right: mu - 2 sigma is often below
    # zero; a spread-out symmetric set in s has a small set
    s = np.float32(np.linspace(0.5, 1.5, 3000))
    s[:4] = 0.01
    ls = np.log(s).astype(np.float32).reshape(3, -1)
    out, g = oracle.dsr(ls, 0.01, 0.001)
    assert out["n_small"] >= 4
    assert np.all(g.reshape(-1)[:4] == pytest.approx(-0.001 / out["n_small"]))
    same = np.full((3, 10), -3.0, np.float32)  # sigma = 0: both sets empty
    out0, g0 = oracle.dsr(same)
    assert out0["n_big"] == 0 and out0["n_small"] == 0 and out0["loss"] == 0.0 and not g0.any()


def test_dsr_gradient_finite_differences():
    """With the sets held (central differences small enough not to move an
    element across a threshold), d loss / d log s of the oracle."""
    rng = np.random.default_rng(9)
    ls = rng.normal(-4.0, 0.5, (3, 400)).astype(np.float32)
    ls[0, :3] = -2.0
    out, g = oracle.dsr(ls, 0.01, 0.001)
    s = _dec_exp(ls.reshape(-1)).astype(np.float64)
    big, small = s > out["mu"] + 2 * out["sigma"], s < out["mu"] - 2 * out["sigma"]
    nb, ns = big.sum(), small.sum()

    def loss(x):  # Eq. (12) with the sets and counts held, in FP64
        e = np.exp(x)
        return 0.01 * (e[big].sum() / max(nb, 1)) + 0.001 * ((-x[small]).sum() / max(ns, 1))

    x0 = np.log(s)
    h = 1e-6
    for j in list(np.flatnonzero(big)[:3]) + list(np.flatnonzero(small)[:3]) + [5, 77]:
        xp, xm = x0.copy(), x0.copy()
        xp[j] += h
        xm[j] -= h
        assert (loss(xp) - loss(xm)) / (2 * h) == pytest.approx(g.reshape(-1)[j], rel=1e-6, abs=1e-12), j
