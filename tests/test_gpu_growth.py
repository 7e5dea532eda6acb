"""GPU parity of gs_expand (adaptive expansion, Sec. 3.3.1-3.3.2) and gs_dsr
(Eq. 12) against the FP64 oracle on seeded synthetic inputs.

  - expansion: candidate count, the device-side Gaussian count, the order of
    the new Gaussians and every copied value (colour, feature, rotation,
    opacity) exact; the unprojected mean within binary32 rounding of the
    inputs (1e-5 relative), log-scale within four binary32 ulps; a full capacity
    truncates and leaves the planes beyond it untouched;
  - DSR: the set counts exact (both sides hold the same binary32 samples),
    L_big, L_small, mu, sigma to 1e-10 relative (double sums in different
    orders), the accumulated gradient to 1e-6.
"""
import numpy as np
import pytest

import oracle
from paper_2603_27781_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _views(sizes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for (W, H) in sizes:
        xi = rng.normal(size=6) * np.array([0.3, 0.3, 0.3, 0.5, 0.5, 0.5])
        out.append(wl.make_view(W, H, float(rng.uniform(0.6, 1.2) * W), wl.se3_exp(xi)))
    return out


def _planes(cap, F, fill=-7.0):
    return {"mu": torch.full((3, cap), fill, device="cuda"), "log_scale": torch.full((3, cap), fill, device="cuda"),
            "quat": torch.full((4, cap), fill, device="cuda"), "logit": torch.full((cap,), fill, device="cuda"),
            "color": torch.full((3, cap), fill, device="cuda"), "feat": torch.full((max(F, 1), cap), fill, device="cuda")}


@pytest.mark.parametrize("sizes,F,frac,trunc", [
    ([(61, 37), (40, 52), (17, 9)], 16, 0.3, False),
    ([(61, 37), (40, 52), (17, 9)], 8, 0.3, True),
    ([(1, 1), (33, 17)], 0, 0.9, False),
    ([(1200, 680)] * 8, 16, 0.05, False),
])
def test_expand_parity(sizes, F, frac, trunc):
    from paper_2603_27781_amd import raster
    views = _views(sizes, 3)
    V = raster.Views(views, 16)
    P = V.total_pixels
    rng = np.random.default_rng(11)
    masks = ((rng.random(P) < frac).astype(np.uint8) << 1) | (rng.random(P) < 0.5).astype(np.uint8)
    dep = rng.uniform(0.3, 5.0, P).astype(np.float32)
    dep[rng.random(P) < 0.05] = 0.0
    rgb = rng.random((3, P)).astype(np.float32)
    fi = rng.normal(size=(max(F, 1), P)).astype(np.float32)
    n0 = 123
    cnt_ref, ref = oracle.expand(views, masks, rgb, dep, fi if F else None, n0, 10 ** 9, F)
    cap = n0 + (cnt_ref // 2 if trunc else cnt_ref) + (0 if trunc else 17)
    planes = _planes(cap, F)
    n_dev = torch.tensor([n0], dtype=torch.int64, device="cuda")
    cand = torch.zeros(1, dtype=torch.int64, device="cuda")
    raster.expand(V, _dev(masks), _dev(rgb), _dev(dep), _dev(fi) if F else None, planes, cap, n_dev, F, cand)
    torch.cuda.synchronize()
    assert int(cand.item()) == cnt_ref
    assert int(n_dev.item()) == min(n0 + cnt_ref, cap)
    hi = min(n0 + cnt_ref, cap)
    got = {k: v.cpu().numpy() for k, v in planes.items()}
    sl = slice(n0, hi)
    # untouched before n0 and after the last written column
    for k, v in got.items():
        assert np.all(v[..., :n0] == -7.0) and np.all(v[..., hi:] == -7.0), k
    mu_ref = ref["mu"][:, sl]
    assert np.max(np.abs(got["mu"][:, sl] - mu_ref)) <= 1e-5 * max(np.max(np.abs(mu_ref)), 1.0)
    # log(D*/fx) in binary32: a correctly rounded quotient and logf, within
    # four ulps of the value (|log s| ~ 5-9 here, so ~1e-6 absolute)
    lref = ref["log_scale"][:, sl]
    assert np.all(np.abs(got["log_scale"][:, sl] - lref) <= 4 * 2.0 ** -23 * np.abs(lref) + 1e-7)
    assert np.array_equal(got["quat"][:, sl], ref["quat"][:, sl].astype(np.float32))
    assert np.array_equal(got["logit"][sl], ref["logit"][sl].astype(np.float32))
    assert np.array_equal(got["color"][:, sl], ref["color"][:, sl].astype(np.float32))
    if F:
        assert np.array_equal(got["feat"][:F, sl], ref["feat"][:F, sl].astype(np.float32))


@pytest.mark.parametrize("n,outliers", [(1, False), (1000, True), (1_000_000, True)])
def test_dsr_parity(n, outliers):
    from paper_2603_27781_amd import raster
    rng = np.random.default_rng(17)
    ls = rng.normal(-4.5, 0.4, (3, n)).astype(np.float32)
    if outliers:
        k = max(n // 500, 3)
        ls[0, :k] = -1.0
        ls[2, -k:] = -9.0
    wb, wsm = float(np.float32(0.01)), float(np.float32(0.001))  # the weights as the device receives them
    ref, gref = oracle.dsr(ls, wb, wsm)
    g0 = rng.normal(0, 1e-3, (3, n)).astype(np.float32)  # the gradient is accumulated
    grad = _dev(g0)
    out = raster.dsr(_dev(ls), 0.01, 0.001, grad).cpu().numpy()
    torch.cuda.synchronize()
    assert out[5] == ref["n_big"] and out[6] == ref["n_small"]
    for i, k in enumerate(("L_big", "L_small", "loss", "mu", "sigma")):
        assert out[i] == pytest.approx(ref[k], rel=1e-10, abs=1e-300), k
    want = g0.astype(np.float64) + gref
    assert np.max(np.abs(grad.cpu().numpy() - want)) <= 1e-6 * max(np.max(np.abs(want)), 1e-12)
