"""Pins of the oracle's optimiser steps (no GPU): Adam against
torch.optim.Adam (FP64, several steps), the SE(3) exponential against the
matrix exponential of the twist's 4x4 matrix (scipy.linalg.expm) including
the small-angle branch, and the pose step against its definition composed
from those two pinned pieces."""
import numpy as np
import pytest
import scipy.linalg

import oracle


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    p0 = rng.normal(size=50)
    p = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    mine, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        g = rng.normal(size=50)
        opt.zero_grad()
        p.grad = torch.tensor(g)
        opt.step()
        mine, m, v = oracle.adam(mine, g, m, v, 0.01, t)
        assert np.allclose(mine, p.detach().numpy(), rtol=1e-13, atol=1e-15), t


@pytest.mark.parametrize("scale", [1e-6, 1e-3, 0.3, 2.0])
def test_se3_exp_matches_expm(scale):
    rng = np.random.default_rng(int(scale * 1e6) % 1000)
    xi = rng.normal(size=6) * scale
    rho, phi = xi[:3], xi[3:]
    M = np.zeros((4, 4))
    M[:3, :3] = [[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]]
    M[:3, 3] = rho
    want = scipy.linalg.expm(M)[:3]
    assert np.allclose(oracle.se3_exp(xi), want, rtol=0, atol=1e-12 * max(1.0, scale))


def test_pose_step_is_adam_then_left_update():
    rng = np.random.default_rng(3)
    V = 3
    Rt = np.stack([oracle.se3_exp(rng.normal(size=6) * 0.5) for _ in range(V)])
    g = rng.normal(size=(V, 6))
    m = rng.normal(size=(V, 6)) * 0.1
    v = np.abs(rng.normal(size=(V, 6))) * 0.1
    R2, m2, v2 = oracle.pose_step(Rt, g, m, v, 0.002, 0.0004, 4)
    for w in range(V):
        x = np.zeros(6)
        mm, vv = m[w].copy(), v[w].copy()
        for k, lr in enumerate([0.002] * 3 + [0.0004] * 3):
            pk, mk, vk = oracle.adam(np.zeros(1), g[w, k:k + 1], mm[k:k + 1], vv[k:k + 1], lr, 4)
            x[k] = pk[0]
            assert mk[0] == pytest.approx(m2[w, k]) and vk[0] == pytest.approx(v2[w, k])
        E = np.vstack([oracle.se3_exp(x), [0, 0, 0, 1]])
        T = np.vstack([Rt[w], [0, 0, 0, 1]])
        assert np.allclose(R2[w], (E @ T)[:3], rtol=0, atol=1e-14)
