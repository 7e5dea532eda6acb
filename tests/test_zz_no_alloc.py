"""gs_pose_grad_noalloc (the pose twist with the library's own scratch
instead of a caller workspace) against gs_pose_grad on the same inputs,
through the C ABI: the same kernels in the same fixed summation order, so the
twists must agree bit for bit.  Two calls in a row, the second on a smaller
input (fewer Gaussians and views), so that the scratch's leftover partials
of the first call cannot leak into the second; and a size beyond the
scratch is refused before anything is launched."""
import ctypes

import numpy as np
import pytest

from paper_2603_27781_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(scene, views, seed):
    from paper_2603_27781_amd import raster
    cfg = raster.Config(tile=16)
    V = raster.Views(views, cfg.tile)
    g = raster.Gaussians.from_numpy(scene)
    r = raster.Rasterizer(scene.n, scene.n_feat, V, cfg)
    r.ensure_capacity(g)
    r.forward(g)
    rng = np.random.default_rng(seed)
    go = torch.from_numpy((rng.normal(size=tuple(r.out.shape)) * 1e-2).astype(np.float32)).cuda()
    r.render_bwd_2d(g, go, 2)
    return r, g


def _both(r, g):
    from paper_2603_27781_amd import _lib
    L = _lib.load()
    r.pose_grad(g)
    torch.cuda.synchronize()
    ref = r.twist.clone()
    out = torch.full_like(r.twist, float("nan"))
    st = L.gs_pose_grad_noalloc(ctypes.byref(g.c()), r.views.host, r.views.dev_ptr(), r.views.n,
                                ctypes.byref(r.cc), r.touched.data_ptr(), r.grad2d.data_ptr(), out.data_ptr(),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.GS_OK, st
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_pose_grad_noalloc_equals_workspace_entry_point():
    # first call: 40 views, 3000 Gaussians (about 28 KB of partials)
    big = wl.tiny_scene(81, 3000, F=8, W=40, H=32, f=32.0)
    rng = np.random.default_rng(81)
    views = list(big.views)
    for _ in range(39):
        xi = rng.normal(size=6) * np.array([0.05, 0.05, 0.05, 0.2, 0.2, 0.1])
        views.append(wl.make_view(int(rng.integers(16, 41)), int(rng.integers(12, 33)),
                                  float(rng.uniform(20.0, 36.0)), wl.se3_exp(xi)))
    r1, g1 = _case(big.scene, views, 1)
    ref1, out1 = _both(r1, g1)
    assert np.isfinite(ref1).all() and np.abs(ref1).max() > 0
    assert np.array_equal(ref1.view(np.uint32), out1.view(np.uint32))
    # second call, smaller: one view, 300 Gaussians
    small = wl.tiny_scene(82, 300, F=16, W=36, H=28, f=30.0)
    r2, g2 = _case(small.scene, small.views, 2)
    ref2, out2 = _both(r2, g2)
    assert np.abs(ref2).max() > 0
    assert np.array_equal(ref2.view(np.uint32), out2.view(np.uint32))


def test_pose_grad_noalloc_refuses_sizes_beyond_its_scratch():
    from paper_2603_27781_amd import _lib
    L = _lib.load()
    small = wl.tiny_scene(83, 200, F=8, W=32, H=24, f=30.0)
    r, g = _case(small.scene, small.views, 3)
    gc = g.c()
    gc.n = 1 << 30  # gs_pose_grad_workspace(2^30, 1) is 24 MiB, beyond the scratch; refused on the host
    b = ctypes.c_size_t(0)
    assert L.gs_pose_grad_workspace(gc.n, 1, ctypes.byref(b)) == _lib.GS_OK
    assert b.value > _lib.GS_NOALLOC_SCRATCH_BYTES
    before = r.twist.clone()
    st = L.gs_pose_grad_noalloc(ctypes.byref(gc), r.views.host, r.views.dev_ptr(), 1, ctypes.byref(r.cc),
                                r.touched.data_ptr(), r.grad2d.data_ptr(), r.twist.data_ptr(),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.GS_ECAPACITY
    torch.cuda.synchronize()
    assert torch.equal(before, r.twist)
