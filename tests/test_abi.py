"""The C-ABI library loads and exports every symbol include/sgs.h declares;
host-only helpers and argument validation (no GPU needed: nothing launches)."""
import ctypes
import os
import re

import pytest

from paper_2603_27781_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sgs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", src)))


def test_header_declarations_are_exported():
    L = _lib.load()
    decl = _declared()
    assert len(decl) >= 14
    assert sorted(_lib.EXPORTS) == decl
    for name in decl:
        assert hasattr(L, name), name


def test_struct_sizes_match_header():
    assert ctypes.sizeof(_lib.GsView) == 88
    assert ctypes.sizeof(_lib.GsConfig) == 40
    assert ctypes.sizeof(_lib.GsGaussians) == 56


def test_default_config_and_layout():
    L = _lib.load()
    c = _lib.GsConfig()
    assert L.gs_default_config(ctypes.byref(c)) == 0
    assert (c.tile, c.lds_batch, c.persistent, c.lds_batch_bwd) == (16, 256, 0, 0)
    assert c.alpha_min == pytest.approx(1 / 255) and c.T_min == pytest.approx(1e-4)
    V = (_lib.GsView * 3)()
    for i, (w, h) in enumerate([(1200, 680), (640, 480), (33, 17)]):
        V[i].width, V[i].height, V[i].fx, V[i].fy = w, h, 500.0, 500.0
    tp, tt = ctypes.c_int64(), ctypes.c_int32()
    assert L.gs_views_layout(V, 3, 16, ctypes.byref(tp), ctypes.byref(tt)) == 0
    assert [V[i].pixel_offset for i in range(3)] == [0, 816000, 816000 + 307200]
    assert [V[i].tile_offset for i in range(3)] == [0, 75 * 43, 75 * 43 + 40 * 30]
    assert tt.value == 75 * 43 + 40 * 30 + 3 * 2 and tp.value == 816000 + 307200 + 33 * 17
    assert L.gs_views_layout(V, 3, 12, ctypes.byref(tp), ctypes.byref(tt)) == _lib.GS_EINVAL
    assert [L.gs_app_stride(f) for f in (0, 8, 16, 32)] == [4, 12, 20, 36]


def test_workspace_queries():
    L = _lib.load()
    b = ctypes.c_size_t()
    b2 = ctypes.c_size_t()
    assert L.gs_render_bwd_workspace(1000, 16, 2, 5000, 1, ctypes.byref(b), ctypes.byref(b2)) == 0
    assert b.value == (2 * 1000 * 8 + 1000 * 20) * 4 and b2.value == 5000 * 28 * 4
    assert L.gs_render_bwd_workspace(1000, 16, 2, 5000, 2, ctypes.byref(b), ctypes.byref(b2)) == 0
    assert b2.value == 5000 * 8 * 4
    assert L.gs_render_bwd_workspace(1000, 12, 2, 5000, 1, ctypes.byref(b), ctypes.byref(b2)) == _lib.GS_EUNSUPPORTED
    assert L.gs_bin_sort_workspace(1000, 2, 5000, ctypes.byref(b)) == 0 and b.value > 5 * 2000 * 4
    assert L.gs_bin_sort_workspace(0, 2, 5000, ctypes.byref(b)) == _lib.GS_EINVAL
    # per-block FP64 partials (6 per view), a block per 2048 Gaussians
    assert L.gs_pose_grad_workspace(1000, 2, ctypes.byref(b)) == 0 and b.value == 1 * 2 * 6 * 8
    assert L.gs_pose_grad_workspace(5000, 3, ctypes.byref(b)) == 0 and b.value == 3 * 3 * 6 * 8


def test_validation_rejects_before_any_launch():
    """Invalid arguments are rejected on the host; the dummy pointers below
    are never dereferenced (no GPU is touched)."""
    L = _lib.load()
    cfg = _lib.GsConfig()
    L.gs_default_config(ctypes.byref(cfg))
    V = (_lib.GsView * 1)()
    V[0].width, V[0].height, V[0].fx, V[0].fy = 64, 64, 64.0, 64.0
    L.gs_views_layout(V, 1, 16, None, None)
    dummy = 1 << 20
    g = _lib.GsGaussians(dummy, dummy, dummy, dummy, dummy, dummy, 100, 16)
    bad = _lib.GsConfig.from_buffer_copy(cfg)
    bad.tile = 12
    assert L.gs_project(ctypes.byref(g), V, dummy, 1, ctypes.byref(bad), dummy, dummy, dummy, dummy,
                        None) == _lib.GS_EUNSUPPORTED
    g12 = _lib.GsGaussians(dummy, dummy, dummy, dummy, dummy, dummy, 100, 12)
    assert L.gs_project(ctypes.byref(g12), V, dummy, 1, ctypes.byref(cfg), dummy, dummy, dummy, dummy,
                        None) == _lib.GS_EUNSUPPORTED
    assert L.gs_project(ctypes.byref(g), V, dummy, 1, ctypes.byref(cfg), None, dummy, dummy, dummy,
                        None) == _lib.GS_EINVAL
    assert L.gs_project(ctypes.byref(g), V, None, 1, ctypes.byref(cfg), dummy, dummy, dummy, dummy,
                        None) == _lib.GS_EINVAL
    V[0].pixel_offset = 7  # not the back-to-back layout
    assert L.gs_project(ctypes.byref(g), V, dummy, 1, ctypes.byref(cfg), dummy, dummy, dummy, dummy,
                        None) == _lib.GS_EINVAL
    L.gs_views_layout(V, 1, 16, None, None)
    assert L.gs_render_bwd(ctypes.byref(g), dummy, dummy, dummy, dummy, dummy, dummy, 100, dummy, V, dummy, 1,
                           ctypes.byref(cfg), dummy, dummy, dummy, 0, dummy, 1 << 30, dummy, 1 << 30, dummy,
                           None) == _lib.GS_EINVAL
    assert L.gs_render_bwd(ctypes.byref(g), dummy, dummy, dummy, dummy, dummy, dummy, 100, dummy, V, dummy, 1,
                           ctypes.byref(cfg), dummy, dummy, dummy, 1, dummy, 16, dummy, 1 << 30, dummy,
                           None) == _lib.GS_ECAPACITY
    assert L.gs_render_bwd(ctypes.byref(g), dummy, dummy, dummy, dummy, dummy, dummy, 100, dummy, V, dummy, 1,
                           ctypes.byref(cfg), dummy, dummy, dummy, 1, dummy, 1 << 30, dummy, 16, dummy,
                           None) == _lib.GS_ECAPACITY
    assert L.gs_project_bwd(ctypes.byref(g), V, dummy, 1, ctypes.byref(cfg), dummy, dummy, 1 << 30, None,
                            None) == _lib.GS_EINVAL
    assert L.gs_project_bwd_write(ctypes.byref(g), V, dummy, 1, ctypes.byref(cfg), dummy, dummy, 1 << 30, None,
                                  None) == _lib.GS_EINVAL
    # the two halves of gs_render_bwd validate on their own
    assert L.gs_render_bwd_records(ctypes.byref(g), dummy, dummy, dummy, dummy, 100, dummy, V, dummy, 1,
                                   ctypes.byref(cfg), dummy, dummy, dummy, 4, dummy, 1 << 30, dummy,
                                   None) == _lib.GS_EINVAL
    assert L.gs_render_bwd_records(ctypes.byref(g), dummy, dummy, dummy, dummy, 100, dummy, V, dummy, 1,
                                   ctypes.byref(cfg), dummy, dummy, dummy, 1, dummy, 16, dummy,
                                   None) == _lib.GS_ECAPACITY
    assert L.gs_reduce_records(None, 1 << 30, dummy, dummy, 100, 16, 1, 100, 1, dummy, 1 << 30,
                               None) == _lib.GS_EINVAL
    assert L.gs_reduce_records(dummy, 1 << 30, dummy, dummy, 100, 16, 1, 100, 1, dummy, 16,
                               None) == _lib.GS_ECAPACITY
    assert L.gs_reduce_records(dummy, 1 << 30, dummy, dummy, 100, 12, 1, 100, 1, dummy, 1 << 30,
                               None) == _lib.GS_EUNSUPPORTED
    assert L.gs_error_string(_lib.GS_ECAPACITY) == b"buffer too small"
    assert L.gs_version() >= 100


def test_slam_loss_host_side():
    """Defaults, workspace sizes and argument checks of gs_slam_loss (host
    only; every rejected call returns before any launch)."""
    L = _lib.load()
    o = _lib.GsSlamLossOpts()
    assert L.gs_default_slam_loss_opts(ctypes.byref(o)) == 0
    assert (o.w_color, o.w_depth, o.ssim_lambda, o.obs_factor, o.unobs_factor, o.flags) == \
        (0.5, 1.0, pytest.approx(0.2), 10.0, 50.0, 0)
    assert o.w_sem == pytest.approx(0.01) and o.tau_obs == pytest.approx(0.99) and o.tau_unobs == 0.5
    V = (_lib.GsView * 2)()
    for i, (w, h) in enumerate([(100, 60), (33, 17)]):
        V[i].width, V[i].height, V[i].fx, V[i].fy = w, h, 50.0, 50.0
    L.gs_views_layout(V, 2, 16, None, None)
    b0, b1, b2 = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    dummy = 1 << 20
    dec = _lib.GsDecoder(dummy, None, None, None, 20, 0)
    nossim = _lib.GsSlamLossOpts.from_buffer_copy(o)
    nossim.ssim_lambda = 0.0
    assert L.gs_slam_loss_workspace(V, 2, 16, ctypes.byref(dec), ctypes.byref(nossim), ctypes.byref(b0)) == 0
    assert L.gs_slam_loss_workspace(V, 2, 16, ctypes.byref(dec), ctypes.byref(o), ctypes.byref(b1)) == 0
    P = 100 * 60 + 33 * 17
    assert b0.value >= P and b1.value >= b0.value + 9 * 4 * P  # the SSIM maps
    dg = _lib.GsDecoder(dummy, None, dummy, dummy, 20, 0)
    assert L.gs_slam_loss_workspace(V, 2, 16, ctypes.byref(dg), ctypes.byref(o), ctypes.byref(b2)) == 0
    assert b2.value >= b1.value + ((P + 255) // 256) * (16 * 20 + 20) * 4  # decoder-gradient partials
    assert L.gs_slam_loss_workspace(V, 0, 16, ctypes.byref(dec), ctypes.byref(o), ctypes.byref(b1)) == _lib.GS_EINVAL
    big = _lib.GsDecoder(dummy, None, None, None, 65, 0)
    assert L.gs_slam_loss_workspace(V, 2, 16, ctypes.byref(big), ctypes.byref(o), ctypes.byref(b1)) == \
        _lib.GS_EUNSUPPORTED
    L.gs_slam_loss_workspace(V, 2, 16, ctypes.byref(dec), ctypes.byref(o), ctypes.byref(b1))
    ws = 1 << 24  # 256-byte aligned

    def call(opts=o, n_feat=16, ws_ptr=ws, ws_bytes=1 << 30, out=dummy, d=dec, labels=dummy):
        return L.gs_slam_loss(out, n_feat, dummy, dummy, labels, ctypes.byref(d) if d is not None else None,
                              ctypes.byref(opts), V, dummy, 2, dummy, dummy, None, None, ws_ptr, ws_bytes, None)

    assert call(n_feat=12) == _lib.GS_EUNSUPPORTED
    assert call(out=None) == _lib.GS_EINVAL
    assert call(labels=None) == _lib.GS_EINVAL
    assert call(d=_lib.GsDecoder(None, None, None, None, 20, 0)) == _lib.GS_EINVAL
    assert call(d=big) == _lib.GS_EUNSUPPORTED
    assert call(ws_ptr=ws + 16) == _lib.GS_EINVAL
    assert call(ws_bytes=b0.value) == _lib.GS_ECAPACITY  # SSIM on: needs the larger size
    assert call(d=dg, ws_bytes=b1.value) == _lib.GS_ECAPACITY  # decoder gradients need their partials
    bad = _lib.GsSlamLossOpts.from_buffer_copy(o)
    bad.flags = 4
    assert call(opts=bad) == _lib.GS_EINVAL


def test_views_check_rejects_before_any_launch():
    """gs_views_check refuses null pointers, view counts outside [1, 64],
    unsupported tiles and host arrays not laid out back to back, on the host
    (the dummy device pointers are never dereferenced)."""
    L = _lib.load()
    V = (_lib.GsView * 2)()
    for i in range(2):
        V[i].width, V[i].height, V[i].fx, V[i].fy = 40, 30, 50.0, 50.0
    assert L.gs_views_layout(V, 2, 16, None, None) == 0
    dummy = 1 << 20
    assert L.gs_views_check(V, None, 2, 16, dummy, None) == _lib.GS_EINVAL
    assert L.gs_views_check(V, dummy, 2, 16, None, None) == _lib.GS_EINVAL
    assert L.gs_views_check(V, dummy, 0, 16, dummy, None) == _lib.GS_EINVAL
    assert L.gs_views_check(V, dummy, 65, 16, dummy, None) == _lib.GS_EINVAL
    assert L.gs_views_check(V, dummy, 2, 12, dummy, None) == _lib.GS_EINVAL
    V[1].tile_offset += 1
    assert L.gs_views_check(V, dummy, 2, 16, dummy, None) == _lib.GS_EINVAL


def test_render_fwd_loss_workspace_and_refusals():
    """gs_render_fwd_loss: the workspace query (per-tile partials, their
    stage sums, the transposed decoder), and the host-side refusals made
    before anything launches: more than 16 feature channels or 20 classes
    (GS_EUNSUPPORTED: the caller makes the two separate calls), a short or
    misaligned workspace, null targets (the dummy device pointers are never
    dereferenced)."""
    L = _lib.load()
    V = (_lib.GsView * 2)()
    for i, (w, h) in enumerate([(40, 30), (33, 17)]):
        V[i].width, V[i].height, V[i].fx, V[i].fy = w, h, 50.0, 50.0
    assert L.gs_views_layout(V, 2, 16, None, None) == 0
    tiles = 3 * 2 + 3 * 2
    b = ctypes.c_size_t()
    assert L.gs_render_fwd_loss_workspace(V, 2, 16, ctypes.byref(b)) == 0
    r256 = lambda x: (x + 255) // 256 * 256
    assert b.value == r256(tiles * 3 * 8) + r256(1 * 3 * 8) + 16 * 20 * 4
    assert L.gs_render_fwd_loss_workspace(V, 2, 12, ctypes.byref(b)) == _lib.GS_EINVAL
    assert L.gs_render_fwd_loss_workspace(V, 0, 16, ctypes.byref(b)) == _lib.GS_EINVAL
    assert L.gs_render_fwd_loss_workspace(V, 2, 16, None) == _lib.GS_EINVAL
    L.gs_render_fwd_loss_workspace(V, 2, 16, ctypes.byref(b))
    cfg = _lib.GsConfig()
    L.gs_default_config(ctypes.byref(cfg))
    d = 1 << 20
    w = (ctypes.c_float * 3)(0.5, 1.0, 0.01)

    def call(F=16, K=20, ws=d, ws_bytes=b.value, rgb=d):
        return L.gs_render_fwd_loss(d, d, 100, F, d, d, d, V, d, 2, ctypes.byref(cfg), d, d, d, d, rgb, d, d, d, K,
                                    w, d, d, ws, ws_bytes, None)

    assert call(F=32, K=20) == _lib.GS_EUNSUPPORTED
    assert call(F=16, K=21) == _lib.GS_EUNSUPPORTED
    assert call(F=12) == _lib.GS_EUNSUPPORTED
    assert call(ws_bytes=b.value - 1) == _lib.GS_ECAPACITY
    assert call(ws=d + 8) == _lib.GS_EINVAL
    assert call(rgb=None) == _lib.GS_EINVAL
