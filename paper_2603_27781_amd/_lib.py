"""ctypes binding of libsgs.so (the C ABI in include/sgs.h).

Argument marshalling only: every computation happens in the library's HIP
kernels.  Loading fails loudly when the library has not been built; there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgs.so")

c_int32, c_int64, c_float, c_double, c_void_p, c_size_t, c_uint32 = (
    ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t,
    ctypes.c_uint32)

GS_OK, GS_EINVAL, GS_ECAPACITY, GS_EHIP, GS_EUNSUPPORTED = 0, -1, -2, -3, -4
GS_GRAD_PARAMS, GS_GRAD_POSE = 1, 2

# symbols declared in include/sgs.h (checked by the ABI test)
EXPORTS = [
    "gs_default_config", "gs_views_layout", "gs_views_check", "gs_app_stride", "gs_project", "gs_bin_sort_workspace", "gs_bin_sort",
    "gs_render_fwd", "gs_render_fwd_loss_workspace", "gs_render_fwd_loss", "gs_loss_grad_workspace", "gs_loss_grad", "gs_render_bwd_workspace", "gs_render_bwd",
    "gs_render_bwd_records", "gs_reduce_records", "gs_project_bwd", "gs_project_bwd_write",
    "gs_pose_grad_workspace",
    "gs_pose_grad", "gs_default_slam_loss_opts", "gs_slam_loss_workspace", "gs_slam_loss", "gs_expand_workspace",
    "gs_expand", "gs_dsr_workspace", "gs_dsr", "gs_adam_step", "gs_pose_step", "gs_pose_step_dev", "gs_pose_grad_noalloc", "gs_error_string",
    "gs_last_hip_error", "gs_version",
]
GS_LOSS_OBS_MASK, GS_LOSS_BCE = 1, 2
GS_NOALLOC_SCRATCH_BYTES = 8 << 20
# gs_render_fwd_loss supports at most this many feature channels and classes
GS_FUSED_MAX_FEAT, GS_FUSED_MAX_CLASSES = 16, 20


class GsGaussians(ctypes.Structure):
    _fields_ = [("mu", c_void_p), ("log_scale", c_void_p), ("quat", c_void_p), ("opacity_logit", c_void_p),
                ("color", c_void_p), ("feat", c_void_p), ("n", c_int32), ("n_feat", c_int32)]


class GsGaussianGrads(ctypes.Structure):
    _fields_ = [("mu", c_void_p), ("log_scale", c_void_p), ("quat", c_void_p), ("opacity_logit", c_void_p),
                ("color", c_void_p), ("feat", c_void_p)]


class GsView(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("fx", c_float), ("fy", c_float), ("cx", c_float),
                ("cy", c_float), ("Rt", c_float * 12), ("pixel_offset", c_int64), ("tile_offset", c_int32),
                ("reserved", c_int32)]


class GsConfig(ctypes.Structure):
    _fields_ = [("z_near", c_float), ("blur", c_float), ("guard", c_float), ("alpha_min", c_float),
                ("alpha_max", c_float), ("T_min", c_float), ("tile", c_int32), ("lds_batch", c_int32),
                ("persistent", c_int32), ("lds_batch_bwd", c_int32)]


class GsSlamLossOpts(ctypes.Structure):
    _fields_ = [("w_color", c_float), ("w_depth", c_float), ("w_sem", c_float), ("ssim_lambda", c_float),
                ("tau_obs", c_float), ("tau_unobs", c_float), ("obs_factor", c_float), ("unobs_factor", c_float),
                ("flags", c_uint32)]


class GsAdamGroup(ctypes.Structure):
    _fields_ = [("param", c_void_p), ("grad", c_void_p), ("m", c_void_p), ("v", c_void_p), ("n", c_int64),
                ("lr", c_float), ("reserved", c_int32)]


class GsDecoder(ctypes.Structure):
    _fields_ = [("weight", c_void_p), ("bias", c_void_p), ("grad_weight", c_void_p), ("grad_bias", c_void_p),
                ("n_classes", c_int32), ("reserved", c_int32)]


assert ctypes.sizeof(GsView) == 88 and ctypes.sizeof(GsConfig) == 40 and ctypes.sizeof(GsSlamLossOpts) == 36
assert ctypes.sizeof(GsDecoder) == 40

_lib = None


class SgsError(RuntimeError):
    pass


def load() -> ctypes.CDLL:
    """Load libsgs.so; raise if it is missing (no CPU or PyTorch fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SgsError(f"{LIB_PATH} is not built: run `python -m paper_2603_27781_amd.build` "
                       "(the rasterizer has no fallback path)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    L.gs_default_config.argtypes = [P(GsConfig)]
    L.gs_views_layout.argtypes = [P(GsView), c_int32, c_int32, P(c_int64), P(c_int32)]
    L.gs_views_check.argtypes = [P(GsView), c_void_p, c_int32, c_int32, c_void_p, c_void_p]
    L.gs_app_stride.argtypes = [c_int32]
    L.gs_app_stride.restype = c_int32
    L.gs_project.argtypes = [P(GsGaussians), P(GsView), c_void_p, c_int32, P(GsConfig), c_void_p, c_void_p,
                             c_void_p, c_void_p, c_void_p]
    L.gs_bin_sort_workspace.argtypes = [c_int32, c_int32, c_int64, P(c_size_t)]
    L.gs_bin_sort.argtypes = [c_void_p, c_void_p, c_int32, P(GsView), c_void_p, c_int32, P(GsConfig),
                              c_void_p, c_size_t, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                              c_void_p, c_void_p]
    L.gs_render_fwd.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p, P(GsView),
                                c_void_p, c_int32, P(GsConfig), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.gs_render_fwd_loss_workspace.argtypes = [P(GsView), c_int32, c_int32, P(c_size_t)]
    L.gs_render_fwd_loss.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p, P(GsView),
                                     c_void_p, c_int32, P(GsConfig), c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p, c_void_p, c_void_p, c_int32, P(c_float), c_void_p,
                                     c_void_p, c_void_p, c_size_t, c_void_p]
    L.gs_loss_grad_workspace.argtypes = [c_int64, P(c_size_t)]
    L.gs_loss_grad.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, P(c_float),
                               P(GsView), c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    L.gs_render_bwd_workspace.argtypes = [c_int32, c_int32, c_int32, c_int64, c_uint32, P(c_size_t), P(c_size_t)]
    L.gs_render_bwd.argtypes = [P(GsGaussians), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int64,
                                c_void_p, P(GsView), c_void_p, c_int32, P(GsConfig), c_void_p, c_void_p, c_void_p,
                                c_uint32, c_void_p, c_size_t, c_void_p, c_size_t, c_void_p, c_void_p]
    L.gs_render_bwd_records.argtypes = [P(GsGaussians), c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_void_p,
                                        P(GsView), c_void_p, c_int32, P(GsConfig), c_void_p, c_void_p, c_void_p,
                                        c_uint32, c_void_p, c_size_t, c_void_p, c_void_p]
    L.gs_reduce_records.argtypes = [c_void_p, c_size_t, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int64,
                                    c_uint32, c_void_p, c_size_t, c_void_p]
    L.gs_project_bwd.argtypes = [P(GsGaussians), P(GsView), c_void_p, c_int32, P(GsConfig), c_void_p, c_void_p,
                                 c_size_t, P(GsGaussianGrads), c_void_p]
    L.gs_project_bwd_write.argtypes = L.gs_project_bwd.argtypes
    L.gs_pose_grad_workspace.argtypes = [c_int32, c_int32, P(c_size_t)]
    L.gs_pose_grad.argtypes = [P(GsGaussians), P(GsView), c_void_p, c_int32, P(GsConfig), c_void_p, c_void_p,
                               c_void_p, c_size_t, c_void_p, c_void_p]
    L.gs_pose_grad_noalloc.argtypes = [P(GsGaussians), P(GsView), c_void_p, c_int32, P(GsConfig), c_void_p,
                                       c_void_p, c_void_p, c_void_p]
    L.gs_default_slam_loss_opts.argtypes = [P(GsSlamLossOpts)]
    L.gs_slam_loss_workspace.argtypes = [P(GsView), c_int32, c_int32, P(GsDecoder), P(GsSlamLossOpts), P(c_size_t)]
    L.gs_slam_loss.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, P(GsDecoder), P(GsSlamLossOpts),
                               P(GsView), c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                               c_size_t, c_void_p]
    L.gs_expand_workspace.argtypes = [c_int64, P(c_size_t)]
    L.gs_expand.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, P(GsView), c_void_p, c_int32,
                            P(GsGaussianGrads), c_int64, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    L.gs_dsr_workspace.argtypes = [c_int64, P(c_size_t)]
    L.gs_dsr.argtypes = [c_void_p, c_int64, c_float, c_float, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    L.gs_adam_step.argtypes = [ctypes.c_void_p, c_int32, c_float, c_float, c_float, c_int32, c_void_p]
    L.gs_pose_step.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_float, c_float, c_float, c_float,
                               c_float, c_int32, c_void_p]
    L.gs_pose_step_dev.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_float, c_float, c_float,
                                   c_float, c_float, c_void_p, c_void_p]
    L.gs_error_string.argtypes = [ctypes.c_int]
    L.gs_error_string.restype = ctypes.c_char_p
    L.gs_last_hip_error.restype = ctypes.c_char_p
    L.gs_version.restype = c_int32
    _lib = L
    return L


def check(status: int, what: str) -> None:
    if status != GS_OK:
        L = load()
        msg = L.gs_error_string(status).decode()
        if status == GS_EHIP:
            msg += ": " + L.gs_last_hip_error().decode()
        raise SgsError(f"{what} failed ({status}: {msg})")
