"""ctypes binding of libflod.so (argument marshalling only; see include/flod.h).

The library is built in-tree by paper_2408_12894_amd/build.py. Loading fails loudly when it
is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libflod.so")

FLOD_OK = 0
FLOD_ERR_INVALID_ARG = -1
FLOD_ERR_WORKSPACE = -2
FLOD_ERR_OVERFLOW = -3
FLOD_ERR_DEVICE = -4
FLOD_ERR_UNSUPPORTED = -5
FLOD_ERR_TOO_LARGE = -6
MAX_LEVELS = 8
NUM_STAGES = 9
STAGES = ("preprocess", "depth_sort", "offsets", "emit", "tile_sort", "ranges", "blend",
          "blend_bwd", "preprocess_bwd")

EXPORTS = ("flod_ctx_create", "flod_ctx_destroy", "flod_ctx_workspace_bytes", "flod_ctx_required_bytes",
           "flod_ctx_trim", "flod_render_level", "flod_render_selective", "flod_render_backward",
           "flod_ctx_stats", "flod_ctx_view", "flod_ctx_keep_backward_state", "flod_ctx_set_timing", "flod_ctx_set_timing_stages", "flod_ctx_stage_times",
           "flod_stage_name", "flod_smin", "flod_dproj", "flod_status_str", "flod_copy_to_host",
           "flod_render_merged", "flod_select_compact", "flod_overlap_prune", "flod_compact_level",
           "flod_level_transition", "flod_adam_step", "flod_l1_ssim_forward", "flod_l1_ssim_backward",
           "flod_l1_loss_forward", "flod_l1_loss_backward", "flod_l1_ssim_forward_noalloc")


class FlodError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})")


class Level(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("n", C.c_int64), ("s_min", C.c_float)]


class Camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("campos", C.c_float * 3),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32)]


class Frame(C.Structure):
    _fields_ = [("image", C.c_void_p), ("final_T", C.c_void_p), ("n_contrib", C.c_void_p),
                ("n_blended", C.c_void_p)]


class LevelState(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p)]


class AdamParams(C.Structure):
    _fields_ = [("lr_means", C.c_float), ("lr_log_scales", C.c_float), ("lr_quats", C.c_float),
                ("lr_opacity", C.c_float), ("lr_sh_dc", C.c_float), ("lr_sh_rest", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float), ("step", C.c_int64)]


class Grads(C.Structure):
    _fields_ = [("d_means", C.c_void_p), ("d_log_scales", C.c_void_p), ("d_quats", C.c_void_p),
                ("d_opacity_logits", C.c_void_p), ("d_sh", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("n_candidates", C.c_int64), ("n_visible", C.c_int64), ("n_instances", C.c_int64),
                ("tiles_x", C.c_int32), ("tiles_y", C.c_int32), ("width", C.c_int32), ("height", C.c_int32)]


class View(C.Structure):
    _fields_ = [("tile_ids", C.c_void_p), ("values", C.c_void_p), ("ranges", C.c_void_p),
                ("depth_bits", C.c_void_p), ("bin", C.c_void_p), ("tiles_touched", C.c_void_p),
                ("xy_conic", C.c_void_p), ("conic_c_opacity_rg", C.c_void_p), ("blue", C.c_void_p),
                ("grad2d", C.c_void_p), ("blended", C.c_void_p), ("tile_blended", C.c_void_p)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)

_lib = None


def load():
    """Load libflod.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libflod.so not found at {LIB_PATH}; run paper_2408_12894_amd/build.py "
                           "(there is no non-HIP fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, f32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_size_t
    L.flod_ctx_create.argtypes = [C.POINTER(vp), C.c_int, ALLOC_FN, FREE_FN, vp]
    L.flod_ctx_create.restype = C.c_int
    L.flod_ctx_destroy.argtypes = [vp]
    L.flod_ctx_destroy.restype = None
    L.flod_ctx_workspace_bytes.argtypes = [vp]
    L.flod_ctx_workspace_bytes.restype = sz
    L.flod_ctx_required_bytes.argtypes = [vp]
    L.flod_ctx_required_bytes.restype = sz
    L.flod_ctx_trim.argtypes = [vp, vp]
    L.flod_ctx_trim.restype = C.c_int
    L.flod_render_level.argtypes = [vp, C.POINTER(Level), C.c_int, C.POINTER(Camera), C.POINTER(C.c_float),
                                    C.POINTER(Frame), vp]
    L.flod_render_level.restype = C.c_int
    L.flod_render_selective.argtypes = [vp, C.POINTER(Level), C.c_int, C.c_int, C.c_int, C.POINTER(C.c_float),
                                        C.POINTER(C.c_float), C.c_int, C.POINTER(Camera), C.POINTER(C.c_float),
                                        C.POINTER(Frame), vp, vp]
    L.flod_render_selective.restype = C.c_int
    L.flod_render_merged.argtypes = [vp, C.POINTER(Level), C.c_int, C.c_int, C.POINTER(Camera),
                                     C.POINTER(C.c_float), C.POINTER(Frame), vp]
    L.flod_render_merged.restype = C.c_int
    L.flod_select_compact.argtypes = [vp, C.POINTER(Level), C.c_int, C.c_int, C.c_int, C.POINTER(C.c_float),
                                      C.POINTER(C.c_float), C.POINTER(Level), C.POINTER(C.c_int64), vp]
    L.flod_select_compact.restype = C.c_int
    L.flod_overlap_prune.argtypes = [vp, C.POINTER(Level), C.c_float, vp, vp, C.POINTER(C.c_int64), vp]
    L.flod_overlap_prune.restype = C.c_int
    L.flod_compact_level.argtypes = [vp, C.POINTER(Level), vp, C.POINTER(Level), C.POINTER(C.c_int64), vp]
    L.flod_compact_level.restype = C.c_int
    L.flod_level_transition.argtypes = [vp, C.POINTER(Level), C.c_float, C.POINTER(Level), vp]
    L.flod_level_transition.restype = C.c_int
    L.flod_adam_step.argtypes = [vp, C.POINTER(LevelState), C.POINTER(Grads), C.POINTER(LevelState),
                                 C.POINTER(LevelState), C.c_int64, C.POINTER(AdamParams), vp]
    L.flod_adam_step.restype = C.c_int
    ci = C.c_int
    L.flod_l1_ssim_forward.argtypes = [vp, vp, vp, ci, ci, ci, C.c_float, vp, vp, vp]
    L.flod_l1_ssim_forward.restype = C.c_int
    L.flod_l1_ssim_forward_noalloc.argtypes = [vp, vp, vp, ci, ci, ci, C.c_float, vp, vp, vp]
    L.flod_l1_ssim_forward_noalloc.restype = C.c_int
    L.flod_l1_ssim_backward.argtypes = [vp, vp, vp, ci, ci, ci, C.c_float, vp, vp, vp, vp]
    L.flod_l1_ssim_backward.restype = C.c_int
    L.flod_l1_loss_forward.argtypes = [vp, vp, vp, C.c_int64, vp, vp]
    L.flod_l1_loss_forward.restype = C.c_int
    L.flod_l1_loss_backward.argtypes = [vp, vp, vp, C.c_int64, vp, vp, vp]
    L.flod_l1_loss_backward.restype = C.c_int
    L.flod_render_backward.argtypes = [vp, vp, C.POINTER(Grads), vp]
    L.flod_render_backward.restype = C.c_int
    L.flod_ctx_stats.argtypes = [vp, C.POINTER(Stats)]
    L.flod_ctx_stats.restype = C.c_int
    L.flod_ctx_view.argtypes = [vp, C.POINTER(View)]
    L.flod_ctx_view.restype = C.c_int
    L.flod_ctx_keep_backward_state.argtypes = [vp, C.c_int]
    L.flod_ctx_keep_backward_state.restype = C.c_int
    L.flod_ctx_set_timing.argtypes = [vp, C.c_int]
    L.flod_ctx_set_timing.restype = C.c_int
    L.flod_ctx_set_timing_stages.argtypes = [vp, C.c_uint]
    L.flod_ctx_set_timing_stages.restype = C.c_int
    L.flod_ctx_stage_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int]
    L.flod_ctx_stage_times.restype = C.c_int
    L.flod_stage_name.argtypes = [C.c_int]
    L.flod_stage_name.restype = C.c_char_p
    L.flod_smin.argtypes = [C.c_int, C.c_int, f32, f32]
    L.flod_smin.restype = f32
    L.flod_dproj.argtypes = [f32, f32, f32]
    L.flod_dproj.restype = f32
    L.flod_status_str.argtypes = [C.c_int]
    L.flod_status_str.restype = C.c_char_p
    L.flod_copy_to_host.argtypes = [vp, vp, sz]
    L.flod_copy_to_host.restype = C.c_int
    _lib = L
    return L


def status_str(status: int) -> str:
    return load().flod_status_str(int(status)).decode()


def check(status: int, what: str) -> None:
    if status != FLOD_OK:
        raise FlodError(status, what)
