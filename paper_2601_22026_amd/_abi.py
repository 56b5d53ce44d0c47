"""ctypes declarations of include/gsfit.h (argument marshalling only).

Every function of the C ABI is exposed under its C name.  Loading fails loudly
(``GsfError``) when libgsfit.so is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsfit.so")

GSF_OK, GSF_E_INVALID, GSF_E_CAPACITY, GSF_E_HIP, GSF_E_STATE, GSF_E_NONFINITE, GSF_E_UNSUPPORTED = range(7)
STATUS_NAMES = {0: "GSF_OK", 1: "GSF_E_INVALID", 2: "GSF_E_CAPACITY", 3: "GSF_E_HIP",
                4: "GSF_E_STATE", 5: "GSF_E_NONFINITE", 6: "GSF_E_UNSUPPORTED"}
GSF_FLAG_CAPACITY = 1
GSF_FLAG_NONFINITE = 2
(GSF_DBG_RECT, GSF_DBG_COUNT, GSF_DBG_DEPTH, GSF_DBG_KEYS, GSF_DBG_VALS, GSF_DBG_RANGES,
 GSF_DBG_TFINAL, GSF_DBG_NCONTRIB, GSF_DBG_G2D, GSF_DBG_PROJ, GSF_DBG_ORDER, GSF_DBG_BG,
 GSF_DBG_VIS) = range(13)

EXPORTED = ["gsf_ctx_create", "gsf_ctx_destroy", "gsf_ctx_set_stream", "gsf_last_error",
            "gsf_plan_create", "gsf_plan_workspace_bytes", "gsf_plan_bind_workspace",
            "gsf_plan_info", "gsf_plan_destroy", "gsf_forward", "gsf_loss_l1", "gsf_backward",
            "gsf_adam", "gsf_step", "gsf_step_capture", "gsf_step_replay", "gsf_poll",
            "gsf_debug_copy", "gsf_plan_set_timing", "gsf_plan_stage_times",
            "gsf_count_pairs", "gsf_loss_l1_rgba", "gsf_seed_scratch_bytes",
            "gsf_seed_volume", "gsf_raymarch", "gsf_adam_masked", "gsf_adam_reset",
            "gsf_view_select", "gsf_reproject", "gsf_reproject_warp",
            "gsf_first_hit_scratch_bytes", "gsf_seed_first_hits", "gsf_loss_count",
            "gsf_autotune_workspace_bytes", "gsf_autotune", "gsf_reproject_warp_noalloc"]
STAGES = ["project", "duplicate", "tile_sort", "ranges", "depth_sort", "render", "loss",
          "render_bwd", "project_bwd", "adam", "grad_sum"]


class GsfError(RuntimeError):
    def __init__(self, status: int, message: str = ""):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")


class gsf_camera(ct.Structure):
    _fields_ = [("viewmat", ct.c_float * 12), ("campos", ct.c_float * 3), ("fx", ct.c_float),
                ("fy", ct.c_float), ("cx", ct.c_float), ("cy", ct.c_float),
                ("tan_half_fov_x", ct.c_float), ("tan_half_fov_y", ct.c_float),
                ("znear", ct.c_float), ("bg", ct.c_float * 3), ("width", ct.c_int32),
                ("height", ct.c_int32), ("reserved", ct.c_int32 * 5)]


class gsf_plan_desc(ct.Structure):
    _fields_ = [("n_max", ct.c_int64), ("sh_degree", ct.c_int32), ("n_views", ct.c_int32),
                ("widths", ct.POINTER(ct.c_int32)), ("heights", ct.POINTER(ct.c_int32)),
                ("tile", ct.c_int32), ("lds_batch", ct.c_int32), ("t_mode", ct.c_int32),
                ("host_sized", ct.c_int32), ("key_capacity", ct.c_int64)]


class gsf_step_args(ct.Structure):
    _fields_ = [("params", ct.c_void_p), ("n", ct.c_int64), ("cams", ct.c_void_p),
                ("target_rgb", ct.c_void_p), ("gaze_px", ct.c_void_p),
                ("mask_radius_frac", ct.c_float), ("loss", ct.c_void_p), ("rgba", ct.c_void_p),
                ("dl_drgba", ct.c_void_p), ("grads", ct.c_void_p), ("adam_m", ct.c_void_p),
                ("adam_v", ct.c_void_p), ("step_dev", ct.c_void_p),
                ("seg_lr", ct.POINTER(ct.c_float)), ("beta1", ct.c_float), ("beta2", ct.c_float),
                ("eps", ct.c_float), ("fovea_cull", ct.c_int32), ("alpha_loss", ct.c_int32),
                ("random_bg", ct.c_int32), ("bg_seed", ct.c_uint64), ("masked_adam", ct.c_int32)]


class gsf_tune_space(ct.Structure):
    _fields_ = [("n_tiles", ct.c_int32), ("tiles", ct.c_int32 * 3),
                ("key_capacity", ct.c_int64 * 3), ("n_batches", ct.c_int32),
                ("batches", ct.c_int32 * 3), ("n_t_modes", ct.c_int32), ("t_modes", ct.c_int32 * 3),
                ("warmup", ct.c_int32), ("reps", ct.c_int32)]


class gsf_tune_result(ct.Structure):
    _fields_ = [("tile", ct.c_int32), ("lds_batch", ct.c_int32), ("t_mode", ct.c_int32),
                ("ms", ct.c_float * 27)]


assert ct.sizeof(gsf_camera) == 128
assert ct.sizeof(gsf_tune_space) == 80 and ct.sizeof(gsf_tune_result) == 120


def _declare(L):
    vp, i64, i32, f32 = ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_float
    pf = ct.POINTER(ct.c_float)
    pvp = ct.POINTER(ct.c_void_p)
    sig = {
        "gsf_ctx_create": [ct.c_int, vp, pvp],
        "gsf_ctx_destroy": [vp],
        "gsf_ctx_set_stream": [vp, vp],
        "gsf_plan_create": [vp, ct.POINTER(gsf_plan_desc), pvp],
        "gsf_plan_workspace_bytes": [vp, ct.POINTER(ct.c_size_t)],
        "gsf_plan_bind_workspace": [vp, vp, ct.c_size_t],
        "gsf_plan_info": [vp, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64)],
        "gsf_plan_destroy": [vp],
        "gsf_forward": [vp, vp, i64, vp, vp, f32, vp],
        "gsf_loss_l1": [vp, vp, vp, vp, f32, i64, i32, vp, vp],
        "gsf_loss_count": [vp, vp, f32, ct.POINTER(ct.c_int64)],
        "gsf_autotune_workspace_bytes": [vp, ct.POINTER(gsf_plan_desc), ct.POINTER(gsf_tune_space),
                                         ct.POINTER(ct.c_size_t)],
        "gsf_autotune": [vp, ct.POINTER(gsf_plan_desc), ct.POINTER(gsf_tune_space),
                         ct.POINTER(gsf_step_args), vp, ct.c_size_t, ct.POINTER(gsf_tune_result)],
        "gsf_loss_l1_rgba": [vp, vp, vp, vp, i32, vp, f32, vp, vp],
        "gsf_backward": [vp, vp, i64, vp, vp, i32, vp],
        "gsf_adam": [vp, vp, vp, vp, vp, i64, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_float), i32,
                     f32, f32, f32, vp],
        "gsf_adam_masked": [vp, vp, vp, vp, vp, i64, i32, ct.POINTER(ct.c_float), vp, f32, f32,
                            f32, vp],
        "gsf_adam_reset": [vp, vp, vp, i64, vp],
        "gsf_view_select": [ct.POINTER(gsf_camera), i32, ct.POINTER(gsf_camera), i32, f32, f32,
                            ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32)],
        "gsf_reproject": [vp, vp, i32, i32, pf, pf, pf, pf, pf, vp],
        "gsf_first_hit_scratch_bytes": [i64, ct.POINTER(ct.c_size_t)],
        "gsf_seed_first_hits": [vp, vp, i32, vp, i32, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32),
                                f32, f32, f32, f32, pf, pf, f32, i32, ct.c_double, i64, ct.c_uint64,
                                vp, vp, ct.POINTER(ct.c_int64), vp, ct.c_size_t],
        "gsf_reproject_warp": [vp, vp, vp, i32, i32, pf, pf, pf, pf, pf, i32, i32, vp, vp, vp],
        "gsf_reproject_warp_noalloc": [vp, vp, vp, i32, i32, pf, pf, pf, pf, pf, i32, i32, vp, vp],
        "gsf_step": [vp, ct.POINTER(gsf_step_args)],
        "gsf_step_capture": [vp, ct.POINTER(gsf_step_args)],
        "gsf_step_replay": [vp],
        "gsf_poll": [vp, ct.POINTER(ct.c_uint32), ct.POINTER(ct.c_int64)],
        "gsf_debug_copy": [vp, ct.c_int, vp, ct.c_size_t, ct.POINTER(ct.c_size_t)],
        "gsf_plan_set_timing": [vp, ct.c_int],
        "gsf_count_pairs": [vp, ct.POINTER(ct.c_int64)],
        "gsf_plan_stage_times": [vp, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64)],
        "gsf_seed_scratch_bytes": [i32, ct.POINTER(ct.c_size_t)],
        "gsf_seed_volume": [vp, vp, i32, ct.c_double, ct.c_double, ct.POINTER(ct.c_double),
                            ct.POINTER(ct.c_double), ct.c_double, i64, ct.c_uint64, vp,
                            ct.POINTER(ct.c_int64), vp, ct.c_size_t],
        "gsf_raymarch": [vp, vp, i32, vp, i32, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32), f32,
                         f32, f32, f32, f32, ct.POINTER(ct.c_float), ct.POINTER(ct.c_float), vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ct.c_int
    L.gsf_last_error.argtypes = [vp]
    L.gsf_last_error.restype = ct.c_char_p
    return L


_lib = None


def lib():
    """The loaded libgsfit.so (raises GsfError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GsfError(GSF_E_UNSUPPORTED,
                           f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2601_22026_amd.build` (no fallback exists)")
        _lib = _declare(ct.CDLL(LIB_PATH))
    return _lib
