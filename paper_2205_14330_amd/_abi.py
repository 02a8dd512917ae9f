"""ctypes mirror of include/dpr.h and the loader of libdpr.so.

There is no fallback: if the HIP library is missing or fails to load, every
entry point raises.  Build it with ``python -m paper_2205_14330_amd.build``.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpr.so")

c_f, c_i32, c_i64, c_p, c_sz = ctypes.c_float, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t

DPR_OK, DPR_ERR_INVALID_ARG, DPR_ERR_WORKSPACE, DPR_ERR_HIP, DPR_ERR_UNSUPPORTED, DPR_ERR_STATE = range(6)
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "WORKSPACE", 3: "HIP", 4: "UNSUPPORTED", 5: "STATE"}
FLAG_TIMING, FLAG_STATS, FLAG_PERSISTENT, FLAG_KERNEL_NORM = 1, 2, 4, 8
BWD_STORED, BWD_RECOMPUTE = 0, 1
STAGES = ["upload", "project", "depth_sort", "tile_count", "tile_scan", "emit", "composite_fwd",
          "recompute", "composite_bwd", "point_bwd"]

EXPORTED = ["dpr_version", "dpr_last_error", "dpr_plan_ws_bytes", "dpr_plan_forward",
            "dpr_workspace_bytes", "dpr_render_forward", "dpr_backward_ws_bytes",
            "dpr_render_backward", "dpr_plan_free", "dpr_plan_get_info", "dpr_stage_times",
            "dpr_render_forward_1", "dpr_loss_ws_bytes", "dpr_loss_l2_tv", "dpr_knn_ws_bytes", "dpr_knn",
            "dpr_hybrid_ws_bytes", "dpr_voxel_reduce", "dpr_hybrid_update", "dpr_hull_ws_bytes", "dpr_hull_sample",
            "dpr_consistency", "dpr_consistency_filter", "dpr_chamfer_ws_bytes", "dpr_chamfer", "dpr_topk_sh",
            "dpr_adam_step", "dpr_render_forward_1_noalloc", "dpr_plan_forward_render"]


class Camera(ctypes.Structure):
    _fields_ = [("R", c_f * 9), ("t", c_f * 3), ("fx", c_f), ("fy", c_f), ("cx", c_f), ("cy", c_f),
                ("width", c_i32), ("height", c_i32)]


class Mask(ctypes.Structure):
    _fields_ = [("data", c_p), ("width", c_i32), ("height", c_i32)]


class Scene(ctypes.Structure):
    _fields_ = [("n", c_i64), ("sh_degree", c_i32), ("reserved", c_i32), ("xyz", c_p), ("sh", c_p),
                ("opacity", c_p), ("radius", c_p)]


class View(ctypes.Structure):
    _fields_ = [("scene", c_i32), ("reserved", c_i32), ("cam", Camera), ("image", c_p), ("trans", c_p)]


class Params(ctypes.Structure):
    _fields_ = [("alpha_min", c_f), ("t_min", c_f), ("alpha_max", c_f), ("z_near", c_f),
                ("sh_frame", c_i32), ("bwd_mode", c_i32), ("flags", c_i32), ("max_splats", c_i32),
                ("timing_stages", c_i32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("items", c_i64), ("pairs", c_i64), ("tiles", c_i64), ("pixels", c_i64), ("chunks", c_i64),
                ("plan_ws_bytes", c_i64), ("fwd_ws_bytes", c_i64), ("bwd_ws_bytes", c_i64),
                ("rec_off", c_i64), ("key_off", c_i64), ("order_off", c_i64), ("rect_off", c_i64),
                ("range_off", c_i64), ("pairs_off", c_i64), ("nlast_off", c_i64), ("stats_off", c_i64),
                ("tile_size", c_i32), ("chunk_items", c_i32)]


class DprError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dpr error {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Loads libdpr.so; raises if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build the HIP library first "
                          f"(python -m paper_2205_14330_amd.build)")
    L = ctypes.CDLL(path)
    PP = ctypes.POINTER(c_p)
    L.dpr_version.argtypes, L.dpr_version.restype = [], c_i32
    L.dpr_last_error.argtypes, L.dpr_last_error.restype = [], ctypes.c_char_p
    L.dpr_plan_ws_bytes.argtypes = [ctypes.POINTER(Scene), c_i32, ctypes.POINTER(View), c_i32]
    L.dpr_plan_ws_bytes.restype = c_sz
    L.dpr_plan_forward.argtypes = [ctypes.POINTER(Scene), c_i32, ctypes.POINTER(View), c_i32,
                                   ctypes.POINTER(Params), c_p, c_sz, c_p, ctypes.POINTER(c_p)]
    L.dpr_plan_forward.restype = c_i32
    L.dpr_plan_forward_render.argtypes = [ctypes.POINTER(Scene), c_i32, ctypes.POINTER(View), c_i32,
                                          ctypes.POINTER(Params), c_p, c_sz, c_p, c_sz, c_p, ctypes.POINTER(c_p),
                                          ctypes.POINTER(c_i32)]
    L.dpr_plan_forward_render.restype = c_i32
    L.dpr_workspace_bytes.argtypes, L.dpr_workspace_bytes.restype = [c_p], c_sz
    L.dpr_backward_ws_bytes.argtypes, L.dpr_backward_ws_bytes.restype = [c_p], c_sz
    L.dpr_render_forward.argtypes, L.dpr_render_forward.restype = [c_p, c_p, c_sz, c_p], c_i32
    L.dpr_render_backward.argtypes = [c_p, c_p, c_sz, PP, PP, PP, PP, PP, c_p, c_sz, c_p]
    L.dpr_render_backward.restype = c_i32
    L.dpr_plan_free.argtypes, L.dpr_plan_free.restype = [c_p], None
    L.dpr_plan_get_info.argtypes, L.dpr_plan_get_info.restype = [c_p, ctypes.POINTER(PlanInfo)], c_i32
    L.dpr_stage_times.argtypes, L.dpr_stage_times.restype = [c_p, ctypes.POINTER(c_f), c_i32], c_i32
    L.dpr_render_forward_1.argtypes = [ctypes.POINTER(Scene), ctypes.POINTER(Camera), ctypes.POINTER(Params),
                                       c_p, c_p, c_p, c_sz, ctypes.POINTER(c_sz), c_p]
    L.dpr_render_forward_1.restype = c_i32
    L.dpr_render_forward_1_noalloc.argtypes = [ctypes.POINTER(Scene), ctypes.POINTER(Camera),
                                               ctypes.POINTER(Params), c_p, c_p, c_p]
    L.dpr_render_forward_1_noalloc.restype = c_i32
    I32P = ctypes.POINTER(c_i32)
    L.dpr_loss_ws_bytes.argtypes, L.dpr_loss_ws_bytes.restype = [c_i32, I32P, I32P], c_sz
    L.dpr_loss_l2_tv.argtypes = [c_i32, PP, PP, I32P, I32P, c_f, PP, c_p, c_p, c_sz, c_p]
    L.dpr_loss_l2_tv.restype = c_i32
    I64P = ctypes.POINTER(c_i64)
    L.dpr_knn_ws_bytes.argtypes, L.dpr_knn_ws_bytes.restype = [c_i64, c_i32], c_sz
    L.dpr_knn.argtypes, L.dpr_knn.restype = [c_i64, c_p, c_i32, c_p, c_p, c_p, c_sz, c_p], c_i32
    L.dpr_hybrid_ws_bytes.argtypes, L.dpr_hybrid_ws_bytes.restype = [c_i64, c_i32, c_i32], c_sz
    L.dpr_voxel_reduce.argtypes = [c_i64, c_i32, c_p, c_p, c_p, c_p, c_i32, c_p, c_p, c_p, c_p, I64P, c_p, c_sz, c_p]
    L.dpr_voxel_reduce.restype = c_i32
    L.dpr_hybrid_update.argtypes = [c_i64, c_i32, c_p, c_p, c_p, c_p, c_i32, c_i32, c_f, c_p, c_p, c_p, c_p, I64P,
                                    c_p, c_sz, c_p]
    L.dpr_hybrid_update.restype = c_i32
    L.dpr_hull_ws_bytes.argtypes, L.dpr_hull_ws_bytes.restype = [c_i64, c_i32, c_p], c_sz
    L.dpr_hull_sample.argtypes = [c_i32, c_p, c_p, c_p, c_p, ctypes.c_uint64, c_i64, c_p, c_i64, I64P, c_p, c_sz, c_p]
    L.dpr_hull_sample.restype = c_i32
    L.dpr_consistency.argtypes = [c_i64, c_p, c_i32, c_p, c_p, c_p, c_p, c_sz, c_p]
    L.dpr_consistency.restype = c_i32
    L.dpr_consistency_filter.argtypes = [c_i64, c_i32, c_p, c_p, c_p, c_p, c_i32, c_p, c_p, c_p, c_p, c_p, c_p, I64P,
                                         c_p, c_sz, c_p]
    L.dpr_consistency_filter.restype = c_i32
    L.dpr_chamfer_ws_bytes.argtypes, L.dpr_chamfer_ws_bytes.restype = [c_i64, c_i64], c_sz
    L.dpr_chamfer.argtypes, L.dpr_chamfer.restype = [c_i64, c_p, c_i64, c_p, c_p, c_p, c_p, c_p, c_p, c_sz, c_p], c_i32
    L.dpr_topk_sh.argtypes, L.dpr_topk_sh.restype = [c_i64, c_p, c_p, c_i64, c_p, c_i32, c_i32, c_p, c_p, c_p], c_i32
    L.dpr_adam_step.argtypes = [c_i64, c_p, c_p, c_p, c_p, c_i32, c_f, c_f, c_f, c_f, c_p]
    L.dpr_adam_step.restype = c_i32
    _lib = L
    return L


def check(rc: int):
    if rc != DPR_OK:
        msg = load().dpr_last_error().decode(errors="replace")
        raise DprError(rc, msg)


def ptr_array(ptrs):
    arr = (c_p * max(1, len(ptrs)))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr
