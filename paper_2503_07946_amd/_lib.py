"""ctypes binding of lib7dgs.so (include/sd7.h).  Argument marshalling only:
every step of the render path runs in the HIP library.  There is no CPU
fallback: loading fails loudly when the library has not been built."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "lib7dgs.so")

SD7_OK, SD7_EINVAL, SD7_EHIP, SD7_EWORKSPACE, SD7_ENOMEM = 0, -1, -2, -3, -4
SD7_MAX_FRAMES = 64
SD7_TILE = 16
SD7_PAIR_ROUND = 2048       # a frame's arena share is a multiple of this (sd7.h)
SD7_FLAG_NONPOS_DIAG, SD7_FLAG_NONFINITE, SD7_FLAG_PAIR_OVERFLOW = 1, 2, 4
SD7_FLAG_SORT_STALL = 8     # a depth-sort wait gave up: the frame is not valid
SD7_OUT_SLICED = 1          # sd7_frame.outputs: keep the sliced statistics
SD7_CNT_KEPT, SD7_CNT_PAIRS, SD7_CNT_PAIR_BASE, SD7_CNT_FLAGS = 0, 1, 2, 3
SD7_CNT_NEEDED = 4          # pairs the frame needs (also written on overflow)
SD7_CNT_WORDS = 16
SD7_AGR_WEIGHTS = 9443      # floats of one scene's AGR weights (sd7.h)
SD7_STATIC_WS_BYTES = 64 << 20  # the library-owned workspace of sd7_render_static

P = ctypes.c_void_p
f32 = ctypes.c_float


class Sd7Scene(ctypes.Structure):
    _fields_ = [("mu_p", P), ("mu_t", P), ("mu_d", P), ("L", P), ("alpha", P), ("sh", P),
                ("n", ctypes.c_int64), ("agr", P)]


class Sd7View(ctypes.Structure):
    _fields_ = [("R_wc", f32 * 9), ("c", f32 * 3), ("fx", f32), ("fy", f32), ("cx", f32),
                ("cy", f32), ("W", ctypes.c_int32), ("H", ctypes.c_int32), ("t", f32),
                ("d", f32 * 3), ("lambda_t", f32), ("lambda_d", f32), ("bg", f32 * 3),
                ("d_per_gaussian", ctypes.c_int32)]


class Sd7SceneGrad(ctypes.Structure):
    _fields_ = [("mu_p", P), ("mu_t", P), ("mu_d", P), ("L", P), ("alpha", P), ("sh", P),
                ("lambda_", P)]


class Sd7Arrays(ctypes.Structure):
    _fields_ = [("mu_p", P), ("mu_t", P), ("mu_d", P), ("L", P), ("alpha", P), ("sh", P)]


class Sd7Adam(ctypes.Structure):
    _fields_ = [("lr", f32 * 6), ("beta1", f32), ("beta2", f32), ("eps", f32), ("step", ctypes.c_int32),
                ("alpha_lo", f32), ("alpha_hi", f32), ("diag_min", f32)]


class Sd7Frame(ctypes.Structure):
    _fields_ = [("scene", Sd7Scene), ("view", Sd7View), ("image", P), ("final_T", P),
                ("last", P), ("dL_dimage", P), ("grad", Sd7SceneGrad), ("ncontrib", P),
                ("outputs", ctypes.c_uint32)]


_OFFS = ["off_table", "off_counts", "off_mu_c", "off_cov_c", "off_alpha_c", "off_splat",
         "off_rect", "off_depth_key", "off_order", "off_pair_g", "off_ranges",
         "off_d_splat", "off_d_mu_c", "off_d_cov_c", "off_d_alpha_c", "off_scratch"]


class Sd7StageTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("calls", ctypes.c_uint64), ("total_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double)]


class Sd7Layout(ctypes.Structure):
    _fields_ = ([("bytes", ctypes.c_size_t), ("nframes", ctypes.c_int32),
                 ("tile_sort_passes", ctypes.c_int32), ("n_total", ctypes.c_int64),
                 ("tiles_total", ctypes.c_int64), ("pair_capacity", ctypes.c_int64)]
                + [(k, ctypes.c_size_t) for k in _OFFS]
                + [("g0", ctypes.c_int64 * SD7_MAX_FRAMES),
                   ("tile0", ctypes.c_int64 * SD7_MAX_FRAMES)])


STAGES = ("sd7_slice", "sd7_project", "sd7_slice_project", "sd7_bin", "sd7_rasterize", "sd7_render",
          "sd7_rasterize_backward", "sd7_project_backward", "sd7_slice_backward")
EXPORTS = ("sd7_create", "sd7_destroy", "sd7_last_error", "sd7_plan", "sd7_read_counts",
           "sd7_cov_decompose", "sd7_split_test", "sd7_adam_step", "sd7_prune_workspace_size",
           "sd7_prune_count", "sd7_prune_apply", "sd7_render_static", "sd7_graph_create",
           "sd7_graph_launch", "sd7_graph_destroy", "sd7_profile_read") + STAGES


class Sd7Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (once).  Raises if it is missing.

    The library and PyTorch must share one HIP runtime: both name it by the
    same soname, so whichever is loaded first serves the process.  PyTorch
    is imported first so that its runtime (the one that owns the device
    memory and streams handed to the library) is that one."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the process's HIP runtime)
    if not os.path.exists(path):
        raise RuntimeError(f"lib7dgs.so not built at {path}; run __graft_entry__.build() "
                           "(the render path has no CPU fallback)")
    L = ctypes.CDLL(path)
    L.sd7_create.argtypes = [ctypes.c_int, ctypes.POINTER(P)]
    L.sd7_create.restype = ctypes.c_int32
    L.sd7_destroy.argtypes = [P]
    L.sd7_destroy.restype = None
    L.sd7_last_error.argtypes = []
    L.sd7_last_error.restype = ctypes.c_char_p
    L.sd7_plan.argtypes = [ctypes.POINTER(Sd7Frame), ctypes.c_int, ctypes.c_int64,
                           ctypes.POINTER(Sd7Layout)]
    L.sd7_plan.restype = ctypes.c_int32
    for name in STAGES:
        fn = getattr(L, name)
        fn.argtypes = [P, ctypes.POINTER(Sd7Frame), ctypes.c_int, ctypes.c_int64, P,
                       ctypes.c_size_t, P]
        fn.restype = ctypes.c_int32
    L.sd7_render_static.argtypes = [P, ctypes.POINTER(Sd7Frame), ctypes.c_int, ctypes.c_int64, P, P]
    L.sd7_render_static.restype = ctypes.c_int32
    L.sd7_graph_create.argtypes = [P, ctypes.POINTER(Sd7Frame), ctypes.c_int, ctypes.c_int64, P, ctypes.c_size_t,
                                   ctypes.POINTER(P)]
    L.sd7_graph_create.restype = ctypes.c_int32
    L.sd7_graph_launch.argtypes = [P, ctypes.POINTER(Sd7Frame), ctypes.c_int, P]
    L.sd7_graph_launch.restype = ctypes.c_int32
    L.sd7_graph_destroy.argtypes = [P]
    L.sd7_graph_destroy.restype = None
    L.sd7_profile_read.argtypes = [P, ctypes.POINTER(Sd7StageTime), ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                   ctypes.c_int]
    L.sd7_profile_read.restype = ctypes.c_int32
    L.sd7_read_counts.argtypes = [P, ctypes.c_int, P, ctypes.POINTER(ctypes.c_uint32), P]
    L.sd7_read_counts.restype = ctypes.c_int32
    L.sd7_cov_decompose.argtypes = [P, ctypes.c_int64, P, P, P, P]
    L.sd7_cov_decompose.restype = ctypes.c_int32
    L.sd7_split_test.argtypes = [P, ctypes.POINTER(Sd7Scene), ctypes.c_float, ctypes.c_float, P, P]
    L.sd7_split_test.restype = ctypes.c_int32
    L.sd7_adam_step.argtypes = [P, ctypes.c_int64, ctypes.POINTER(Sd7Arrays), ctypes.POINTER(Sd7SceneGrad),
                                ctypes.POINTER(Sd7Arrays), ctypes.POINTER(Sd7Arrays), ctypes.POINTER(Sd7Adam), P]
    L.sd7_adam_step.restype = ctypes.c_int32
    L.sd7_prune_workspace_size.argtypes = [ctypes.c_int64]
    L.sd7_prune_workspace_size.restype = ctypes.c_size_t
    L.sd7_prune_count.argtypes = [P, ctypes.c_int64, P, ctypes.c_float, P, ctypes.c_size_t, P, P]
    L.sd7_prune_count.restype = ctypes.c_int32
    L.sd7_prune_apply.argtypes = [P, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(P), ctypes.POINTER(P),
                                  ctypes.POINTER(ctypes.c_int32), ctypes.c_int, P, ctypes.c_size_t, P]
    L.sd7_prune_apply.restype = ctypes.c_int32
    _lib = L
    return L


def check(code: int):
    if code != SD7_OK:
        msg = load().sd7_last_error().decode(errors="replace")
        raise Sd7Error(code, msg)
