"""ctypes declarations of the C ABI in include/contentarea.h.

Argument marshalling only.  The shared library is built in-tree by
``paper_2210_14771_amd.build``; if it is missing this module raises instead
of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

from .build import LIB_PATH

CA_OK = 0
CA_E_INVAL = -1
CA_E_UNSUPPORTED = -2
CA_E_NOMEM = -3
CA_E_DEVICE = -4
CA_E_SCRATCH = -5
CA_NOALLOC_SCRATCH_BYTES = 4 << 20
CA_NOALLOC_MAX_FRAMES = 1024
CA_NOALLOC_MAX_SHAPES = 64
CA_MAX_STRIPS = 64
CA_MAX_ATTEMPTS = 4096
CA_MAX_EXTENT = 16384
CA_SG_CAPACITY = 11541

EXPORTS = ("ca_default_params", "ca_create", "ca_destroy", "ca_estimate_area",
           "ca_estimate_area_noalloc",
           "ca_debug_candidates", "ca_debug_attempts", "ca_check_args", "ca_strip_positions",
           "ca_score_tables", "ca_profile_begin", "ca_profile_end", "ca_set_option",
           "ca_get_option", "ca_device_status", "ca_graph_create", "ca_graph_launch",
           "ca_graph_destroy", "ca_set_model", "ca_get_model", "ca_set_momentum",
           "ca_cnn_window_logits", "ca_cnn_gradients", "ca_cnn_sgd_step", "ca_selftest_mfma",
           "ca_set_model_2d", "ca_get_model_2d", "ca_set_momentum_2d", "ca_cnn2d_window_logits",
           "ca_cnn2d_gradients", "ca_cnn2d_sgd_step",
           "ca_autotune", "ca_get_tuning", "ca_get_last_autotune", "ca_server_create", "ca_server_destroy",
           "ca_server_open", "ca_server_close", "ca_server_submit", "ca_server_step",
           "ca_server_stats",
           "ca_error_string", "ca_version")
CA_SCORER_HANDCRAFTED = 0
CA_SCORER_LEARNED = 1
CA_SCORER_LEARNED_2D = 2
CA_CNN2D_PARAMS = 6215
CA_REASON_FALLBACK = 256
CA_CNN_PARAMS = 12273
CA_CNN_WINDOW = 128
CA_CNN_OUTPUTS = 112
CA_OPT_SCHEDULE = 1
CA_OPT_LAG = 2
CA_OPT_QUEUES = 3
CA_OPT_GRID = 4
CA_OPT_SPIN_LIMIT = 5
CA_OPT_PIPELINE = 6
CA_OPT_STRIPS_PER_GROUP = 7
CA_OPT_RANSAC_LANES = 8
CA_SCHEDULE_SPLIT = 0
CA_SCHEDULE_FUSED = 1
CA_SCHEDULE_AUTO = 2


class FrameDesc(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("row_stride", C.c_int32),
                ("pixel_stride", C.c_int32), ("byte_offset", C.c_int64),
                ("frame_uid", C.c_uint64)]


class Params(C.Structure):
    _fields_ = [("n_hstrips", C.c_int32), ("n_vstrips", C.c_int32), ("alpha", C.c_double),
                ("t_g", C.c_double), ("t_theta_deg", C.c_double), ("t_iota", C.c_double),
                ("t_ps", C.c_double), ("t_cs", C.c_double), ("t_px", C.c_int32),
                ("refine_iters", C.c_int32), ("t_ri", C.c_double), ("r_min", C.c_double),
                ("r_max", C.c_double), ("d_max", C.c_double), ("ransac_attempts", C.c_int32),
                ("sampler", C.c_int32), ("seed", C.c_uint64), ("scorer", C.c_int32),
                ("fallback_inlier_frac", C.c_float)]


class ResultRec(C.Structure):
    _fields_ = [("cx", C.c_float), ("cy", C.c_float), ("r", C.c_float), ("score", C.c_float),
                ("inliers", C.c_int32), ("n_points", C.c_int32), ("valid", C.c_int32),
                ("reason", C.c_int32)]


class PointRec(C.Structure):
    _fields_ = [("x", C.c_int16), ("y", C.c_int16), ("score", C.c_float)]


class AttemptRec(C.Structure):
    _fields_ = [("status", C.c_int32), ("fail_stage", C.c_int32), ("i0", C.c_int32),
                ("i1", C.c_int32), ("i2", C.c_int32), ("inliers", C.c_int32),
                ("qsum", C.c_uint64), ("cx", C.c_double), ("cy", C.c_double),
                ("r2", C.c_double)]


class ServerConfig(C.Structure):
    _fields_ = [("max_streams", C.c_int32), ("ring_slots", C.c_int32), ("max_batch", C.c_int32),
                ("max_inflight", C.c_int32), ("hbm_budget", C.c_uint64), ("smooth", C.c_float),
                ("reserved", C.c_int32), ("params", Params)]


class Served(C.Structure):
    _fields_ = [("stream_id", C.c_int32), ("filtered_valid", C.c_int32), ("seq", C.c_uint64),
                ("result", ResultRec), ("fcx", C.c_float), ("fcy", C.c_float),
                ("fr", C.c_float), ("fweight", C.c_float), ("t_submit_ns", C.c_int64),
                ("t_launch_ns", C.c_int64), ("t_done_ns", C.c_int64), ("batch_size", C.c_int32),
                ("pad", C.c_int32)]


class KernelTimes(C.Structure):
    _fields_ = [("total_ms", C.c_double * 3), ("launches", C.c_int64 * 3)]


assert C.sizeof(FrameDesc) == 32 and C.sizeof(ResultRec) == 32
assert C.sizeof(PointRec) == 8 and C.sizeof(AttemptRec) == 56

_lib = None


class NativeError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = lib().ca_error_string(code).decode()
        super().__init__(f"{what} failed: {msg} ({code})")
        self.code = code


def lib() -> C.CDLL:
    """Load libcontentarea.so (built beforehand by ``build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2210_14771_amd.build.build() "
                              "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        vp, i32 = C.c_void_p, C.c_int32
        L.ca_default_params.argtypes = [C.POINTER(Params)]
        L.ca_default_params.restype = None
        L.ca_create.argtypes = [C.POINTER(vp), C.c_int, C.c_size_t]
        L.ca_destroy.argtypes = [vp]
        L.ca_destroy.restype = None
        run_args = [vp, vp, C.POINTER(FrameDesc), i32, C.POINTER(Params)]
        L.ca_estimate_area.argtypes = run_args + [vp, vp]
        L.ca_estimate_area_noalloc.argtypes = run_args + [vp, vp]
        L.ca_debug_candidates.argtypes = run_args + [vp, vp, vp]
        L.ca_debug_attempts.argtypes = run_args + [vp, vp, vp]
        L.ca_check_args.argtypes = [C.POINTER(FrameDesc), i32, C.POINTER(Params)]
        L.ca_strip_positions.argtypes = [i32, i32, C.c_double, C.POINTER(C.c_int32)]
        L.ca_score_tables.argtypes = [C.POINTER(Params), C.POINTER(C.c_float),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_float),
                                      C.POINTER(C.c_float)]
        L.ca_graph_create.argtypes = run_args + [vp, i32, C.POINTER(vp)]
        L.ca_graph_launch.argtypes = [vp, vp]
        L.ca_graph_destroy.argtypes = [vp]
        L.ca_graph_destroy.restype = None
        L.ca_set_model.argtypes = [vp, C.POINTER(C.c_float), i32]
        L.ca_get_model.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_float), i32]
        L.ca_set_momentum.argtypes = [vp, C.POINTER(C.c_float), i32]
        L.ca_cnn_window_logits.argtypes = [vp, vp, vp, i32, vp, vp]
        L.ca_cnn_gradients.argtypes = [vp, vp, vp, vp, vp, i32, C.c_float, vp, vp, vp]
        L.ca_cnn_sgd_step.argtypes = [vp, vp, C.c_float, C.c_float, vp]
        L.ca_selftest_mfma.argtypes = [vp, vp, vp]
        L.ca_set_model_2d.argtypes = [vp, C.POINTER(C.c_float), i32]
        L.ca_get_model_2d.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_float), i32]
        L.ca_set_momentum_2d.argtypes = [vp, C.POINTER(C.c_float), i32]
        L.ca_cnn2d_window_logits.argtypes = [vp, vp, vp, vp, i32, vp, vp]
        L.ca_cnn2d_gradients.argtypes = [vp, vp, vp, vp, vp, vp, i32, C.c_float, vp, vp, vp]
        L.ca_cnn2d_sgd_step.argtypes = [vp, vp, C.c_float, C.c_float, vp]
        L.ca_autotune.argtypes = [vp, vp, C.POINTER(FrameDesc), i32, C.POINTER(Params), i32, vp,
                                  C.POINTER(C.c_int32)]
        L.ca_server_create.argtypes = [vp, C.POINTER(ServerConfig), C.POINTER(vp)]
        L.ca_server_destroy.argtypes = [vp]
        L.ca_server_destroy.restype = None
        L.ca_server_open.argtypes = [vp, i32, i32, i32, C.POINTER(C.c_int32)]
        L.ca_server_close.argtypes = [vp, i32]
        L.ca_server_submit.argtypes = [vp, i32, C.c_uint64, vp, C.c_int64, i32]
        L.ca_server_step.argtypes = [vp, vp, i32, C.POINTER(C.c_int32)]
        L.ca_server_stats.argtypes = [vp, C.POINTER(C.c_int64)]
        L.ca_get_tuning.argtypes = [vp, i32, i32, i32, i32, C.POINTER(C.c_int32)]
        L.ca_get_last_autotune.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.ca_set_option.argtypes = [vp, i32, C.c_int64]
        L.ca_get_option.argtypes = [vp, i32, C.POINTER(C.c_int64)]
        L.ca_device_status.argtypes = [vp]
        L.ca_profile_begin.argtypes = [vp, i32]
        L.ca_profile_end.argtypes = [vp, C.POINTER(KernelTimes)]
        L.ca_error_string.argtypes = [C.c_int]
        L.ca_error_string.restype = C.c_char_p
        L.ca_version.restype = C.c_char_p
        _lib = L
    return _lib


def check(code: int, what: str) -> None:
    if code != CA_OK:
        raise NativeError(code, what)
