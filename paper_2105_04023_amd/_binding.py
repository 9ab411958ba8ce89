"""ctypes binding of include/im.h: argument marshalling only, every step runs in the HIP library.

The library is loaded from this package directory (libhipfuser.so, built in-tree by
``build.py``).  If it is missing, loading raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhipfuser.so")

IM_OK = 0
IM_ERR_INVALID_ARG, IM_ERR_INVALID_GRAPH, IM_ERR_OUT_OF_BUDGET, IM_ERR_DEVICE, IM_ERR_STATE = -1, -2, -3, -4, -5
STATUS_NAMES = {0: "IM_OK", -1: "IM_ERR_INVALID_ARG", -2: "IM_ERR_INVALID_GRAPH", -3: "IM_ERR_OUT_OF_BUDGET",
                -4: "IM_ERR_DEVICE", -5: "IM_ERR_STATE"}
IM_PROB_CONSTANT, IM_PROB_WEIGHTED_CASCADE, IM_PROB_PER_EDGE = 0, 1, 2
IM_BUILD_TIME_SWEEPS, IM_BUILD_IN_PLACE, IM_BUILD_ATOMIC_REVERSE, IM_BUILD_TIME_PIECES = 1, 2, 4, 8
IM_NOALLOC_MAX_K = 4096  # largest K of im_select_seeds_noalloc

# Every symbol include/im.h declares (checked by the CPU test suite).
EXPORTED = [
    "im_ctx_create", "im_ctx_free", "im_ctx_bytes_in_use", "im_sketch_bytes_needed", "im_build_sketches",
    "im_estimate", "im_estimate_all", "im_select_seeds", "im_sketch_get_info", "im_sketch_get_trace",
    "im_sketch_get_registers", "im_sketch_get_blocked", "im_sketch_free", "im_last_error", "im_version",
    "im_sketch_get_sweep_log", "im_sketch_clear_sweep_log", "im_batch_create", "im_batch_run", "im_batch_get_result",
    "im_batch_get_registers", "im_batch_device_bytes", "im_batch_free", "im_server_create", "im_server_add_graph",
    "im_server_submit", "im_server_wait", "im_server_get_stats", "im_server_free", "im_evaluate_influence",
    "im_select_seeds_noalloc", "im_server_cancel", "im_select_seeds_resume",
]


class ImError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class im_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("xadj", ctypes.c_void_p), ("adj", ctypes.c_void_p),
                ("on_device", ctypes.c_int32), ("offset_bits", ctypes.c_int32)]


class im_probs(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("p", ctypes.c_float), ("per_edge", ctypes.c_void_p)]


class im_build_opts(ctypes.Structure):
    _fields_ = [("eps_c", ctypes.c_double), ("heavy_degree", ctypes.c_int32), ("piece_edges", ctypes.c_int32),
                ("sparse_div", ctypes.c_int32), ("flags", ctypes.c_int32)]


class im_select_opts(ctypes.Structure):
    _fields_ = [("eps_g", ctypes.c_double), ("eps_l", ctypes.c_double)]


class im_step(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_int32), ("rebuilt", ctypes.c_int32), ("fresh", ctypes.c_int32),
                ("sweeps", ctypes.c_int32), ("score", ctypes.c_int64), ("reach", ctypes.c_int64),
                ("e", ctypes.c_double), ("sigma", ctypes.c_double), ("delta", ctypes.c_double),
                ("err_l", ctypes.c_double), ("err_g", ctypes.c_double), ("visits", ctypes.c_int64)]


class im_sketch_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("R", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("visits", ctypes.c_int64), ("build_ms", ctypes.c_double), ("prep_ms", ctypes.c_double),
                ("device_bytes", ctypes.c_size_t), ("heavy_rows", ctypes.c_int64),
                ("heavy_pieces", ctypes.c_int64)]


class im_sweep_rec(ctypes.Structure):
    _fields_ = [("simulate", ctypes.c_int32), ("sweep", ctypes.c_int32), ("ran", ctypes.c_int32),
                ("kernel_ms", ctypes.c_float), ("sweep_ms", ctypes.c_float), ("heavy_ms", ctypes.c_float),
                ("light_visits", ctypes.c_int64), ("visits", ctypes.c_int64), ("live", ctypes.c_int64),
                ("live_next", ctypes.c_int64), ("sparse", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("light_merged", ctypes.c_int64), ("merged", ctypes.c_int64)]


class im_select_stats(ctypes.Structure):
    _fields_ = [("rebuilds", ctypes.c_int32), ("reserved", ctypes.c_int32), ("rebuild_sweeps", ctypes.c_int64),
                ("rebuild_visits", ctypes.c_int64), ("bfs_levels", ctypes.c_int64), ("device_ms", ctypes.c_double),
                ("wall_ms", ctypes.c_double)]


class im_batch_job(ctypes.Structure):
    _fields_ = [("graph", im_csr), ("probs", im_probs), ("R", ctypes.c_int32), ("K", ctypes.c_int32),
                ("hash_seed", ctypes.c_uint32), ("reserved", ctypes.c_int32), ("eps_c", ctypes.c_double),
                ("eps_g", ctypes.c_double), ("eps_l", ctypes.c_double)]


class im_batch_opts(ctypes.Structure):
    _fields_ = [("autotune", ctypes.c_int32), ("lanes_per_row", ctypes.c_int32), ("tile_edges", ctypes.c_int32),
                ("heavy_degree", ctypes.c_int32), ("piece_edges", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("pin_edges", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class im_batch_job_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("build_sweeps", ctypes.c_int32), ("rebuilds", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("build_visits", ctypes.c_int64), ("rebuild_sweeps", ctypes.c_int64),
                ("rebuild_visits", ctypes.c_int64), ("bfs_levels", ctypes.c_int64)]


class im_batch_stats(ctypes.Structure):
    _fields_ = [("device_ms", ctypes.c_double), ("wall_ms", ctypes.c_double), ("tiles", ctypes.c_int64),
                ("phases", ctypes.c_int64), ("lanes_per_row", ctypes.c_int32), ("tile_edges", ctypes.c_int32),
                ("heavy_degree", ctypes.c_int32), ("piece_edges", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("candidates", ctypes.c_int32)]


class im_server_opts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("max_copies", ctypes.c_int32), ("hbm_budget", ctypes.c_size_t)]


class im_request(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("kind", ctypes.c_int), ("p", ctypes.c_float), ("R", ctypes.c_int32),
                ("K", ctypes.c_int32), ("hash_seed", ctypes.c_uint32), ("eps_c", ctypes.c_double),
                ("eps_g", ctypes.c_double), ("eps_l", ctypes.c_double)]


class im_response(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("slot", ctypes.c_int32), ("sketch_reused", ctypes.c_int32),
                ("rebuilds", ctypes.c_int32), ("queue_ms", ctypes.c_double), ("build_ms", ctypes.c_double),
                ("select_ms", ctypes.c_double), ("latency_ms", ctypes.c_double)]


class im_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("sketches_built", ctypes.c_int64), ("evictions", ctypes.c_int64),
                ("resident_sketches", ctypes.c_int64), ("device_bytes", ctypes.c_size_t)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


def load(path: str = LIB_PATH):
    """Loads libhipfuser.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2105_04023_amd/build.py (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    p, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "im_ctx_create": ([i32, p, sz, ALLOC_FN, FREE_FN, p, ctypes.POINTER(p)], ctypes.c_int),
        "im_ctx_free": ([p], None),
        "im_ctx_bytes_in_use": ([p], sz),
        "im_sketch_bytes_needed": ([i64, i64, i32, ctypes.c_int], sz),
        "im_build_sketches": ([p, ctypes.POINTER(im_csr), ctypes.POINTER(im_probs), i32, ctypes.c_uint32,
                               ctypes.POINTER(im_build_opts), ctypes.POINTER(p)], ctypes.c_int),
        "im_estimate": ([p, p, i64, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
        "im_estimate_all": ([p, p, i32], ctypes.c_int),
        "im_select_seeds": ([p, i32, ctypes.POINTER(im_select_opts), p, p, ctypes.POINTER(im_select_stats)],
                            ctypes.c_int),
        "im_select_seeds_noalloc": ([p, i32, ctypes.POINTER(im_select_opts), p, p,
                                     ctypes.POINTER(im_select_stats)], ctypes.c_int),
        "im_select_seeds_resume": ([p, i32, ctypes.POINTER(im_select_opts), p, p,
                                    ctypes.POINTER(im_select_stats)], ctypes.c_int),
        "im_sketch_get_info": ([p, ctypes.POINTER(im_sketch_info)], ctypes.c_int),
        "im_sketch_get_trace": ([p, p, p, i32, ctypes.POINTER(i32)], ctypes.c_int),
        "im_sketch_get_registers": ([p, i32, p], ctypes.c_int),
        "im_sketch_get_blocked": ([p, p], ctypes.c_int),
        "im_sketch_free": ([p], None),
        "im_last_error": ([], ctypes.c_char_p),
        "im_version": ([], ctypes.c_char_p),
        "im_sketch_get_sweep_log": ([p, p, i32], i32),
        "im_sketch_clear_sweep_log": ([p], None),
        "im_batch_create": ([p, i32, p, ctypes.POINTER(im_batch_opts), ctypes.POINTER(p)], ctypes.c_int),
        "im_batch_run": ([p, ctypes.POINTER(im_batch_stats)], ctypes.c_int),
        "im_batch_get_result": ([p, i32, p, p, ctypes.POINTER(im_batch_job_result)], ctypes.c_int),
        "im_batch_get_registers": ([p, i32, i32, p], ctypes.c_int),
        "im_batch_device_bytes": ([p], sz),
        "im_batch_free": ([p], None),
        "im_server_create": ([i32, ctypes.POINTER(im_server_opts), ctypes.POINTER(p)], ctypes.c_int),
        "im_server_add_graph": ([p, ctypes.POINTER(im_csr), ctypes.POINTER(i32)], ctypes.c_int),
        "im_server_submit": ([p, ctypes.POINTER(im_request), p, ctypes.POINTER(i64)], ctypes.c_int),
        "im_server_wait": ([p, i64, ctypes.POINTER(im_response)], ctypes.c_int),
        "im_server_cancel": ([p, i64], ctypes.c_int),
        "im_server_get_stats": ([p, ctypes.POINTER(im_server_stats)], ctypes.c_int),
        "im_server_free": ([p], None),
        "im_evaluate_influence": ([p, ctypes.POINTER(im_csr), ctypes.POINTER(im_probs), i32, ctypes.c_uint32, p, i32,
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(status: int):
    if status != IM_OK:
        msg = load().im_last_error().decode(errors="replace")
        raise ImError(status, msg)
