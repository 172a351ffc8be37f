"""ctypes declarations of the C ABI in include/tmotif.h.

Loading fails loudly when the built library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtmotif.so")

# Status codes (tmotif.h)
TM_OK, TM_E_INVALID, TM_E_OOM, TM_E_COMPILE, TM_E_DEVICE, TM_E_CAPACITY, TM_E_UNSUPPORTED, TM_E_BUSY, \
    TM_E_CANCELLED = range(9)
STATUS_NAMES = {0: "TM_OK", 1: "TM_E_INVALID", 2: "TM_E_OOM", 3: "TM_E_COMPILE", 4: "TM_E_DEVICE",
                5: "TM_E_CAPACITY", 6: "TM_E_UNSUPPORTED", 7: "TM_E_BUSY", 8: "TM_E_CANCELLED"}

TM_PARAM_BLOCK, TM_PARAM_ROOT_CHUNK, TM_PARAM_GRID = 1, 2, 3
TM_PARAM_PROFILE, TM_PARAM_SPLIT, TM_PARAM_SPLIT_MIN, TM_PARAM_TIER, TM_PARAM_AUTOTUNE = 5, 6, 7, 8, 9
TM_PARAM_WORK_BUDGET, TM_PARAM_MIN_WAVES, TM_PARAM_LEAF_MIN, TM_PARAM_TRACE_US = 10, 11, 12, 13
TM_PARAM_ROOT_HANDOFF = 14
TM_PARAM_HUB_LDS = 15
TM_PARAM_STEP_FORM = 16
TM_PARAM_LINE_SAMPLES = 17
TM_PARAM_XCD_ORDER = 18

# Every function the header declares, for the export check.
EXPORTED = [
    "tm_last_error", "tm_version", "tm_create", "tm_destroy", "tm_set_param", "tm_get_param", "tm_last_kernel_ms",
    "tm_last_launch", "tm_last_trace", "tm_tune_save", "tm_tune_load", "tm_tune_clear",
    "tm_load_graph", "tm_free_graph", "tm_graph_get_info", "tm_graph_edge_order", "tm_graph_copy_csr",
    "tm_graph_set_node_labels", "tm_graph_set_edge_labels",
    "tm_compile_motif", "tm_free_motif", "tm_motif_source", "tm_motif_compile_check", "tm_batch_compile_check",
    "tm_generic_compile_check",
    "tm_count", "tm_enumerate",
    "tm_work_stats", "tm_count_batch", "tm_count_batch_noalloc", "tm_server_start", "tm_submit_query", "tm_poll", "tm_release",
    "tm_server_stats", "tm_server_stop",
]


class EdgePred(ctypes.Structure):
    _fields_ = [("edge", ctypes.c_int32), ("op", ctypes.c_int32), ("theta", ctypes.c_float)]


class MotifDesc(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_edges", ctypes.c_int32), ("edges", ctypes.c_void_p),
                ("delta", ctypes.c_int64), ("gap_max", ctypes.c_void_p), ("pred_edge", ctypes.c_int32),
                ("pred_op", ctypes.c_int32), ("pred_theta", ctypes.c_float), ("n_anti", ctypes.c_int32),
                ("anti", ctypes.c_void_p), ("anti_delta", ctypes.c_void_p), ("node_label", ctypes.c_void_p),
                ("n_pred", ctypes.c_int32), ("preds", ctypes.c_void_p), ("node_label_hi", ctypes.c_void_p),
                ("edge_label", ctypes.c_void_p)]


class RootRange(ctypes.Structure):
    _fields_ = [("t_lo", ctypes.c_int64), ("t_hi", ctypes.c_int64)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("stream_slots", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("enum_pool_bytes", ctypes.c_int64),
                ("queue_capacity", ctypes.c_int32), ("tier", ctypes.c_int32), ("work_budget", ctypes.c_int64),
                ("tune_path", ctypes.c_char_p), ("probe_budget", ctypes.c_int64)]


class Query(ctypes.Structure):
    _fields_ = [("motif", MotifDesc), ("range", RootRange), ("has_range", ctypes.c_int32),
                ("enumerate", ctypes.c_int32), ("tag", ctypes.c_uint64), ("work_budget", ctypes.c_int64)]


class Result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("n_edges", ctypes.c_int32), ("count", ctypes.c_uint64), ("rows", ctypes.c_void_p),
                ("n_rows", ctypes.c_uint64), ("t_arrival_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_launch_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64), ("error", ctypes.c_char * 128),
                ("kernel_tier", ctypes.c_int32), ("probed", ctypes.c_int32)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_edges", ctypes.c_int64), ("t_min", ctypes.c_int64),
                ("t_max", ctypes.c_int64), ("key_bytes", ctypes.c_int32), ("has_weights", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("was_sorted", ctypes.c_int32), ("has_labels", ctypes.c_int32),
                ("has_edge_labels", ctypes.c_int32), ("hub_lists", ctypes.c_int32), ("hub_bytes", ctypes.c_int32)]


_lib = None


class NativeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"native library not built: {LIB_PATH} (build it: python -m paper_2310_02800_amd.build)")
    # PyTorch ships its own HIP runtime. Importing it first makes the library
    # bind to that already-loaded runtime, so the process holds one runtime and
    # torch's device buffers and streams are valid handles for the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "tm_last_error": (ctypes.c_char_p, []),
        "tm_version": (i32, []),
        "tm_create": (i32, [i32, pp]),
        "tm_destroy": (None, [P]),
        "tm_set_param": (i32, [P, i32, i64]),
        "tm_get_param": (i32, [P, i32, P]),
        "tm_last_kernel_ms": (i32, [P, P, P]),
        "tm_last_launch": (i32, [P, P, P, P, P, P]),
        "tm_last_trace": (i32, [P, P, i64, P]),
        "tm_tune_save": (i32, [P, ctypes.c_char_p]),
        "tm_tune_load": (i32, [P, ctypes.c_char_p]),
        "tm_tune_clear": (i32, [P, P]),
        "tm_load_graph": (i32, [P, i64, i64, P, P, P, P, u32, pp]),
        "tm_free_graph": (None, [P]),
        "tm_graph_get_info": (i32, [P, P]),
        "tm_graph_edge_order": (i32, [P, P]),
        "tm_graph_copy_csr": (i32, [P, i32, P, P, P, P]),
        "tm_graph_set_node_labels": (i32, [P, P]),
        "tm_graph_set_edge_labels": (i32, [P, P]),
        "tm_compile_motif": (i32, [P, P, pp]),
        "tm_free_motif": (None, [P]),
        "tm_motif_source": (i32, [P, i32, P, i64, P]),
        "tm_motif_compile_check": (i32, [P, i32, i32, P]),
        "tm_batch_compile_check": (i32, [P, i32, i32, i32, P]),
        "tm_generic_compile_check": (i32, [i32, i32, P]),
        "tm_count": (i32, [P, P, P, P, P, P]),
        "tm_enumerate": (i32, [P, P, P, P, P, P, ctypes.c_uint64, P]),
        "tm_work_stats": (i32, [P, P, P, P, P, P]),
        "tm_count_batch": (i32, [P, P, i32, P, P, P, P]),
        "tm_count_batch_noalloc": (i32, [P, P, i32, P, P, P, P]),
        "tm_server_start": (i32, [P, P, P, pp]),
        "tm_submit_query": (i32, [P, P, P]),
        "tm_poll": (i32, [P, P, i32, P, i32]),
        "tm_release": (i32, [P, ctypes.c_uint64]),
        "tm_server_stats": (i32, [P, P, P, P]),
        "tm_server_stop": (i32, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(status):
    if status != TM_OK:
        msg = lib().tm_last_error()
        raise NativeError(status, msg.decode() if msg else "")
    return status
