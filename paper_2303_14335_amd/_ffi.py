"""ctypes declarations of include/mpld.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpld.so")

MPLD_OK = 0
MPLD_E_INVALID = -1
MPLD_E_NOMEM = -2
MPLD_E_DEVICE = -3
MPLD_E_NOT_READY = -4
MPLD_E_CANCELLED = -5
MPLD_E_INTERNAL = -6
MPLD_E_UNSUPPORTED = -7

MPLD_FEASIBLE, MPLD_INFEASIBLE, MPLD_BUDGET_EXHAUSTED = 0, 1, 2

MPLD_SIMPLIFY = 1 << 0
MPLD_TRACE_HASH = 1 << 1
MPLD_PLAIN = 1 << 2
MPLD_FORCE_WAVE = 1 << 3
MPLD_FORCE_LDS = 1 << 4
MPLD_FORCE_GLOBAL = 1 << 5
MPLD_DIRECT = 1 << 6
MPLD_FORCE_DEVICE = 1 << 7
MPLD_SPLIT_HEAVY = 1 << 8
MPLD_UNTIMED = 1 << 9
MPLD_MARK_CONFLICTS = 1 << 10
MPLD_STITCH_ORDER = 1 << 11
MPLD_ROUNDTRIP = 1 << 12
MPLD_MINIMIZE = 1 << 13

c_i32, c_i64, c_u32, c_u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
vp = ctypes.c_void_p


class mpld_rect(ctypes.Structure):
    _fields_ = [("x0", c_i32), ("y0", c_i32), ("x1", c_i32), ("y1", c_i32)]


class mpld_graph(ctypes.Structure):
    _fields_ = [("num_nodes", c_i32), ("reserved", c_i32), ("num_ce", c_i64), ("ce", vp),
                ("num_se", c_i64), ("se", vp)]


class mpld_options(ctypes.Structure):
    _fields_ = [("struct_size", c_u32), ("k", c_i32), ("node_budget", c_i64),
                ("flags", c_u32), ("min_budget", c_i32)]


class mpld_comp_record(ctypes.Structure):
    _fields_ = [("size", c_i32), ("status", c_i32), ("nodes", c_i64), ("trace_hash", c_u64),
                ("depth_at_stop", c_i32), ("stitches", c_i32), ("first_node", c_i32),
                ("num_edges", c_i32), ("conflicts", c_i32), ("min_nodes", c_i32)]


class mpld_component(ctypes.Structure):
    _fields_ = [("n", c_i32), ("reserved", c_i32), ("m", c_i64), ("edges", vp)]


ALLOC_FN = ctypes.CFUNCTYPE(vp, ctypes.c_size_t, vp)
FREE_FN = ctypes.CFUNCTYPE(None, vp, vp)


class mpld_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", vp)]


class mpld_batch_info(ctypes.Structure):
    _fields_ = [("num_components", c_i32), ("num_wave", c_i32), ("num_lds", c_i32),
                ("num_global", c_i32), ("core_nodes", c_i32), ("max_size", c_i32),
                ("image_bytes", c_i64), ("core_edges", c_i64), ("last_search_ms", ctypes.c_float),
                ("last_total_ms", ctypes.c_float), ("launches", c_i32), ("num_device", c_i32),
                ("heavy_components", c_i32), ("split_rounds", c_i32), ("split_tasks", c_i32),
                ("split_reruns", c_i32), ("last_roundtrip_ms", ctypes.c_float), ("big_waves", c_i32)]


class mpld_tune(ctypes.Structure):
    _fields_ = [("struct_size", c_u32), ("waves_per_block", c_i32), ("max_blocks", c_i32),
                ("use_graph", c_i32), ("order", c_i32), ("giant_device", c_i32),
                ("giant_min_nodes", c_i32), ("best_ms", ctypes.c_float),
                ("default_ms", ctypes.c_float), ("candidates", c_i32), ("from_cache", c_i32),
                ("heavy_first_cap", c_i32), ("heavy_round_cap", c_i32), ("heavy_levels", c_i32),
                ("heavy_device", c_i32), ("root_split", c_i32), ("root_split_min_n", c_i32),
                ("root_split_max", c_i32), ("root_split_chunk", c_i32),
                ("big_one_wave", c_i32)]


class mpld_server_options(ctypes.Structure):
    _fields_ = [("struct_size", c_u32), ("max_components", c_i32), ("arena_bytes", c_i64),
                ("slice_nodes", c_i64), ("host_threads", c_i32), ("graph_builders", c_i32),
                ("device_split", c_i32), ("reserved", c_i32)]


class mpld_server_stats(ctypes.Structure):
    _fields_ = [("submitted", c_i64), ("completed", c_i64), ("failed", c_i64), ("ticks", c_i64),
                ("resident_bytes", c_i64), ("resident_components", c_i64),
                ("peak_bytes", c_i64), ("search_nodes", c_i64), ("admission_waits", c_i64),
                ("device_ms", ctypes.c_double)]


P = ctypes.POINTER

# name -> (restype, argtypes); every entry point of include/mpld.h
SIGNATURES = {
    "mpld_abi_version": (c_u32, []),
    "mpld_error_string": (ctypes.c_char_p, [c_i32]),
    "mpld_last_error": (ctypes.c_char_p, []),
    "mpld_build_graph": (c_i32, [vp, c_i32, c_i32, c_i32, P(vp)]),
    "mpld_build_graph_device": (c_i32, [vp, vp, c_i32, c_i32, c_i32, P(vp)]),
    "mpld_split_graph_device": (c_i32, [vp, P(mpld_graph), c_i32, c_u32, vp, P(c_i32), vp, vp,
                                        vp, P(c_i32)]),
    "mpld_owned_graph_view": (c_i32, [vp, P(mpld_graph)]),
    "mpld_owned_graph_free": (None, [vp]),
    "mpld_context_create": (c_i32, [c_i32, P(mpld_allocator), vp, P(vp)]),
    "mpld_context_destroy": (c_i32, [vp]),
    "mpld_decompose": (c_i32, [vp, P(mpld_graph), P(mpld_options), P(vp)]),
    "mpld_batch_create": (c_i32, [vp, P(mpld_graph), P(mpld_options), P(vp)]),
    "mpld_batch_solve": (c_i32, [vp, c_u32]),
    "mpld_batch_result": (c_i32, [vp, P(vp)]),
    "mpld_batch_get_info": (c_i32, [vp, P(mpld_batch_info)]),
    "mpld_batch_free": (None, [vp]),
    "mpld_batch_autotune": (c_i32, [vp, c_i32, ctypes.c_char_p, P(mpld_tune)]),
    "mpld_batch_get_tune": (c_i32, [vp, P(mpld_tune)]),
    "mpld_batch_set_tune": (c_i32, [vp, P(mpld_tune)]),
    "mpld_solve_components": (c_i32, [vp, P(mpld_component), c_i32, P(mpld_options),
                                      P(mpld_comp_record), vp]),
    "mpld_solve_components_noalloc": (c_i32, [vp, P(mpld_component), c_i32, P(mpld_options),
                                              P(mpld_comp_record), vp]),
    "mpld_measure_lds_read_rate": (c_i32, [vp, c_i32, c_i32, P(ctypes.c_double),
                                           P(ctypes.c_double)]),
    "mpld_measure_launch_floor": (c_i32, [vp, c_i32, c_i32, c_i32, P(ctypes.c_double)]),
    "mpld_measure_touch_floor": (c_i32, [vp, c_i32, c_i32, c_i32, P(ctypes.c_double)]),
    "mpld_result_colors": (vp, [vp, P(c_i32)]),
    "mpld_result_component_of": (vp, [vp]),
    "mpld_result_num_components": (c_i32, [vp]),
    "mpld_result_components": (vp, [vp]),
    "mpld_result_totals": (None, [vp, P(c_i64), P(c_i64), P(c_i64)]),
    "mpld_result_timing": (None, [vp, P(ctypes.c_double), P(ctypes.c_double)]),
    "mpld_result_free": (None, [vp]),
    "mpld_server_create": (c_i32, [vp, P(mpld_server_options), P(vp)]),
    "mpld_server_submit": (c_i32, [vp, P(mpld_graph), P(mpld_options), P(c_u64)]),
    "mpld_server_submit_layout": (c_i32, [vp, vp, c_i32, c_i32, c_i32, P(mpld_options),
                                          P(c_u64)]),
    "mpld_server_poll": (c_i32, [vp, c_u64, P(vp)]),
    "mpld_server_wait": (c_i32, [vp, c_u64, c_i64, P(vp)]),
    "mpld_server_get_stats": (c_i32, [vp, P(mpld_server_stats)]),
    "mpld_server_destroy": (c_i32, [vp]),
}

_lib = None


def load():
    """Loads libmpld.so; raises if it is not built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: the HIP library must be built "
                "(python -m paper_2303_14335_amd.build) - there is no CPU fallback")
        # torch first: it ships its own HIP and HSA runtimes; with the
        # library loaded before torch, context creation has reported no
        # visible device
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
