"""ctypes declarations of the C ABI in include/gm.h (argument marshalling only).

The shared library is built in-tree (``paper_1503_07241_amd/libgm.so``) by
``paper_1503_07241_amd.build``. There is no fallback: if the library is
missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgm.so")

GM_OK, GM_EINVAL, GM_ENOMEM, GM_EHIP, GM_EUNSUPPORTED, GM_ESTATE = range(6)
STATUS_NAMES = {0: "GM_OK", 1: "GM_EINVAL", 2: "GM_ENOMEM", 3: "GM_EHIP", 4: "GM_EUNSUPPORTED",
                5: "GM_ESTATE"}

GM_PREP_DROP_SELF_LOOPS, GM_PREP_SYMMETRIZE, GM_PREP_UPPER_DAG = 1, 2, 4
GM_W_NONE, GM_W_U32, GM_W_F32 = 0, 1, 2
GM_LAYOUT_OUT, GM_LAYOUT_IN = 1, 2
GM_PROG_BFS, GM_PROG_SSSP, GM_PROG_PAGERANK, GM_PROG_PPR, GM_PROG_TC, GM_PROG_DEGREE = range(1, 7)
GM_ORDER_OUT, GM_ORDER_IN, GM_ORDER_ALL = 1, 2, 3
GM_VARIANT_LIST_FRONTIER, GM_VARIANT_VERTEX_PUSH, GM_VARIANT_ROW_PULL = 1, 2, 4
GM_VARIANT_DEGREE_ORDER = 8


class GmError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__("%s failed with %s: %s" % (where, STATUS_NAMES.get(status, status), message))


class gm_graph_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("max_out", ctypes.c_int64),
                ("max_in", ctypes.c_int64), ("wtype", ctypes.c_int32), ("prep", ctypes.c_uint32),
                ("layouts", ctypes.c_uint32), ("device", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("n_src", ctypes.c_int64),
                ("n_dst", ctypes.c_int64)]


class gm_program(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("order", ctypes.c_int32), ("r", ctypes.c_float),
                ("flags", ctypes.c_uint32)]


class gm_frontier(ctypes.Structure):
    _fields_ = [("ids", ctypes.c_void_p), ("count", ctypes.c_int64), ("bitmap", ctypes.c_void_p)]


class gm_run_stats(ctypes.Structure):
    _fields_ = [("supersteps", ctypes.c_int32), ("push_supersteps", ctypes.c_int32),
                ("pull_supersteps", ctypes.c_int32), ("edges_scanned", ctypes.c_int64)]


class gm_plan_run(ctypes.Structure):
    _fields_ = [("g", ctypes.c_void_p), ("prog", gm_program), ("batched", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("ids", ctypes.c_void_p), ("count", ctypes.c_int64),
                ("vprop", ctypes.c_void_p)]


class gm_plan_result(ctypes.Structure):
    _fields_ = [("iters_done", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("edges_scanned", ctypes.c_int64)]


TUNING_FIELDS = ("pull_div", "superstep_batch", "push_blocks", "ppr_chunk", "tc_wave_max",
                 "tc_wave_work", "tc_block_work", "pr_hot", "variant")


class gm_tuning(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint32) for f in TUNING_FIELDS]


_lib = None


def load():
    """Load libgm.so once; raises OSError if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError("libgm.so is not built (%s); run paper_1503_07241_amd.build.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sigs = {
        "gm_last_error": ([], ctypes.c_char_p),
        "gm_version": ([], ctypes.c_char_p),
        "gm_graph_from_coo": ([i64, i64, vp, vp, vp, i32, u32, u32, vp, ctypes.POINTER(vp)], i32),
        "gm_graph_get_info": ([vp, ctypes.POINTER(gm_graph_info)], i32),
        "gm_graph_edges": ([vp, vp, vp, vp], i32),
        "gm_graph_destroy": ([vp], i32),
        "gm_run_vertex_program": ([vp, ctypes.POINTER(gm_program), ctypes.POINTER(gm_frontier), i32,
                                   vp, vp, ctypes.POINTER(i32), vp], i32),
        "gm_last_run_stats": ([vp, ctypes.POINTER(gm_run_stats)], i32),
        "gm_triangle_count": ([vp, vp, ctypes.POINTER(ctypes.c_uint64), vp], i32),
        "gm_run_batched": ([vp, ctypes.POINTER(gm_program), vp, i32, i32, vp, ctypes.POINTER(i32),
                            vp], i32),
        "gm_bipartite_from_coo": ([i64, i64, i64, vp, vp, vp, vp, ctypes.POINTER(vp)], i32),
        "gm_cf_forward": ([vp, i32, vp, vp, ctypes.c_float, vp, vp], i32),
        "gm_cf_backward": ([vp, i32, vp, vp, ctypes.c_float, ctypes.c_float, vp, vp, vp], i32),
        "gm_cf_gd": ([vp, i32, vp, vp, ctypes.c_float, ctypes.c_float, i32, vp, vp], i32),
        "gm_pagerank_forward_w": ([vp, vp, ctypes.c_float, i32, vp, vp], i32),
        "gm_pagerank_vjp_w": ([vp, vp, ctypes.c_float, i32, vp, vp, vp, vp], i32),
        "gm_graph_union": ([vp, i32, vp, ctypes.POINTER(vp)], i32),
        "gm_plan_create": ([ctypes.POINTER(gm_plan_run), i32, vp, ctypes.POINTER(vp)], i32),
        "gm_plan_launch": ([vp, vp], i32),
        "gm_plan_results": ([vp, ctypes.POINTER(gm_plan_result), vp], i32),
        "gm_plan_destroy": ([vp], i32),
        "gm_graph_get_tuning": ([vp, ctypes.POINTER(gm_tuning)], i32),
        "gm_graph_set_tuning": ([vp, ctypes.POINTER(gm_tuning)], i32),
        "gm_autotune": ([vp, ctypes.POINTER(gm_program), i32, vp, i64, i32, i32,
                         ctypes.c_char_p, ctypes.POINTER(gm_tuning), vp], i32),
        "gm_graph_prepare": ([vp, ctypes.POINTER(gm_program), vp], i32),
        "gm_mtx_read": ([ctypes.c_char_p, ctypes.POINTER(i64), ctypes.POINTER(i64), vp, vp, vp,
                         ctypes.POINTER(i32)], i32),
        "gm_graph_from_mtx": ([ctypes.c_char_p, u32, u32, vp, ctypes.POINTER(vp)], i32),
        "gm_graph_release": ([vp], i32),
        "gm_pagerank_noalloc": ([vp, ctypes.c_float, i32, vp, vp], i32),
        "gm_run_multi_graph": ([ctypes.POINTER(vp), i32, ctypes.POINTER(gm_program),
                                ctypes.POINTER(i32), ctypes.POINTER(vp), i32,
                                ctypes.POINTER(i32), vp], i32),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != GM_OK:
        raise GmError(status, where, load().gm_last_error().decode(errors="replace"))
