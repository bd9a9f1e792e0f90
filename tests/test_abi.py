"""C-ABI checks that need no GPU: the library loads, exports every function
include/*.h declares, and rejects bad arguments before touching the device."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import paper_1503_07241_amd as gm
from paper_1503_07241_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1503_07241_amd import build
        build.build()
    return _lib.load()


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(gm_\w+)\s*\(", text, re.M):
            names.add(m.group(1))
    return names


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "gm_run_vertex_program" in names and "gm_graph_from_coo" in names
    for name in sorted(names):
        assert hasattr(lib, name), "libgm.so does not export %s" % name


def test_version_and_clean_error(lib):
    assert b"gfx950" in lib.gm_version()


def status(lib, fn, *args):
    st = getattr(lib, fn)(*args)
    return st, lib.gm_last_error().decode()


def test_from_coo_argument_errors(lib):
    src = np.array([0, 1, 2], dtype=np.int32)
    dst = np.array([1, 2, 5], dtype=np.int32)
    out = ctypes.c_void_p()
    P = src.ctypes.data
    Q = dst.ctypes.data
    # out NULL
    assert status(lib, "gm_graph_from_coo", 4, 3, P, Q, None, 0, 1, 1, None, None)[0] == _lib.GM_EINVAL
    # n <= 0, n too large
    for n in (0, -3, 2**31):
        st, msg = status(lib, "gm_graph_from_coo", n, 3, P, Q, None, 0, 1, 1, None, ctypes.byref(out))
        assert st == _lib.GM_EINVAL and "n =" in msg
    # m < 0
    assert status(lib, "gm_graph_from_coo", 8, -1, P, Q, None, 0, 1, 1, None, ctypes.byref(out))[0] == _lib.GM_EINVAL
    # src NULL with m > 0
    assert status(lib, "gm_graph_from_coo", 8, 3, None, Q, None, 0, 1, 1, None, ctypes.byref(out))[0] == _lib.GM_EINVAL
    # id out of range (dst 5 with n = 4)
    st, msg = status(lib, "gm_graph_from_coo", 4, 3, P, Q, None, 0, 1, 1, None, ctypes.byref(out))
    assert st == _lib.GM_EINVAL and "outside" in msg
    # negative id
    neg = np.array([0, -1, 2], dtype=np.int32)
    assert status(lib, "gm_graph_from_coo", 8, 3, neg.ctypes.data, Q, None, 0, 1, 1, None, ctypes.byref(out))[0] == _lib.GM_EINVAL
    # unknown wtype, weights vs wtype mismatch
    assert status(lib, "gm_graph_from_coo", 8, 3, P, Q, None, 7, 1, 1, None, ctypes.byref(out))[0] == _lib.GM_EINVAL
    assert status(lib, "gm_graph_from_coo", 8, 3, P, Q, None, _lib.GM_W_U32, 1, 1, None, ctypes.byref(out))[0] == _lib.GM_EINVAL
    w = np.ones(3, dtype=np.uint32)
    assert status(lib, "gm_graph_from_coo", 8, 3, P, Q, w.ctypes.data, 0, 1, 1, None, ctypes.byref(out))[0] == _lib.GM_EINVAL
    # non-finite float weight
    wf = np.array([1.0, np.nan, 2.0], dtype=np.float32)
    assert status(lib, "gm_graph_from_coo", 8, 3, P, Q, wf.ctypes.data, _lib.GM_W_F32, 1, 1, None, ctypes.byref(out))[0] == _lib.GM_EINVAL
    # unknown prep / layout bits
    assert status(lib, "gm_graph_from_coo", 8, 3, P, Q, None, 0, 64, 1, None, ctypes.byref(out))[0] == _lib.GM_EINVAL
    assert status(lib, "gm_graph_from_coo", 8, 3, P, Q, None, 0, 1, 0, None, ctypes.byref(out))[0] == _lib.GM_EINVAL
    assert status(lib, "gm_graph_from_coo", 8, 3, P, Q, None, 0, 1, 8, None, ctypes.byref(out))[0] == _lib.GM_EINVAL
    assert out.value is None


def test_dead_handles_are_estate(lib):
    bogus = ctypes.c_void_p(0x1234)
    info = _lib.gm_graph_info()
    assert lib.gm_graph_get_info(None, ctypes.byref(info)) == _lib.GM_ESTATE
    assert lib.gm_graph_get_info(bogus, ctypes.byref(info)) == _lib.GM_ESTATE
    assert lib.gm_graph_destroy(None) == _lib.GM_ESTATE
    assert lib.gm_graph_destroy(bogus) == _lib.GM_ESTATE
    assert "not live" in lib.gm_last_error().decode()
    prog = _lib.gm_program(_lib.GM_PROG_BFS, _lib.GM_ORDER_OUT, 0.15, 0)
    it = ctypes.c_int32()
    assert lib.gm_run_vertex_program(bogus, ctypes.byref(prog), None, -1, None, None,
                                     ctypes.byref(it), None) == _lib.GM_ESTATE
    st = _lib.gm_run_stats()
    assert lib.gm_last_run_stats(bogus, ctypes.byref(st)) == _lib.GM_ESTATE
    assert lib.gm_graph_edges(bogus, None, None, None) == _lib.GM_ESTATE


def test_python_binding_raises(lib):
    with pytest.raises(gm.GmError) as ei:
        gm.Graph.from_coo(4, [0, 1], [1, 9])
    assert ei.value.status == _lib.GM_EINVAL
    with pytest.raises(ValueError):
        gm.Graph.from_coo(4, [0, 1], [1])


def test_union_plan_tuning_validation_without_device(lib):
    bogus = ctypes.c_void_p(0x1234)
    out = ctypes.c_void_p()
    parts = (ctypes.c_void_p * 2)(0x1234, 0x5678)
    assert lib.gm_graph_union(None, 2, None, ctypes.byref(out)) == _lib.GM_EINVAL
    assert lib.gm_graph_union(parts, 0, None, ctypes.byref(out)) == _lib.GM_EINVAL
    assert lib.gm_graph_union(parts, 2, None, None) == _lib.GM_EINVAL
    assert lib.gm_graph_union(parts, 2, None, ctypes.byref(out)) == _lib.GM_ESTATE
    runs = (_lib.gm_plan_run * 1)()
    runs[0].g = 0x1234
    runs[0].prog = _lib.gm_program(_lib.GM_PROG_BFS, _lib.GM_ORDER_OUT, 0.15, 0)
    runs[0].max_iters = 8
    assert lib.gm_plan_create(None, 1, None, ctypes.byref(out)) == _lib.GM_EINVAL
    assert lib.gm_plan_create(runs, 0, None, ctypes.byref(out)) == _lib.GM_EINVAL
    assert lib.gm_plan_create(runs, 1, None, ctypes.byref(out)) == _lib.GM_ESTATE
    assert out.value is None
    res = (_lib.gm_plan_result * 1)()
    assert lib.gm_plan_launch(bogus, None) == _lib.GM_ESTATE
    assert lib.gm_plan_results(bogus, res, None) == _lib.GM_ESTATE
    assert lib.gm_plan_destroy(bogus) == _lib.GM_ESTATE
    t = _lib.gm_tuning()
    assert lib.gm_graph_get_tuning(bogus, ctypes.byref(t)) == _lib.GM_ESTATE
    assert lib.gm_graph_set_tuning(bogus, ctypes.byref(t)) == _lib.GM_ESTATE
    prog = _lib.gm_program(_lib.GM_PROG_BFS, _lib.GM_ORDER_OUT, 0.15, 0)
    assert lib.gm_autotune(bogus, ctypes.byref(prog), 0, None, 0, -1, 3, None, None,
                           None) == _lib.GM_ESTATE
    assert lib.gm_autotune(bogus, ctypes.byref(prog), 0, None, 0, -1, 3, b"/tmp/x.json", None,
                           None) == _lib.GM_ESTATE


def test_prepare_release_multi_graph_validation_without_device(lib):
    bogus = ctypes.c_void_p(0x1234)
    prog = _lib.gm_program(_lib.GM_PROG_BFS, _lib.GM_ORDER_OUT, 0.15, 0)
    assert lib.gm_graph_prepare(bogus, ctypes.byref(prog), None) == _lib.GM_ESTATE
    assert lib.gm_graph_release(bogus) == _lib.GM_ESTATE
    graphs = (ctypes.c_void_p * 2)(0x1234, 0x5678)
    vprops = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    src = (ctypes.c_int32 * 2)(0, 0)
    it = ctypes.c_int32(0)
    run = lib.gm_run_multi_graph
    assert run(None, 2, ctypes.byref(prog), src, vprops, -1, ctypes.byref(it), None) == _lib.GM_EINVAL
    assert run(graphs, 0, ctypes.byref(prog), src, vprops, -1, None, None) == _lib.GM_EINVAL
    assert run(graphs, 2, ctypes.byref(prog), None, vprops, -1, None, None) == _lib.GM_EINVAL
    assert run(graphs, 2, ctypes.byref(prog), src, vprops, -1, None, None) == _lib.GM_ESTATE
    ppr = _lib.gm_program(_lib.GM_PROG_PPR, _lib.GM_ORDER_OUT, 0.15, 0)
    assert run(graphs, 2, ctypes.byref(ppr), src, vprops, 20, None, None) == _lib.GM_EUNSUPPORTED
    pr = _lib.gm_program(_lib.GM_PROG_PAGERANK, _lib.GM_ORDER_OUT, 0.15, 0)
    assert run(graphs, 2, ctypes.byref(pr), src, vprops, 20, None, None) == _lib.GM_EINVAL
    # a bitmap frontier and ids together are refused before the graph is read
    fr = _lib.gm_frontier(0x1000, 1, 0x2000)
    assert fr.bitmap == 0x2000


def test_binding_refuses_host_tensors():
    import torch
    # the library sees only an address: a host buffer must not reach it
    with pytest.raises(ValueError, match="device tensor"):
        gm._dev(torch.zeros(4, dtype=torch.float32), "vprop", 4, gm._F32)
    assert gm._dev(None, "active_out", 4, gm._I32) is None


class _DeviceStandIn:
    """Reports a device tensor's attributes without a GPU (the binding's
    checks read only these)."""

    def __init__(self, dtype, numel, contiguous=True):
        import types
        self.device = types.SimpleNamespace(type="cuda")
        self.dtype, self._n, self._c = dtype, numel, contiguous

    def numel(self):
        return self._n

    def is_contiguous(self):
        return self._c

    def data_ptr(self):
        return 0x1000


def test_binding_checks_dtype_length_and_layout():
    import torch
    ok = _DeviceStandIn(torch.int32, 10)
    assert gm._dev(ok, "vprop", 10, gm._I32) == 0x1000
    assert gm._dev(_DeviceStandIn(torch.uint32, 10), "vprop", 10, gm._I32) == 0x1000
    with pytest.raises(ValueError, match="elements"):
        gm._dev(ok, "vprop", 11, gm._I32)
    with pytest.raises(ValueError, match="dtype"):
        gm._dev(_DeviceStandIn(torch.float32, 10), "vprop", 10, gm._I32)
    with pytest.raises(ValueError, match="dtype"):
        gm._dev(_DeviceStandIn(torch.int32, 10), "counts", 10, gm._U64)
    with pytest.raises(ValueError, match="contiguous"):
        gm._dev(_DeviceStandIn(torch.float32, 10, contiguous=False), "hist", 10, gm._F32)
