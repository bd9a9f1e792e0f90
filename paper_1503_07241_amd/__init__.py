"""GraphMat generalized SpMSpV on AMD MI355X: Python binding of libgm.so.

Thin marshalling over the C ABI of ``include/gm.h``: every step of every
program runs in the library's HIP kernels. Device buffers are torch tensors
(``data_ptr()``); work is enqueued on ``torch.cuda.current_stream()``.

    import paper_1503_07241_amd as gm
    g = gm.Graph.from_coo(n, src, dst, prep=gm.GM_PREP_DROP_SELF_LOOPS | gm.GM_PREP_SYMMETRIZE)
    level = torch.full((n,), 2**31 - 1, dtype=torch.int32, device="cuda"); level[0] = 0
    iters = gm.run_vertex_program(g, gm.GM_PROG_BFS, torch.tensor([0], ...), -1, level)
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (GM_LAYOUT_IN, GM_LAYOUT_OUT, GM_ORDER_ALL, GM_ORDER_IN, GM_ORDER_OUT,  # noqa: F401
                   GM_PREP_DROP_SELF_LOOPS, GM_PREP_SYMMETRIZE, GM_PREP_UPPER_DAG, GM_PROG_BFS,
                   GM_PROG_DEGREE, GM_PROG_PAGERANK, GM_PROG_PPR, GM_PROG_SSSP, GM_PROG_TC,
                   GM_W_F32, GM_W_NONE,
                   GM_W_U32,
                   GmError)

INF_LEVEL = 2**31 - 1
INF_DIST = 2**32 - 1


def _stream(stream=None) -> int:
    if stream is not None:
        return int(stream)
    import torch
    if not torch.cuda.is_available():
        return 0  # the library reports the missing device itself
    return int(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("device buffers must be contiguous")
    return int(t.data_ptr())


def _dtypes(*names):
    import torch
    return tuple(getattr(torch, n) for n in names if hasattr(torch, n))


# Element types the library reads through each kind of device pointer
# (unsigned values may sit in signed tensors of the same width).
_I32 = ("int32", "uint32")
_U64 = ("int64", "uint64")
_F32 = ("float32",)
_F64 = ("float64",)


def _dev(t, name: str, numel: int, kinds) -> int | None:
    """Device pointer of tensor t after checking what the kernels will assume
    of it: on the GPU, of one of the element types `kinds`, contiguous, and
    at least `numel` elements long (the library sees only the address)."""
    if t is None:
        return None
    if t.device.type != "cuda":
        raise ValueError("%s must be a device tensor (got %s)" % (name, t.device))
    allowed = _dtypes(*kinds)
    if t.dtype not in allowed:
        raise ValueError("%s has dtype %s; expected one of %s" % (name, t.dtype, list(kinds)))
    if t.numel() < numel:
        raise ValueError("%s holds %d elements; the call needs %d" % (name, t.numel(), numel))
    return _ptr(t)


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


def read_mtx(path: str):
    """gm_mtx_read: (n, src, dst, w) host arrays of a Matrix Market file; w is
    None, uint32 or float32 by the file's field."""
    lib = _lib.load()
    n, m, wt = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int32(0)
    p = str(path).encode()
    _lib.check(lib.gm_mtx_read(p, ctypes.byref(n), ctypes.byref(m), None, None, None,
                               ctypes.byref(wt)), "gm_mtx_read")
    src = np.empty(m.value, dtype=np.int32)
    dst = np.empty(m.value, dtype=np.int32)
    w = None
    if wt.value == GM_W_U32:
        w = np.empty(m.value, dtype=np.uint32)
    elif wt.value == GM_W_F32:
        w = np.empty(m.value, dtype=np.float32)
    _lib.check(lib.gm_mtx_read(p, ctypes.byref(n), ctypes.byref(m), src.ctypes.data,
                               dst.ctypes.data, None if w is None else w.ctypes.data,
                               ctypes.byref(wt)), "gm_mtx_read")
    return int(n.value), src, dst, w


def version() -> str:
    return _lib.load().gm_version().decode()


class Graph:
    """A device graph (gm_graph handle); freed by close() or garbage collection."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)
        self._dims = None

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise GmError(_lib.GM_ESTATE, "Graph", "graph was closed")
        return self._h

    @classmethod
    def from_coo(cls, n: int, src, dst, w=None, prep: int = GM_PREP_DROP_SELF_LOOPS,
                 layouts: int = GM_LAYOUT_OUT | GM_LAYOUT_IN, stream=None) -> "Graph":
        """gm_graph_from_coo on host arrays src, dst (int32) and optional w
        (uint32 or float32)."""
        lib = _lib.load()
        s, sp = _host(src, np.int32)
        d, dp = _host(dst, np.int32)
        if len(s) != len(d):
            raise ValueError("src and dst differ in length")
        wtype, wp = GM_W_NONE, None
        if w is not None:
            w = np.asarray(w)
            if w.dtype == np.uint32:
                wtype = GM_W_U32
            elif w.dtype == np.float32:
                wtype = GM_W_F32
            else:
                raise ValueError("w must be uint32 or float32")
            w, wp = _host(w, w.dtype)
            if len(w) != len(s):
                raise ValueError("w differs in length from src")
        out = ctypes.c_void_p()
        _lib.check(lib.gm_graph_from_coo(n, len(s), sp, dp, wp, wtype, prep, layouts,
                                         _stream(stream), ctypes.byref(out)), "gm_graph_from_coo")
        return cls(out.value)

    @classmethod
    def from_mtx(cls, path: str, prep: int = GM_PREP_DROP_SELF_LOOPS,
                 layouts: int = GM_LAYOUT_OUT | GM_LAYOUT_IN, stream=None) -> "Graph":
        """gm_graph_from_mtx: a Matrix Market file (App. A, ReadMTX)."""
        out = ctypes.c_void_p()
        _lib.check(_lib.load().gm_graph_from_mtx(str(path).encode(), prep, layouts,
                                                 _stream(stream), ctypes.byref(out)),
                   "gm_graph_from_mtx")
        return cls(out.value)

    def info(self) -> _lib.gm_graph_info:
        info = _lib.gm_graph_info()
        _lib.check(_lib.load().gm_graph_get_info(self.handle, ctypes.byref(info)),
                   "gm_graph_get_info")
        return info

    def _nm(self):
        if self._dims is None:  # a graph's sizes never change
            info = self.info()
            self._dims = (info.n, info.m)
        return self._dims

    @property
    def n(self) -> int:
        return self._nm()[0]

    @property
    def m(self) -> int:
        return self._nm()[1]

    def edges(self, with_weights: bool = False):
        """Canonical (src, dst[, w]) host arrays, sorted by (src, dst)."""
        info = self.info()
        src = np.empty(info.m, dtype=np.int32)
        dst = np.empty(info.m, dtype=np.int32)
        w = None
        if with_weights:
            w = np.empty(info.m, dtype=np.uint32 if info.wtype == GM_W_U32 else np.float32)
        _lib.check(_lib.load().gm_graph_edges(self.handle, src.ctypes.data, dst.ctypes.data,
                                              None if w is None else w.ctypes.data),
                   "gm_graph_edges")
        return (src, dst, w) if with_weights else (src, dst)

    @classmethod
    def union(cls, parts, stream=None) -> "Graph":
        """gm_graph_union: block-diagonal union; part i's vertex v becomes
        base_i + v (see ``union_bases``)."""
        arr = (ctypes.c_void_p * len(parts))(*[p.handle.value for p in parts])
        out = ctypes.c_void_p()
        _lib.check(_lib.load().gm_graph_union(arr, len(parts), _stream(stream), ctypes.byref(out)),
                   "gm_graph_union")
        return cls(out.value)

    def tuning(self) -> dict:
        t = _lib.gm_tuning()
        _lib.check(_lib.load().gm_graph_get_tuning(self.handle, ctypes.byref(t)),
                   "gm_graph_get_tuning")
        return {f: int(getattr(t, f)) for f in _lib.TUNING_FIELDS}

    def set_tuning(self, **values) -> None:
        """gm_graph_set_tuning with the given fields changed."""
        cur = self.tuning()
        unknown = set(values) - set(cur)
        if unknown:
            raise ValueError("unknown tuning fields: %s" % sorted(unknown))
        cur.update(values)
        t = _lib.gm_tuning(*[cur[f] for f in _lib.TUNING_FIELDS])
        _lib.check(_lib.load().gm_graph_set_tuning(self.handle, ctypes.byref(t)),
                   "gm_graph_set_tuning")

    def prepare(self, kind: int, stream=None) -> None:
        """gm_graph_prepare: build now the schedules a run of `kind` needs."""
        prog = _lib.gm_program(kind, GM_ORDER_OUT, 0.15, 0)
        _lib.check(_lib.load().gm_graph_prepare(self.handle, ctypes.byref(prog), _stream(stream)),
                   "gm_graph_prepare")

    def release(self) -> None:
        """gm_graph_release: free the per-graph schedules and workspaces."""
        _lib.check(_lib.load().gm_graph_release(self.handle), "gm_graph_release")

    def last_run_stats(self) -> _lib.gm_run_stats:
        st = _lib.gm_run_stats()
        _lib.check(_lib.load().gm_last_run_stats(self.handle, ctypes.byref(st)),
                   "gm_last_run_stats")
        return st

    def close(self) -> None:
        if self._h is not None:
            _lib.check(_lib.load().gm_graph_destroy(self._h), "gm_graph_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_vertex_program(g: Graph, kind: int, frontier, max_iters: int, vprop, active_out=None,
                       r: float = 0.15, stream=None, bitmap=None, order: int = GM_ORDER_OUT) -> int:
    """gm_run_vertex_program. frontier: device int32 tensor of active ids (or
    None for PageRank); bitmap: instead of ids, a device int32/uint32 tensor
    of ceil(n / 32) words with bit v set for an active v; vprop: device
    property tensor (int32 levels, uint32 distances as int32 storage, float32
    ranks); order: GM_ORDER_OUT / IN / ALL, the edges messages travel
    along. Returns supersteps done."""
    prog = _lib.gm_program(kind, order, r, 0)
    n = g.n
    fr = None
    if bitmap is not None:
        if frontier is not None:
            raise ValueError("give frontier ids or a bitmap, not both")
        fr = _lib.gm_frontier(None, 0, _dev(bitmap, "bitmap", (n + 31) // 32, _I32))
    elif frontier is not None:
        fr = _lib.gm_frontier(_dev(frontier, "frontier", 0, _I32), frontier.numel(), None)
    pv = _dev(vprop, "vprop", n, _U64 if kind == GM_PROG_TC else
              _F32 if kind in (GM_PROG_PAGERANK, GM_PROG_PPR) else _I32)
    it = ctypes.c_int32(0)
    _lib.check(_lib.load().gm_run_vertex_program(
        g.handle, ctypes.byref(prog), None if fr is None else ctypes.byref(fr), max_iters,
        pv, _dev(active_out, "active_out", n, _I32), ctypes.byref(it), _stream(stream)),
        "gm_run_vertex_program")
    return it.value


def triangle_count(g: Graph, counts=None, stream=None) -> int:
    """gm_triangle_count: exact triangle total; per-vertex counts (device
    uint64 stored in an int64 tensor) are written to `counts` when given."""
    total = ctypes.c_uint64(0)
    _lib.check(_lib.load().gm_triangle_count(g.handle, _dev(counts, "counts", g.n, _U64),
                                             ctypes.byref(total),
                                             _stream(stream)), "gm_triangle_count")
    return int(total.value)


def run_batched(g: Graph, kind: int, sources, max_iters: int, vprop_block, r: float = 0.15,
                stream=None) -> int:
    """gm_run_batched: sources is a device int32 tensor of k ids; vprop_block a
    device (n, k) tensor (int32 levels, int32-stored uint32 distances, float32
    ranks) that the call initialises. Returns supersteps run."""
    prog = _lib.gm_program(kind, GM_ORDER_OUT, r, 0)
    it = ctypes.c_int32(0)
    k = sources.numel()
    pb = _dev(vprop_block, "vprop_block", g.n * k, _F32 if kind == GM_PROG_PPR else _I32)
    _lib.check(_lib.load().gm_run_batched(g.handle, ctypes.byref(prog),
                                          _dev(sources, "sources", k, _I32),
                                          k, max_iters, pb,
                                          ctypes.byref(it), _stream(stream)), "gm_run_batched")
    return it.value


def run_multi_graph(graphs, kind: int, sources, vprops, max_iters: int, r: float = 0.15,
                    stream=None) -> int:
    """gm_run_multi_graph: one run of `kind` over all graphs (their
    block-diagonal union); vprops[i] is graph i's device property tensor,
    initialised by the caller; sources: one id per graph (-1: none) for BFS
    and SSSP, None for PageRank and TC. Returns supersteps run."""
    k = len(graphs)
    if len(vprops) != k or (sources is not None and len(sources) != k):
        raise ValueError("one property tensor (and source) per graph")
    kinds = (_U64 if kind == GM_PROG_TC else
             _F32 if kind in (GM_PROG_PAGERANK, GM_PROG_PPR) else _I32)
    hs = (ctypes.c_void_p * k)(*[g.handle.value for g in graphs])
    vp = (ctypes.c_void_p * k)(*[_dev(v, "vprops[%d]" % i, graphs[i].n, kinds)
                                 for i, v in enumerate(vprops)])
    src = None
    if sources is not None:
        src = (ctypes.c_int32 * k)(*[int(x) for x in sources])
    prog = _lib.gm_program(kind, GM_ORDER_OUT, r, 0)
    it = ctypes.c_int32(0)
    _lib.check(_lib.load().gm_run_multi_graph(hs, k, ctypes.byref(prog), src, vp, max_iters,
                                              ctypes.byref(it), _stream(stream)),
               "gm_run_multi_graph")
    return it.value


def union_bases(parts) -> np.ndarray:
    """First vertex of each part in their union (plus the total at the end)."""
    return np.concatenate([[0], np.cumsum([p.n for p in parts])]).astype(np.int64)


def autotune(g: Graph, kind: int, ids=None, batched: bool = False, max_iters: int = -1,
             trials: int = 3, r: float = 0.15, stream=None, cache: str | None = None) -> dict:
    """gm_autotune: times the program for candidate schedule parameters and
    keeps the fastest on g; returns the parameters kept. cache: path of a
    JSON file of earlier choices (read first, extended after tuning)."""
    prog = _lib.gm_program(kind, GM_ORDER_OUT, r, 0)
    t = _lib.gm_tuning()
    count = 0 if ids is None else ids.numel()
    path = None if cache is None else str(cache).encode()
    _lib.check(_lib.load().gm_autotune(g.handle, ctypes.byref(prog), 1 if batched else 0,
                                       _dev(ids, "ids", count, _I32), count, max_iters, trials,
                                       path, ctypes.byref(t), _stream(stream)), "gm_autotune")
    return {f: int(getattr(t, f)) for f in _lib.TUNING_FIELDS}


class PlanRun:
    """One run of a Plan: `vprop` is the output tensor the plan initialises;
    `ids` the device int32 frontier / sources (None for PageRank and TC)."""

    def __init__(self, g: Graph, kind: int, vprop, ids=None, max_iters: int = 64,
                 batched: bool = False, r: float = 0.15):
        self.g, self.kind, self.vprop, self.ids = g, kind, vprop, ids
        self.max_iters, self.batched, self.r = max_iters, batched, r


class Plan:
    """gm_plan_*: runs recorded once as a HIP graph, replayed by launch().
    Keeps references to its graphs and tensors so they outlive it."""

    def __init__(self, runs, stream=None):
        self._keep = list(runs)
        arr = (_lib.gm_plan_run * len(runs))()
        for i, r in enumerate(runs):
            arr[i].g = r.g.handle.value
            arr[i].prog = _lib.gm_program(r.kind, GM_ORDER_OUT, r.r, 0)
            arr[i].batched = 1 if r.batched else 0
            arr[i].max_iters = r.max_iters
            count = 0 if r.ids is None else r.ids.numel()
            arr[i].ids = _dev(r.ids, "ids of run %d" % i, count, _I32)
            arr[i].count = count
            kinds = (_U64 if r.kind == GM_PROG_TC else
                     _F32 if r.kind in (GM_PROG_PAGERANK, GM_PROG_PPR) else _I32)
            arr[i].vprop = _dev(r.vprop, "vprop of run %d" % i,
                                r.g.n * (count if r.batched else 1), kinds)
        out = ctypes.c_void_p()
        _lib.check(_lib.load().gm_plan_create(arr, len(runs), _stream(stream), ctypes.byref(out)),
                   "gm_plan_create")
        self._h = out

    def launch(self, stream=None) -> None:
        _lib.check(_lib.load().gm_plan_launch(self._h, _stream(stream)), "gm_plan_launch")

    def results(self, stream=None):
        """[(iters_done, converged, edges_scanned)] of the last launch."""
        res = (_lib.gm_plan_result * len(self._keep))()
        _lib.check(_lib.load().gm_plan_results(self._h, res, _stream(stream)), "gm_plan_results")
        return [(r.iters_done, r.converged, r.edges_scanned) for r in res]

    def close(self) -> None:
        if self._h is not None:
            _lib.check(_lib.load().gm_plan_destroy(self._h), "gm_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# Differentiation (adjoint products) and torch.autograd wrappers
# --------------------------------------------------------------------------
class RatingGraph(Graph):
    """Rating matrix for collaborative filtering (gm_bipartite_from_coo)."""

    @classmethod
    def from_coo(cls, n_rows: int, n_cols: int, row, col, val, stream=None) -> "RatingGraph":
        r, rp = _host(row, np.int32)
        c, cp = _host(col, np.int32)
        v, vpp = _host(val, np.uint8)
        if not (len(r) == len(c) == len(v)):
            raise ValueError("row, col and val differ in length")
        out = ctypes.c_void_p()
        _lib.check(_lib.load().gm_bipartite_from_coo(n_rows, n_cols, len(r), rp, cp, vpp,
                                                     _stream(stream), ctypes.byref(out)),
                   "gm_bipartite_from_coo")
        g = cls(out.value)
        g.n_rows, g.n_cols = int(n_rows), int(n_cols)
        return g


def _factors(g: RatingGraph, PU, PV) -> int:
    """K of the factor matrices P_U (n_rows x K) and P_V (n_cols x K)."""
    if PU.dim() != 2 or PV.dim() != 2 or PU.shape[1] != PV.shape[1]:
        raise ValueError("PU and PV must be 2-D with the same number of columns")
    rows, cols = getattr(g, "n_rows", None), getattr(g, "n_cols", None)
    if rows is not None and (PU.shape[0] != rows or PV.shape[0] != cols):
        raise ValueError("PU must have %d rows and PV %d" % (rows, cols))
    return PU.shape[1]  # a graph that is no rating graph is refused by the library


def cf_forward(g: RatingGraph, PU, PV, lam: float, loss_out, stream=None) -> None:
    """gm_cf_forward: writes the Eq. (3) loss into loss_out (device float64[1])."""
    K = _factors(g, PU, PV)
    _lib.check(_lib.load().gm_cf_forward(g.handle, K, _dev(PU, "PU", PU.numel(), _F32),
                                         _dev(PV, "PV", PV.numel(), _F32), lam,
                                         _dev(loss_out, "loss_out", 1, _F64), _stream(stream)),
               "gm_cf_forward")


def cf_backward(g: RatingGraph, PU, PV, lam: float, scale: float, gPU=None, gPV=None,
                stream=None) -> None:
    """gm_cf_backward: scale * dL/dP_U into gPU, scale * dL/dP_V into gPV."""
    K = _factors(g, PU, PV)
    _lib.check(_lib.load().gm_cf_backward(g.handle, K, _dev(PU, "PU", PU.numel(), _F32),
                                          _dev(PV, "PV", PV.numel(), _F32), lam, scale,
                                          _dev(gPU, "gPU", PU.numel(), _F32),
                                          _dev(gPV, "gPV", PV.numel(), _F32), _stream(stream)),
               "gm_cf_backward")


def cf_gd(g: RatingGraph, PU, PV, lam: float, gamma: float, iters: int, loss_hist=None,
          stream=None) -> None:
    """gm_cf_gd: `iters` gradient-descent steps of Eqs. (5)-(6) on PU, PV in
    place; loss_hist (device float64[iters + 1]) receives the losses."""
    K = _factors(g, PU, PV)
    _lib.check(_lib.load().gm_cf_gd(g.handle, K, _dev(PU, "PU", PU.numel(), _F32),
                                    _dev(PV, "PV", PV.numel(), _F32), lam, gamma, iters,
                                    _dev(loss_hist, "loss_hist", iters + 1, _F64),
                                    _stream(stream)), "gm_cf_gd")


def pagerank_forward_w(g: Graph, w, r: float, T: int, hist, stream=None) -> None:
    """gm_pagerank_forward_w: hist[0] holds PR^0; rows 1..T are written."""
    n, m = g.n, g.m
    _lib.check(_lib.load().gm_pagerank_forward_w(g.handle, _dev(w, "w", m, _F32), r, T,
                                                 _dev(hist, "hist", (max(T, 0) + 1) * n, _F32),
                                                 _stream(stream)), "gm_pagerank_forward_w")


def pagerank_vjp_w(g: Graph, w, r: float, T: int, hist, grad_out, grad_w, stream=None) -> None:
    """gm_pagerank_vjp_w: grad_w = dL/dw given grad_out = dL/dPR^T."""
    n, m = g.n, g.m
    _lib.check(_lib.load().gm_pagerank_vjp_w(g.handle, _dev(w, "w", m, _F32), r, T,
                                             _dev(hist, "hist", (max(T, 0) + 1) * n, _F32),
                                             _dev(grad_out, "grad_out", n, _F32),
                                             _dev(grad_w, "grad_w", m, _F32), _stream(stream)),
               "gm_pagerank_vjp_w")


def _autograd():
    import torch

    class CFLoss(torch.autograd.Function):
        """L(P_U, P_V) of Eq. (3) on a RatingGraph; backward runs the row pass
        and the transpose (column) pass of the library."""

        @staticmethod
        def forward(ctx, PU, PV, g, lam):
            PU = PU.contiguous()
            PV = PV.contiguous()
            loss = torch.empty(1, dtype=torch.float64, device=PU.device)
            cf_forward(g, PU, PV, lam, loss)
            ctx.save_for_backward(PU, PV)
            ctx.g, ctx.lam = g, lam
            return loss[0]

        @staticmethod
        def backward(ctx, grad):
            PU, PV = ctx.saved_tensors
            gPU = torch.empty_like(PU) if ctx.needs_input_grad[0] else None
            gPV = torch.empty_like(PV) if ctx.needs_input_grad[1] else None
            if gPU is not None or gPV is not None:
                cf_backward(ctx.g, PU, PV, ctx.lam, float(grad), gPU, gPV)
            return gPU, gPV, None, None

    class PageRankW(torch.autograd.Function):
        """PR^T of the edge-weighted Eq. (1) (PR^0 = 1) as a function of the
        edge weights w (canonical order); backward is the adjoint SpMV."""

        @staticmethod
        def forward(ctx, w, g, r, T):
            w = w.contiguous()
            n = g.n
            hist = torch.empty((T + 1, n), dtype=torch.float32, device=w.device)
            hist[0].fill_(1.0)
            pagerank_forward_w(g, w, r, T, hist)
            ctx.save_for_backward(w, hist)
            ctx.g, ctx.r, ctx.T = g, r, T
            return hist[T].clone()

        @staticmethod
        def backward(ctx, grad_out):
            w, hist = ctx.saved_tensors
            gw = torch.empty_like(w)
            pagerank_vjp_w(ctx.g, w, ctx.r, ctx.T, hist, grad_out.contiguous().float(), gw)
            return gw, None, None, None

    return CFLoss, PageRankW


def __getattr__(name):
    if name in ("CFLoss", "PageRankW"):
        CFLoss, PageRankW = _autograd()
        globals()["CFLoss"], globals()["PageRankW"] = CFLoss, PageRankW
        return globals()[name]
    raise AttributeError(name)
