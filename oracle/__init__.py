"""CPU oracle for the GraphMat generalized-SpMSpV path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg; never by the product package, which must
fail loudly rather than fall back to anything here. It shares no code with
the GPU path: preprocessing is numpy (a sort/unique is the only library
primitive used), the algorithms are the plain single-threaded C in
``oracle.c`` (liboracle.so, built with gcc).

Paper: Sundaram et al., "GraphMat: High performance graph analytics made
productive", VLDB 2015 (arXiv 1503.07241). Function docstrings name the
section or equation each follows.

Pinned by the tests in ``tests/test_oracle_*.py`` against closed forms,
brute force, invariants and independent library routines. Parity unpinned:
nothing in this module (every function has at least one independent pin).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

INF_I32 = np.iinfo(np.int32).max
INF_U32 = np.iinfo(np.uint32).max


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (single-threaded, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            # built only by __graft_entry__.build() (or build() called
            # directly): a process that already uses the GPU never starts a
            # compiler
            raise RuntimeError("%s is not built: run __graft_entry__.build()" % _LIB)
        lib = ctypes.CDLL(_LIB)
        i32, i64, f64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        lib.orc_bfs.argtypes = [i64, vp, vp, i64, vp, vp]
        lib.orc_bfs.restype = i32
        lib.orc_dijkstra.argtypes = [i64, vp, vp, vp, i64, vp, vp]
        lib.orc_dijkstra.restype = ctypes.c_int
        lib.orc_run_min_program.argtypes = [i64, vp, vp, vp, vp, vp, i32]
        lib.orc_run_min_program.restype = i32
        lib.orc_pagerank.argtypes = [i64, vp, vp, vp, vp, f64, i32, vp, vp]
        lib.orc_pagerank.restype = ctypes.c_int
        lib.orc_pagerank_vjp_w.argtypes = [i64, vp, vp, vp, f64, i32, vp, vp, vp]
        lib.orc_pagerank_vjp_w.restype = ctypes.c_int
        lib.orc_tc_per_vertex.argtypes = [i64, vp, vp, i64, vp, vp]
        lib.orc_tc_per_vertex.restype = ctypes.c_int
        lib.orc_tc_total.argtypes = [i64, vp, vp]
        lib.orc_tc_total.restype = ctypes.c_uint64
        lib.orc_cf.argtypes = [i64, i64, i64, vp, vp, vp, i32, vp, vp, f64, vp, vp, vp]
        lib.orc_cf.restype = ctypes.c_int
        lib.orc_bfs_certificate.argtypes = [i64, i64, vp, vp, vp, i32, i32]
        lib.orc_bfs_certificate.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a) -> int | None:
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be contiguous"
    return a.ctypes.data


# --------------------------------------------------------------------------
# Graphs and preprocessing (Sec. 5.1: self-loops removed; PageRank and SSSP
# on the directed graph; BFS on the symmetrised graph; triangle counting on
# the symmetrised graph with the lower triangle discarded).
# --------------------------------------------------------------------------
@dataclass
class Graph:
    """Compressed adjacency: row u lists idx[off[u]:off[u+1]] (sorted)."""
    n: int
    off: np.ndarray            # int64[n+1]
    idx: np.ndarray            # int32[m]
    w: np.ndarray | None = None  # per-edge weight in the same order

    @property
    def m(self) -> int:
        return int(self.off[-1])

    def rows(self) -> np.ndarray:
        """Row id of every stored entry (int64[m])."""
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.off))

    def degree(self) -> np.ndarray:
        return np.diff(self.off)

    def transpose(self) -> "Graph":
        """The same edges indexed by column: entry (u, v) becomes row v."""
        r = self.rows()
        c = self.idx.astype(np.int64)
        order = np.lexsort((r, c))  # by column, then row
        off = np.zeros(self.n + 1, dtype=np.int64)
        np.cumsum(np.bincount(c, minlength=self.n), out=off[1:])
        w = None if self.w is None else np.ascontiguousarray(self.w[order])
        return Graph(self.n, off, np.ascontiguousarray(r[order].astype(np.int32)), w)


def prepare(n: int, src: np.ndarray, dst: np.ndarray, w: np.ndarray | None = None,
            mode: str = "directed") -> Graph:
    """Raw edge list -> simple graph as row-compressed out-adjacency.

    mode: 'directed' (drop self-loops, merge duplicates), 'symmetric' (also add
    every reverse edge) or 'dag' (symmetric, then keep only u < v). Duplicate
    edges keep the smallest weight.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    s, d = src[keep], dst[keep]
    ww = None if w is None else np.asarray(w)[keep]
    if mode in ("symmetric", "dag"):
        s, d = np.concatenate([s, d]), np.concatenate([d, s])
        if ww is not None:
            ww = np.concatenate([ww, ww])
    if mode == "dag":
        up = s < d
        s, d = s[up], d[up]
        if ww is not None:
            ww = ww[up]
    elif mode not in ("directed", "symmetric"):
        raise ValueError(mode)
    key = s * n + d
    if ww is None:
        key = np.unique(key)
        wout = None
    else:
        order = np.argsort(key, kind="stable")
        key_s = key[order]
        first = np.ones(len(key_s), dtype=bool)
        first[1:] = key_s[1:] != key_s[:-1]
        heads = np.flatnonzero(first)
        key = key_s[heads]
        w_s = ww[order]
        wout = np.ascontiguousarray(np.minimum.reduceat(w_s, heads) if len(heads) else w_s[:0])
    rows = key // n
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=off[1:])
    return Graph(n, off, np.ascontiguousarray((key % n).astype(np.int32)), wout)


# --------------------------------------------------------------------------
# Programs
# --------------------------------------------------------------------------
def bfs(g: Graph, roots) -> np.ndarray:
    """Hop distance from the roots (Sec. 3 II, Eq. (2)); INT32_MAX if unreached."""
    roots = np.ascontiguousarray(np.atleast_1d(roots).astype(np.int32))
    level = np.empty(g.n, dtype=np.int32)
    if _load().orc_bfs(g.n, _p(g.off), _p(g.idx), len(roots), _p(roots), _p(level)) < 0:
        raise MemoryError
    return level


def sssp(g: Graph, sources) -> np.ndarray:
    """Shortest-path distances (Sec. 3 V, Eq. (8)) by Dijkstra; UINT32_MAX if unreached."""
    srcs = np.ascontiguousarray(np.atleast_1d(sources).astype(np.int32))
    assert g.w is not None and g.w.dtype == np.uint32
    dist = np.empty(g.n, dtype=np.uint32)
    if _load().orc_dijkstra(g.n, _p(g.off), _p(g.idx), _p(g.w), len(srcs), _p(srcs), _p(dist)):
        raise MemoryError
    return dist


def run_min_program(g: Graph, prop: np.ndarray, active: np.ndarray, weighted: bool,
                    max_iters: int = -1):
    """Alg. 2 supersteps with the Alg. 1 SpMV for BFS (weighted=False) or SSSP.

    prop: uint32 vertex property (INF = UINT32_MAX), updated copy returned;
    active: bool mask of initially active vertices. Returns (prop, active, iters).
    """
    prop = np.ascontiguousarray(prop.astype(np.uint32).copy())
    act = np.ascontiguousarray(active.astype(np.uint8).copy())
    w = None
    if weighted:
        assert g.w is not None
        w = np.ascontiguousarray(g.w.astype(np.uint32))
    it = _load().orc_run_min_program(g.n, _p(g.off), _p(g.idx), _p(w), _p(prop), _p(act),
                                     max_iters)
    if it < 0:
        raise MemoryError
    return prop, act.astype(bool), int(it)


def pagerank_history(g: Graph, r: float = 0.15, T: int = 20, w: np.ndarray | None = None,
                     tele: np.ndarray | None = None, pr0: np.ndarray | None = None,
                     g_in: Graph | None = None) -> np.ndarray:
    """PR^0..PR^T of Eq. (1) (float64, shape (T+1, n)).

    PR^{t+1}(v) = r*tele(v) + (1-r) * sum_{u->v} w_uv PR^t(u)/outdeg(u), with
    tele = 1 and w = 1 by default (exactly Eq. (1)); PR^0 = 1 (Sec. 3 I).
    w is given in the out-adjacency (CSR) edge order of g; alternatively a
    prebuilt in-adjacency g_in may carry the edge values in its own order (g
    then serves only for the out-degrees).
    """
    n = g.n
    if w is not None:
        g_in = Graph(g.n, g.off, g.idx, np.asarray(w, dtype=np.float64)).transpose()
        in_w = np.ascontiguousarray(g_in.w)
    else:
        if g_in is None:
            g_in = g.transpose()
        # edge values may come with a prebuilt in-adjacency (in its own order)
        in_w = None if g_in.w is None else np.ascontiguousarray(g_in.w, dtype=np.float64)
    outdeg = np.ascontiguousarray(np.diff(g.off).astype(np.int64))
    tele = np.ones(n) if tele is None else np.asarray(tele, dtype=np.float64)
    hist = np.empty((T + 1, n), dtype=np.float64)
    hist[0] = 1.0 if pr0 is None else pr0
    _load().orc_pagerank(n, _p(g_in.off), _p(g_in.idx), _p(in_w), _p(outdeg), r, T,
                         _p(np.ascontiguousarray(tele)), _p(hist))
    return hist


def pagerank(g: Graph, r: float = 0.15, T: int = 20, **kw) -> np.ndarray:
    """PR^T of Eq. (1) in float64."""
    return pagerank_history(g, r, T, **kw)[-1]


def personalized_pagerank(g: Graph, seed: int, r: float = 0.15, T: int = 20,
                          g_in: Graph | None = None) -> np.ndarray:
    """PPR_s^T: teleport only to the seed, PPR_s^0 = e_s (a reading; not in the paper)."""
    tele = np.zeros(g.n)
    tele[seed] = 1.0
    return pagerank_history(g, r, T, tele=tele, pr0=tele, g_in=g_in)[-1]


def pagerank_vjp_w(g: Graph, w: np.ndarray, c: np.ndarray, r: float = 0.15, T: int = 20,
                   hist: np.ndarray | None = None) -> np.ndarray:
    """dL/dw (CSR edge order) for L with dL/dPR^T = c, weighted Eq. (1) forward."""
    w64 = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    if hist is None:
        hist = pagerank_history(g, r, T, w=w64)
    hist = np.ascontiguousarray(hist, dtype=np.float64)
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
    grad = np.empty(g.m, dtype=np.float64)
    if _load().orc_pagerank_vjp_w(g.n, _p(g.off), _p(g.idx), _p(w64), r, T, _p(hist), _p(c),
                                  _p(grad)):
        raise MemoryError
    return grad


def bfs_certificate(n: int, src: np.ndarray, dst: np.ndarray, levels: np.ndarray,
                    root: int) -> int:
    """0 iff `levels` are the BFS hop distances from `root` (Sec. 3 II,
    Eq. (2)) on the undirected graph whose directed entries are (src, dst),
    both directions listed; else the code of the first failed condition
    (see oracle.c). Linear in the number of entries, so it checks results at
    any size."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    lv = np.ascontiguousarray(levels, dtype=np.int32)
    return int(_load().orc_bfs_certificate(n, len(src), _p(src), _p(dst), _p(lv), root, INF_I32))


def pagerank_step_rows(prev: np.ndarray, outdeg: np.ndarray, src: np.ndarray, dst: np.ndarray,
                       rows: np.ndarray, r: float = 0.15, w: np.ndarray | None = None) -> np.ndarray:
    """One superstep of Eq. (1) (with edge weights w when given) for the
    listed rows only, in FP64: r + (1 - r) * sum over the edges (u -> v) with
    v a listed row of w_uv * prev[u] / outdeg(u). (src, dst[, w]) must hold
    every in-edge of the listed rows (other edges are ignored)."""
    rows = np.asarray(rows, dtype=np.int64)
    order = np.argsort(rows, kind="stable")
    y = np.zeros(len(rows), dtype=np.float64)
    mark = np.zeros(len(prev), dtype=bool)
    mark[rows] = True
    sel = mark[dst]
    su = src[sel].astype(np.int64)
    sv = dst[sel].astype(np.int64)
    val = prev[su].astype(np.float64) / outdeg[su].astype(np.float64)
    if w is not None:
        val = val * w[sel].astype(np.float64)
    np.add.at(y, order[np.searchsorted(rows[order], sv)], val)
    return r + (1.0 - r) * y


def degree(g: Graph, order: str = "out") -> np.ndarray:
    """The degree program of Fig. 1 (an SpMV of the adjacency with a ones
    vector) by counting: messages along out-edges reach each vertex once per
    in-edge, so order 'out' gives in-degrees; 'in' gives out-degrees; 'all'
    their sum (int64)."""
    indeg = np.bincount(g.idx, minlength=g.n).astype(np.int64)
    outdeg = np.diff(g.off).astype(np.int64)
    return {"out": indeg, "in": outdeg, "all": indeg + outdeg}[order]


def cf_gd(n_users: int, n_items: int, user, item, rating, PU, PV, lam: float, gamma: float,
          iters: int):
    """Gradient descent of Eqs. (5)-(6) in float64: both factor matrices
    updated from the same point, p <- p - (gamma / 2) dL/dp (the paper's
    p + gamma (sum e p_other - lambda p)), `iters` times. Returns (PU, PV,
    losses) with losses[t] = L at the point of step t (t = 0..iters)."""
    pu = np.array(PU, dtype=np.float64)
    pv = np.array(PV, dtype=np.float64)
    losses = []
    for _ in range(iters):
        L, gu, gv = _cf_loss_grad64(n_users, n_items, user, item, rating, pu, pv, lam)
        losses.append(L)
        pu = pu - 0.5 * gamma * gu
        pv = pv - 0.5 * gamma * gv
    losses.append(_cf_loss_grad64(n_users, n_items, user, item, rating, pu, pv, lam)[0])
    return pu, pv, np.array(losses)


def _cf_loss_grad64(n_users, n_items, user, item, rating, pu, pv, lam):
    """Eq. (3) loss and gradients at float64 factors (numpy, one pass)."""
    user = np.asarray(user, dtype=np.int64)
    item = np.asarray(item, dtype=np.int64)
    e = np.asarray(rating, dtype=np.float64) - np.einsum("ij,ij->i", pu[user], pv[item])
    L = float(e @ e + lam * (np.sum(pu * pu) + np.sum(pv * pv)))
    gu = 2.0 * lam * pu
    gv = 2.0 * lam * pv
    np.add.at(gu, user, -2.0 * e[:, None] * pv[item])
    np.add.at(gv, item, -2.0 * e[:, None] * pu[user])
    return L, gu, gv


def dag_in_lists(dag: Graph) -> Graph:
    """Program 1 of the triangle count (Sec. 4.2): sorted in-neighbour lists."""
    return dag.transpose()


def triangle_count(dag: Graph, dag_in: Graph | None = None) -> int:
    """N_triangles of Eq. (7) via the two-program DAG form (Sec. 4.2)."""
    if dag_in is None:
        dag_in = dag_in_lists(dag)
    return int(_load().orc_tc_total(dag.n, _p(dag_in.off), _p(dag_in.idx)))


def triangles_at(dag_in: Graph, verts) -> np.ndarray:
    """Per-receiver counts sum_{u in in(v)} |in(u) ∩ in(v)| for the listed v."""
    verts = np.ascontiguousarray(np.atleast_1d(verts).astype(np.int32))
    out = np.empty(len(verts), dtype=np.uint64)
    _load().orc_tc_per_vertex(dag_in.n, _p(dag_in.off), _p(dag_in.idx), len(verts), _p(verts),
                              _p(out))
    return out


def cf_loss_grad(n_users: int, n_items: int, user: np.ndarray, item: np.ndarray,
                 rating: np.ndarray, PU: np.ndarray, PV: np.ndarray, lam: float):
    """Eq. (3) loss and its gradients w.r.t. P_U and P_V (float64)."""
    K = PU.shape[1]
    user = np.ascontiguousarray(user, dtype=np.int32)
    item = np.ascontiguousarray(item, dtype=np.int32)
    rating = np.ascontiguousarray(rating, dtype=np.uint8)
    PU = np.ascontiguousarray(PU, dtype=np.float32)
    PV = np.ascontiguousarray(PV, dtype=np.float32)
    gU = np.empty((n_users, K), dtype=np.float64)
    gV = np.empty((n_items, K), dtype=np.float64)
    loss = ctypes.c_double(0.0)
    _load().orc_cf(n_users, n_items, len(user), _p(user), _p(item), _p(rating), K, _p(PU),
                   _p(PV), lam, ctypes.addressof(loss), _p(gU), _p(gV))
    return float(loss.value), gU, gV
