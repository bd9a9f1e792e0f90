"""Cached synthetic workloads and oracle results shared by the tests.

Raw inputs come from the seeded generators (graphgen); expected values come
only from the oracle.
"""
from __future__ import annotations

import functools
import os

import numpy as np

import graphgen as gg
import oracle

# RMAT scale 14 is the small configuration the oracle finishes in
# milliseconds; scale 22 is the full-size single-source configuration.
SMALL_SCALE = 14
FULL_SCALE = 22


@functools.lru_cache(maxsize=None)
def raw(scale: int, seed: int = gg.SEED_RMAT):
    n, s, d = gg.rmat(scale, seed=seed)
    return n, s, d


@functools.lru_cache(maxsize=None)
def weights(scale: int, seed: int = gg.SEED_RMAT):
    _, s, d = raw(scale, seed)
    return gg.weights_u32(s, d)


@functools.lru_cache(maxsize=None)
def ograph(scale: int, mode: str, weighted: bool = False, seed: int = gg.SEED_RMAT):
    n, s, d = raw(scale, seed)
    return oracle.prepare(n, s, d, w=weights(scale, seed) if weighted else None, mode=mode)


@functools.lru_cache(maxsize=None)
def otranspose(scale: int, mode: str, seed: int = gg.SEED_RMAT):
    return ograph(scale, mode, False, seed).transpose()


@functools.lru_cache(maxsize=None)
def bfs_levels(scale: int, root: int = 0):
    return oracle.bfs(ograph(scale, "symmetric"), root)


@functools.lru_cache(maxsize=None)
def sssp_dist(scale: int, source: int = 0):
    return oracle.sssp(ograph(scale, "directed", True), source)


@functools.lru_cache(maxsize=None)
def sssp_supersteps(scale: int, source: int = 0) -> int:
    g = ograph(scale, "directed", True)
    prop = np.full(g.n, oracle.INF_U32, dtype=np.uint32)
    prop[source] = 0
    act = np.zeros(g.n, dtype=bool)
    act[source] = True
    return oracle.run_min_program(g, prop, act, weighted=True)[2]


@functools.lru_cache(maxsize=None)
def pagerank(scale: int, T: int = 20, r: float = 0.15):
    return oracle.pagerank(ograph(scale, "directed"), r, T, g_in=otranspose(scale, "directed"))


def max_rel_err(got, ref) -> float:
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref) / np.abs(ref))) if len(ref) else 0.0


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def sssp_hand_trace():
    """The hand-worked SSSP superstep trace of golden/sssp_supersteps_hand.txt:
    (n, src, dst, w, source, [(dist after k, active set after k), ...], supersteps)."""
    trace, n, src, dst, w, source, steps = [], 0, [], [], [], 0, 0
    for line in open(os.path.join(GOLDEN, "sssp_supersteps_hand.txt")):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if f[0] == "edges":
            e = np.array(f[1:], dtype=np.int64).reshape(-1, 3)
            src, dst, w = e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), e[:, 2].astype(np.uint32)
        elif f[0] == "n":
            n = int(f[1])
        elif f[0] == "source":
            source = int(f[1])
        elif f[0] == "after":
            a = f.index("active")
            dist = np.array([oracle.INF_U32 if x == "-" else int(x) for x in f[3:a]], np.uint32)
            act = np.zeros(n, dtype=bool)
            act[[int(x) for x in f[a + 1:]]] = True
            trace.append((dist, act))
        elif f[0] == "supersteps":
            steps = int(f[1])
    return n, src, dst, w, source, trace, steps
