"""Seeded synthetic inputs shared by the GPU path's tests/bench and the CPU oracle.

Nothing here computes any part of GraphMat's method: the functions only draw
counter-based random numbers (SplitMix64 streams, see ``graphgen.c``) and
shape them into raw inputs of the paper's workloads (Sec. 5.1, Table 1):

* RMAT edge lists (Graph500 quadrant recursion, a/b/c/d parameters), raw:
  self-loops and duplicates are still present, preprocessing is the
  consumer's job;
* edge weights drawn per ordered vertex pair (duplicates share a weight);
* source/seed vertex sets;
* a bipartite user x item rating graph shaped like the Netflix matrix;
* dense factor matrices and upstream gradients.

The compiled helper ``libgraphgen.so`` is built from ``graphgen.c`` with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None

# RMAT parameters of the paper's PageRank/BFS/SSSP graphs (Sec. 5.1).
RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19
EDGE_FACTOR = 16

# Seeds (the paper names none).
SEED_RMAT = 1
SEED_WEIGHTS = 2
SEED_BATCH_SOURCES = 3
SEED_PPR_SEEDS = 4
SEED_CF_DEGREE = 5
SEED_CF_ITEMS = 6
SEED_CF_TRUE = 7
SEED_CF_NOISE = 8
SEED_CF_POINT = 9
SEED_PR_UPSTREAM = 10
SEED_SCRAMBLE = 11
SEED_MIXED_BASE = 100


def build(force: bool = False) -> str:
    """Compile libgraphgen.so with gcc (OpenMP) and return its path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        )
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
        i32, i64, u64, f64, vp = (
            ctypes.c_int32,
            ctypes.c_int64,
            ctypes.c_uint64,
            ctypes.c_double,
            ctypes.c_void_p,
        )
        lib.gg_rmat.argtypes = [i32, i64, f64, f64, f64, u64, vp, vp]
        lib.gg_rmat.restype = None
        lib.gg_weights_u32.argtypes = [i64, vp, vp, u64, ctypes.c_uint32, ctypes.c_uint32, vp]
        lib.gg_weights_u32.restype = None
        lib.gg_weights_f32.argtypes = [i64, vp, vp, u64, f64, f64, vp]
        lib.gg_weights_f32.restype = None
        lib.gg_uniform_f32.argtypes = [i64, u64, f64, f64, vp]
        lib.gg_uniform_f32.restype = None
        lib.gg_normal_f32.argtypes = [i64, u64, f64, vp]
        lib.gg_normal_f32.restype = None
        lib.gg_sources.argtypes = [i64, i64, vp, vp, i64, u64, i32, vp]
        lib.gg_sources.restype = i64
        lib.gg_cf_degrees.argtypes = [i64, i64, i64, f64, i64, u64, vp]
        lib.gg_cf_degrees.restype = ctypes.c_int
        lib.gg_cf_ratings.argtypes = [i64, i64, vp, f64, u64, i32, vp, vp, f64, vp, vp]
        lib.gg_cf_ratings.restype = ctypes.c_int
        lib.gg_rng_u64.argtypes = [u64, u64, u64]
        lib.gg_rng_u64.restype = u64
        _lib = lib
    return _lib


def _p(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def rng_u64(seed: int, stream: int, i: int) -> int:
    """Raw output i of counter-based stream (seed, stream)."""
    return int(_load().gg_rng_u64(seed, stream, i))


def rmat(scale: int, edge_factor: int = EDGE_FACTOR, a: float = RMAT_A, b: float = RMAT_B,
         c: float = RMAT_C, seed: int = SEED_RMAT, m: int | None = None):
    """Raw RMAT edge list with 2**scale vertices and edge_factor * 2**scale edges.

    Returns (n, src, dst) with int32 arrays; self-loops and duplicates kept.
    """
    n = 1 << scale
    if m is None:
        m = edge_factor * n
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    _load().gg_rmat(scale, m, a, b, c, seed, _p(src), _p(dst))
    return n, src, dst


def weights_u32(src: np.ndarray, dst: np.ndarray, seed: int = SEED_WEIGHTS, lo: int = 1,
                hi: int = 255) -> np.ndarray:
    """Integer weights uniform in [lo, hi], one per ordered vertex pair."""
    w = np.empty(len(src), dtype=np.uint32)
    _load().gg_weights_u32(len(src), _p(src), _p(dst), seed, lo, hi, _p(w))
    return w


def weights_f32(src: np.ndarray, dst: np.ndarray, seed: int, lo: float, hi: float) -> np.ndarray:
    """Real weights uniform in [lo, hi), one per ordered vertex pair."""
    w = np.empty(len(src), dtype=np.float32)
    _load().gg_weights_f32(len(src), _p(src), _p(dst), seed, lo, hi, _p(w))
    return w


def uniform_f32(n: int, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    out = np.empty(n, dtype=np.float32)
    _load().gg_uniform_f32(n, seed, lo, hi, _p(out))
    return out


def normal_f32(n: int, seed: int, std: float = 1.0) -> np.ndarray:
    out = np.empty(n, dtype=np.float32)
    _load().gg_normal_f32(n, seed, std, _p(out))
    return out


def label_permutation(n: int, seed: int = SEED_SCRAMBLE) -> np.ndarray:
    """A seeded random permutation of [0, n) (vertex v becomes perm[v]): the
    vertices ordered by uniform keys of stream (seed, 0), ties by label."""
    keys = uniform_f32(n, seed)
    order = np.argsort(keys, kind="stable")  # order[j] = vertex taking label j
    perm = np.empty(n, dtype=np.int32)
    perm[order] = np.arange(n, dtype=np.int32)
    return perm


def sources(n: int, src: np.ndarray, dst: np.ndarray, k: int, seed: int,
            first: int = 0) -> np.ndarray:
    """k distinct vertices that own a non-loop out-edge in the raw list; `first` leads."""
    out = np.empty(k, dtype=np.int32)
    got = _load().gg_sources(n, len(src), _p(src), _p(dst), k, seed, first, _p(out))
    if got < 0:
        raise MemoryError("gg_sources")
    return out[:got]


@dataclass
class Ratings:
    """Bipartite rating graph: users are rows, items are columns."""
    n_users: int
    n_items: int
    user: np.ndarray    # int32[m], nondecreasing
    item: np.ndarray    # int32[m], increasing within a user
    rating: np.ndarray  # uint8[m] in 1..5

    @property
    def m(self) -> int:
        return len(self.item)


# Shape of the Netflix prize matrix (Table 1) and the degree law fitted to it.
NETFLIX_USERS, NETFLIX_ITEMS, NETFLIX_RATINGS = 480_189, 17_770, 100_000_000
CF_DMIN, CF_GAMMA, CF_ITEM_ALPHA, CF_NOISE_SIGMA, CF_K = 10, 1.677, 0.5, 0.5, 32


def cf_ratings(n_users: int = NETFLIX_USERS, n_items: int = NETFLIX_ITEMS,
               total: int = NETFLIX_RATINGS, dmin: int = CF_DMIN, gamma: float = CF_GAMMA,
               alpha: float = CF_ITEM_ALPHA, k: int = CF_K, sigma: float = CF_NOISE_SIGMA,
               seeds=(SEED_CF_DEGREE, SEED_CF_ITEMS, SEED_CF_TRUE, SEED_CF_NOISE)) -> Ratings:
    """Synthetic rating graph: power-law user degrees summing to `total`, items
    drawn by popularity without replacement, ratings from a rank-k factor model
    plus N(0, sigma^2) noise, rounded and clipped to 1..5."""
    lib = _load()
    deg = np.empty(n_users, dtype=np.int64)
    dmax = n_items
    if lib.gg_cf_degrees(n_users, dmin, dmax, gamma, total, seeds[0], _p(deg)) != 0:
        raise ValueError("cf degrees: total out of range")
    off = np.zeros(n_users + 1, dtype=np.int64)
    np.cumsum(deg, out=off[1:])
    std = float(k) ** -0.25  # factor entries ~ N(0, k^-1/2): u*.v* has unit variance
    ustar = normal_f32(n_users * k, seeds[2] * 1000 + 1, std)
    vstar = normal_f32(n_items * k, seeds[2] * 1000 + 2, std)
    item = np.empty(total, dtype=np.int32)
    rating = np.empty(total, dtype=np.uint8)
    if lib.gg_cf_ratings(n_users, n_items, _p(off), alpha, seeds[1], k, _p(ustar), _p(vstar),
                         sigma, _p(item), _p(rating)) != 0:
        raise MemoryError("cf ratings")
    user = np.repeat(np.arange(n_users, dtype=np.int32), deg)
    return Ratings(n_users, n_items, user, item, rating)


def cf_point(n_users: int, n_items: int, k: int = CF_K, seed: int = SEED_CF_POINT):
    """Evaluation point (P_U, P_V): iid N(0, k^-1/2) entries, float32 row-major."""
    std = float(k) ** -0.25
    pu = normal_f32(n_users * k, seed * 1000 + 1, std).reshape(n_users, k)
    pv = normal_f32(n_items * k, seed * 1000 + 2, std).reshape(n_items, k)
    return pu, pv


def grid2d(rows: int, cols: int):
    """A rows x cols 4-neighbour grid as a directed edge list with both
    directions of every grid edge: vertex (i, j) is i * cols + j. Returns
    (n, src, dst), int32 arrays. A long-diameter graph (rows + cols - 2
    hops corner to corner), the shape of road networks' long paths."""
    n = rows * cols
    v = np.arange(n, dtype=np.int64).reshape(rows, cols)
    right = (v[:, :-1].ravel(), v[:, 1:].ravel())
    down = (v[:-1, :].ravel(), v[1:, :].ravel())
    a = np.concatenate([right[0], down[0]])
    b = np.concatenate([right[1], down[1]])
    src = np.concatenate([a, b]).astype(np.int32)
    dst = np.concatenate([b, a]).astype(np.int32)
    return n, src, dst


def mixed_batch_specs(count: int = 32, base_scale: int = 12, span: int = 7):
    """(scale, seed) of the graphs of the mixed batch: scale 12 + (i mod 7)."""
    return [(base_scale + (i % span), SEED_MIXED_BASE + i) for i in range(count)]
