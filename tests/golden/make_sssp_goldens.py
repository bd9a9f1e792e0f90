"""Write the expected SSSP results of the paper's SSSP workloads.

Calls only the oracle (and the seeded input generators). For each workload:
the number of reached vertices, the largest distance, the SHA-256 of the
whole uint32 distance array (little-endian; UINT32_MAX = unreached) from the
oracle's Dijkstra (Sec. 3 V, Eq. (8)), and the number of Alg. 2 supersteps
from the oracle's superstep loop, whose distances must equal Dijkstra's.

  sssp_rmat24_a50: RMAT scale 24, a = .50, b = c = .10 (the paper's
    GPU-comparison graph, Sec. 5.1 Table 1), edge factor 16, seed 1, weights
    uint32 uniform in [1, 255] per ordered pair (seed 2), source 0;
  sssp_grid2048: a 2048 x 2048 4-neighbour grid, both directions of each
    grid edge, weights as above, source 0 (a long-diameter graph: road-like
    path lengths, thousands of supersteps).

Usage: python tests/golden/make_sssp_goldens.py [name ...]  (minutes)
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def workload(name: str):
    """(n, src, dst, w, description) of a named SSSP workload."""
    if name == "sssp_rmat24_a50":
        n, s, d = gg.rmat(24, a=0.50, b=0.10, c=0.10)
        desc = "RMAT scale 24, a=.50 b=c=.10, edge factor 16, seed 1"
    elif name == "sssp_grid2048":
        n, s, d = gg.grid2d(2048, 2048)
        desc = "2048 x 2048 grid, 4-neighbour, both directions"
    else:
        raise KeyError(name)
    return n, s, d, gg.weights_u32(s, d), desc


WORKLOADS = ("sssp_rmat24_a50", "sssp_grid2048")


def make(name: str) -> str:
    t0 = time.time()
    n, s, d, w, desc = workload(name)
    g = oracle.prepare(n, s, d, w=w)
    dist = oracle.sssp(g, 0)
    prop = np.full(n, oracle.INF_U32, dtype=np.uint32)
    prop[0] = 0
    act = np.zeros(n, dtype=bool)
    act[0] = True
    sup, left, steps = oracle.run_min_program(g, prop, act, weighted=True)
    assert np.array_equal(sup, dist) and not left.any(), name
    reached = dist != oracle.INF_U32
    digest = hashlib.sha256(np.ascontiguousarray(dist, dtype="<u4").tobytes()).hexdigest()
    path = os.path.join(HERE, name + ".txt")
    with open(path, "w") as f:
        f.write("# SSSP from vertex 0 (Sec. 3 V, Eq. (8)) on %s;\n" % desc)
        f.write("# self-loops dropped, duplicates merged (smallest weight); weights uint32\n")
        f.write("# uniform in [1, 255] per ordered pair (seed 2). Written by\n")
        f.write("# tests/golden/make_sssp_goldens.py from the oracle only (Dijkstra; the\n")
        f.write("# superstep count from its Alg. 2 loop, which reaches the same distances).\n")
        f.write("n %d\nm %d\n" % (n, g.m))
        f.write("reached %d\n" % int(reached.sum()))
        f.write("max_dist %d\n" % int(dist[reached].max()))
        f.write("supersteps %d\n" % steps)
        f.write("dist_sha256 %s\n" % digest)
    print("%s: m %d, reached %d, supersteps %d (%.0f s)" % (name, g.m, int(reached.sum()), steps,
                                                           time.time() - t0), flush=True)
    return path


def read(name: str) -> dict:
    out = {}
    with open(os.path.join(HERE, name + ".txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            out[k] = v if k.endswith("sha256") else int(v)
    return out


if __name__ == "__main__":
    for nm in sys.argv[1:] or WORKLOADS:
        make(nm)
