"""Write the expected triangle counts of the full-size RMAT workloads.

Calls only the oracle (and the seeded input generators): for each workload
it runs the oracle's per-receiver count of Eq. (7) (two-program DAG form,
Sec. 4.2) over every vertex and stores the total (their sum) and the
SHA-256 of the whole per-vertex uint64 array (little-endian), so a test can
check every receiver's count without storing the array.

Usage: python tests/golden/make_tc_goldens.py [name ...]   (default: all)
Takes minutes per workload on one core (scale 22: about five).
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

# name -> (scale, a, b, c, description)
WORKLOADS = {
    # the full-size single-source workload: RMAT scale 22, a/b/c = .57/.19/.19
    "tc_rmat22": (22, gg.RMAT_A, gg.RMAT_B, gg.RMAT_C,
                  "RMAT scale 22, a=.57 b=c=.19, edge factor 16, seed 1"),
    # the paper's triangle-counting graph (Sec. 5.1, Table 1): scale 20, a=.45 b=c=.15
    "tc_rmat20_a45": (20, 0.45, 0.15, 0.15,
                      "RMAT scale 20, a=.45 b=c=.15, edge factor 16, seed 1"),
}


def make(name: str) -> str:
    scale, a, b, c, desc = WORKLOADS[name]
    t0 = time.time()
    n, s, d = gg.rmat(scale, a=a, b=b, c=c)
    dag = oracle.prepare(n, s, d, mode="dag")
    dag_in = oracle.dag_in_lists(dag)
    counts = oracle.triangles_at(dag_in, np.arange(n, dtype=np.int32))
    total = int(counts.sum(dtype=np.uint64))
    digest = hashlib.sha256(np.ascontiguousarray(counts, dtype="<u8").tobytes()).hexdigest()
    path = os.path.join(HERE, name + ".txt")
    with open(path, "w") as f:
        f.write("# Triangle counts (Eq. (7), counted once each at the largest vertex of the\n")
        f.write("# triangle, Sec. 4.2 two-program form) of %s,\n" % desc)
        f.write("# self-loops dropped, symmetrised, upper-triangle DAG.\n")
        f.write("# Written by tests/golden/make_tc_goldens.py from the oracle only.\n")
        f.write("n %d\n" % n)
        f.write("m_dag %d\n" % dag.m)
        f.write("total %d\n" % total)
        f.write("counts_sha256 %s\n" % digest)
    print("%s: total %d, m_dag %d (%.0f s)" % (name, total, dag.m, time.time() - t0), flush=True)
    return path


def read(name: str) -> dict:
    """Parsed golden file: n, m_dag, total (ints) and counts_sha256 (hex)."""
    out = {}
    with open(os.path.join(HERE, name + ".txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            out[k] = v if k.endswith("sha256") else int(v)
    return out


if __name__ == "__main__":
    for nm in sys.argv[1:] or list(WORKLOADS):
        make(nm)
