"""Write the expected directional derivative of the PageRank edge-weight
gradient on RMAT scale 26 (67,108,864 vertices, 2^30 generated edges).

L(w) = c . PR^T(w) with PR^{t+1}(v) = r + (1 - r) sum_{u -> v} w_uv PR^t(u) /
outdeg(u) (Eq. (1) with edge weights, unweighted out-degree), T = 20,
r = 0.15, PR^0 = 1, c ~ U(0, 1) (seed 10), evaluated at w = 1. The
gradient's component along a direction d (d_uv uniform in [0.5, 1.5), drawn
per ordered pair (u, v), seed 11) is

    <dL/dw, d> = (L(1 + h d) - L(1 - h d)) / (2 h),

a central difference of the oracle's FP64 forward (h = 3e-5: truncation
error about h^2 T^2 / 6, far below 1e-7 relative; rounding about 1e-9). All
arithmetic of the method is the oracle's (pagerank_history); this script
only builds the loop-free, deduplicated in-adjacency with numpy, in place, to
fit in host memory (peak about 35 GB), and draws the inputs from graphgen.

Usage: python tests/golden/make_pr_grad26.py     (about 20 minutes)
"""
from __future__ import annotations

import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SCALE, T, R, H = 26, 20, 0.15, 3e-5
SEED_DIR = 11
CHUNK = 1 << 26


def in_adjacency(scale: int):
    """(n, off, src, dst): in-edges sorted by (dst, src), self-loops dropped,
    duplicates merged; dst is each in-edge's row."""
    n, s, d = gg.rmat(scale)
    b = scale
    key = np.empty(len(s), dtype=np.int64)
    k = 0
    for lo in range(0, len(s), CHUNK):
        ss = s[lo:lo + CHUNK].astype(np.int64)
        dd = d[lo:lo + CHUNK].astype(np.int64)
        keep = ss != dd
        kk = (dd[keep] << b) | ss[keep]
        key[k:k + len(kk)] = kk
        k += len(kk)
    del s, d
    key = key[:k]
    key.sort()
    first = np.empty(len(key), dtype=bool)
    first[0] = True
    np.not_equal(key[1:], key[:-1], out=first[1:])
    key = key[first]
    del first
    m = len(key)
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    cnt = np.zeros(n, dtype=np.int64)
    for lo in range(0, m, CHUNK):
        kk = key[lo:lo + CHUNK]
        src[lo:lo + len(kk)] = kk & ((1 << b) - 1)
        dst[lo:lo + len(kk)] = kk >> b
        cnt += np.bincount(dst[lo:lo + len(kk)], minlength=n)
    del key
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt, out=off[1:])
    return n, off, src, dst


def main():
    t0 = time.time()
    n, off, src, dst = in_adjacency(SCALE)
    m = len(src)
    print("in-adjacency: n %d, m %d (%.0f s)" % (n, m, time.time() - t0), flush=True)
    outdeg_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=outdeg_off[1:])
    gout = oracle.Graph(n, outdeg_off, np.empty(0, dtype=np.int32))  # out-degrees only
    d = np.empty(m, dtype=np.float64)
    for lo in range(0, m, CHUNK):
        d[lo:lo + CHUNK] = gg.weights_f32(np.ascontiguousarray(src[lo:lo + CHUNK]),
                                          np.ascontiguousarray(dst[lo:lo + CHUNK]),
                                          SEED_DIR, 0.5, 1.5)
    del dst
    c = gg.uniform_f32(n, gg.SEED_PR_UPSTREAM).astype(np.float64)
    vals = {}
    for name, sign in (("L_plus", 1.0), ("L_minus", -1.0), ("L_w1", 0.0)):
        w = 1.0 + sign * H * d
        gin = oracle.Graph(n, off, src, w)
        t1 = time.time()
        pr = oracle.pagerank(gout, R, T, g_in=gin)
        vals[name] = float(np.dot(c, pr))
        print("%s = %.17g (%.0f s)" % (name, vals[name], time.time() - t1), flush=True)
        del w, gin, pr
    dd = (vals["L_plus"] - vals["L_minus"]) / (2 * H)
    path = os.path.join(HERE, "pr_grad_rmat26.txt")
    with open(path, "w") as f:
        f.write("# PageRank edge-weight gradient on RMAT scale 26 (a=.57 b=c=.19, edge factor\n")
        f.write("# 16, seed 1; self-loops dropped, duplicates merged), Eq. (1) with weights,\n")
        f.write("# T=20, r=0.15, PR^0=1, at w=1; c = graphgen uniform_f32(n, seed 10);\n")
        f.write("# d_uv = graphgen weights_f32(u, v, seed 11, 0.5, 1.5).\n")
        f.write("# Written by tests/golden/make_pr_grad26.py from the oracle's FP64 forward.\n")
        f.write("n %d\nm %d\nT %d\nr %.17g\nh %.17g\nseed_dir %d\n" % (n, m, T, R, H, SEED_DIR))
        for k in ("L_plus", "L_minus", "L_w1"):
            f.write("%s %.17g\n" % (k, vals[k]))
        f.write("dir_deriv %.17g\n" % dd)
    print("directional derivative %.12g (%.0f s total)" % (dd, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
