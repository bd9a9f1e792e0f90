"""RMAT scale 26 (67,108,864 vertices, 16 * 2^26 generated edges; over a
billion directed and two billion symmetrised entries): PageRank (20
supersteps), BFS from vertex 0, 32-source batched BFS and the PageRank
edge-weight gradient, on one GPU.

A full oracle run is impractical at this size, so results are checked where
the oracle can compute them one by one and through properties that hold at
any size:
  PageRank: every superstep recomputed in FP64 by the oracle for sampled
    rows from the GPU's previous iterate (max relative error <= 1e-6), the
    total-mass identity of Eq. (1) at every superstep, and the plain call
    equal to the weighted forward with w = 1;
  BFS: the oracle's linear-time level certificate (root 0, no edge spans more
    than one level, every reached vertex has a parent one level up) and the
    superstep count = max level + 1;
  batched BFS: column 0 equals the certified plain run, sampled columns equal
    plain runs from their sources, one more column certified;
  weight gradient: the T = 1 closed form (1 - r) c_v / outdeg(u) on every
    edge; at T = 20, c . PR^T and the gradient's component along a fixed
    direction against the oracle's FP64 values (golden/pr_grad_rmat26.txt,
    written by golden/make_pr_grad26.py: a central difference of the
    oracle's forward, since a full oracle reverse pass at this size does not
    fit a test run), and linearity in the upstream gradient.
"""
import gc
import os

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_1503_07241_amd as gm

pytestmark = pytest.mark.gpu
DEV = "cuda"
SCALE = 26
R = 0.15


def read_golden():
    out = {}
    for line in open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                  "pr_grad_rmat26.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split()
        out[k] = float(v) if ("." in v or "e" in v) else int(v)
    return out


@pytest.fixture(scope="module")
def raw():
    n, s, d = gg.rmat(SCALE)
    return n, s, d


@pytest.fixture(scope="module")
def gdir(raw):
    n, s, d = raw
    g = gm.Graph.from_coo(n, s, d)
    yield g
    g.close()
    torch.cuda.empty_cache()


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.int32, device=DEV)


def test_pagerank_scale26(raw, gdir):
    n = raw[0]
    m = gdir.m
    assert m > 1_000_000_000
    T = 20
    w = torch.ones(m, dtype=torch.float32, device=DEV)
    hist = torch.empty((T + 1, n), dtype=torch.float32, device=DEV)
    hist[0].fill_(1.0)
    gm.pagerank_forward_w(gdir, w, R, T, hist)
    rank = torch.ones(n, dtype=torch.float32, device=DEV)
    assert gm.run_vertex_program(gdir, gm.GM_PROG_PAGERANK, None, T, rank) == T
    assert torch.equal(rank, hist[T]) or float(((rank - hist[T]).abs() / hist[T]).max()) <= 1e-6
    del w, rank
    src, dst = gdir.edges()
    outdeg = np.bincount(src, minlength=n).astype(np.int64)
    indeg = np.bincount(dst, minlength=n)
    rng = np.random.default_rng(26)
    rows = np.unique(np.concatenate([[0, 1, n - 1], np.argsort(indeg)[-8:],
                                     rng.integers(0, n, 3000)]))
    sends = outdeg > 0
    mark = np.zeros(n, dtype=bool)
    mark[rows] = True
    sel = mark[dst]  # the in-edges of the sampled rows
    ssrc, sdst = src[sel], dst[sel]
    for t in range(T):
        prev = hist[t].cpu().numpy().astype(np.float64)
        nxt = hist[t + 1].cpu().numpy().astype(np.float64)
        ref = oracle.pagerank_step_rows(prev, outdeg, ssrc, sdst, rows, R)
        err = float(np.max(np.abs(nxt[rows] - ref) / ref))
        assert err <= 1e-6, "superstep %d: max rel err %g" % (t, err)
        # Eq. (1) summed over v: sum PR^{t+1} = r n + (1 - r) sum_{u sends} PR^t(u)
        lhs = nxt.sum()
        rhs = R * n + (1 - R) * prev[sends].sum()
        assert abs(lhs - rhs) <= 1e-6 * rhs, "superstep %d: mass %g vs %g" % (t, lhs, rhs)
    del hist, src, dst
    gc.collect()


def test_pagerank_weight_gradient_scale26(raw, gdir):
    n = raw[0]
    m = gdir.m
    w = torch.ones(m, dtype=torch.float32, device=DEV)
    c = torch.tensor(gg.uniform_f32(n, gg.SEED_PR_UPSTREAM), device=DEV)
    # T = 1: dL/dw_uv = (1 - r) c_v PR^0(u) / outdeg(u), on every edge
    hist = torch.empty((2, n), dtype=torch.float32, device=DEV)
    hist[0].fill_(1.0)
    gm.pagerank_forward_w(gdir, w, R, 1, hist)
    gw = torch.empty_like(w)
    gm.pagerank_vjp_w(gdir, w, R, 1, hist, c, gw)
    src, dst = gdir.edges()
    outdeg = np.bincount(src, minlength=n).astype(np.float64)
    ch = c.cpu().numpy().astype(np.float64)
    g1 = gw.cpu().numpy()
    worst = 0.0
    for lo in range(0, m, 1 << 27):
        hi = min(m, lo + (1 << 27))
        ref = (1 - R) * ch[dst[lo:hi]] / outdeg[src[lo:hi]]
        worst = max(worst, float(np.max(np.abs(g1[lo:hi] - ref) / ref)))
    assert worst <= 1e-6, worst
    del hist, g1, src, dst
    # T = 20: c . PR^T and the gradient's component along a direction d
    # against the FP64 oracle (golden/pr_grad_rmat26.txt: a central difference
    # of the oracle's forward), then linearity in the upstream gradient
    ref = read_golden()
    assert ref["n"] == n and ref["m"] == m and ref["T"] == 20
    T = 20
    hist = torch.empty((T + 1, n), dtype=torch.float32, device=DEV)
    hist[0].fill_(1.0)
    gm.pagerank_forward_w(gdir, w, R, T, hist)
    L = float(torch.dot(hist[T].double(), c.double()))
    assert abs(L - ref["L_w1"]) <= 1e-5 * abs(ref["L_w1"]), (L, ref["L_w1"])
    ga = torch.empty_like(w)
    gm.pagerank_vjp_w(gdir, w, R, T, hist, c, ga)
    src, dst = gdir.edges()
    dd = 0.0
    for lo in range(0, m, 1 << 27):
        hi = min(m, lo + (1 << 27))
        dvec = torch.tensor(gg.weights_f32(src[lo:hi], dst[lo:hi], int(ref["seed_dir"]), 0.5, 1.5),
                            device=DEV)
        dd += float(torch.dot(ga[lo:hi].double(), dvec.double()))
    del src, dst, dvec
    assert abs(dd - ref["dir_deriv"]) <= 1e-5 * abs(ref["dir_deriv"]), (dd, ref["dir_deriv"])
    c2 = torch.tensor(gg.uniform_f32(n, gg.SEED_PR_UPSTREAM + 1), device=DEV)
    gb, gab = torch.empty_like(w), torch.empty_like(w)
    gm.pagerank_vjp_w(gdir, w, R, T, hist, c2, gb)
    gm.pagerank_vjp_w(gdir, w, R, T, hist, c + c2, gab)
    assert bool(torch.isfinite(gab).all())
    num = float(torch.linalg.vector_norm((ga.double() + gb.double()) - gab.double()))
    den = float(torch.linalg.vector_norm(gab.double()))
    assert num <= 1e-6 * den, num / den
    del hist, ga, gb, gab, gw, w
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def gsym(raw, gdir):
    n, s, d = raw
    gdir.close()  # only one large graph at a time on the host side
    g = gm.Graph.from_coo(n, s, d, prep=gm.GM_PREP_DROP_SELF_LOOPS | gm.GM_PREP_SYMMETRIZE,
                          layouts=gm.GM_LAYOUT_OUT)
    src, dst = g.edges()
    yield g, src, dst
    g.close()


def plain_bfs(g, n, root):
    lv = torch.full((n,), gm.INF_LEVEL, dtype=torch.int32, device=DEV)
    lv[root] = 0
    it = gm.run_vertex_program(g, gm.GM_PROG_BFS, dev([root]), -1, lv)
    return lv.cpu().numpy(), it


def test_bfs_scale26_certified(raw, gsym):
    n = raw[0]
    g, src, dst = gsym
    lv, it = plain_bfs(g, n, 0)
    assert oracle.bfs_certificate(n, src, dst, lv, 0) == 0
    assert it == int(lv[lv != oracle.INF_I32].max()) + 1
    assert (lv != oracle.INF_I32).sum() > n // 4


def test_batched_bfs32_scale26(raw, gsym):
    n, s, d = raw
    g, src, dst = gsym
    S = gg.sources(n, s, d, 32, gg.SEED_BATCH_SOURCES)
    assert S[0] == 0 and len(S) == 32
    blk = torch.empty((n, 32), dtype=torch.int32, device=DEV)
    gm.run_batched(g, gm.GM_PROG_BFS, dev(S), -1, blk)
    for j in (0, 9, 31):
        col = blk[:, j].contiguous().cpu().numpy()
        ref, _ = plain_bfs(g, n, int(S[j]))
        assert np.array_equal(col, ref), "column %d" % j
    col = blk[:, 20].contiguous().cpu().numpy()
    assert oracle.bfs_certificate(n, src, dst, col, int(S[20])) == 0
    del blk
    torch.cuda.empty_cache()
