"""Batched runs (gm_run_batched): column s of a k-source run equals the plain run
from source s - bit-exact for BFS and SSSP, <= 1e-5 (L1 relative per seed)
for personalised PageRank against the FP64 oracle."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_1503_07241_amd as gm
from tests import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda"
P_DIR = gm.GM_PREP_DROP_SELF_LOOPS
P_SYM = gm.GM_PREP_DROP_SELF_LOOPS | gm.GM_PREP_SYMMETRIZE
BATCH_SCALE = 20  # RMAT scale of the batched configuration


def srcs(scale, k, seed=gg.SEED_BATCH_SOURCES):
    n, s, d = W.raw(scale)
    return gg.sources(n, s, d, k, seed)


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.int32, device=DEV)


def batched(g, kind, sources, n, dtype, max_iters=-1):
    block = torch.empty((n, len(sources)), dtype=dtype, device=DEV)
    it = gm.run_batched(g, kind, dev(sources), max_iters, block)
    return block.cpu().numpy(), it


def plain_bfs(g, n, root):
    lv = torch.full((n,), gm.INF_LEVEL, dtype=torch.int32, device=DEV)
    lv[root] = 0
    it = gm.run_vertex_program(g, gm.GM_PROG_BFS, dev([root]), -1, lv)
    return lv.cpu().numpy(), it


def plain_sssp(g, n, root):
    dist = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    dist[root] = 0
    it = gm.run_vertex_program(g, gm.GM_PROG_SSSP, dev([root]), -1, dist)
    return dist.cpu().numpy().view(np.uint32), it


@pytest.mark.parametrize("scale,k", [(W.SMALL_SCALE, 64), (W.SMALL_SCALE, 37), (12, 1)])
def test_bfs_batched_vs_oracle(scale, k):
    n, s, d = W.raw(scale)
    g = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    S = srcs(scale, k)
    lv, it = batched(g, gm.GM_PROG_BFS, S, n, torch.int32)
    og = W.ograph(scale, "symmetric")
    maxlev = 0
    for j, r in enumerate(S):
        ref = oracle.bfs(og, r)
        assert np.array_equal(lv[:, j], ref), "column %d (source %d)" % (j, r)
        maxlev = max(maxlev, int(ref[ref != oracle.INF_I32].max()))
    assert it == maxlev + 1


def test_bfs_batched_full_size():
    n, s, d = W.raw(BATCH_SCALE)
    g = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    S = srcs(BATCH_SCALE, 64)
    lv, it = batched(g, gm.GM_PROG_BFS, S, n, torch.int32)
    og = W.ograph(BATCH_SCALE, "symmetric")
    for j in (0, 1, 31, 63):  # oracle on sampled columns
        assert np.array_equal(lv[:, j], oracle.bfs(og, S[j]))
    its = []
    for j, r in enumerate(S):  # every column equals the plain GPU run
        ref, pit = plain_bfs(g, n, r)
        assert np.array_equal(lv[:, j], ref)
        its.append(pit)
    assert it == max(its)


@pytest.mark.parametrize("scale,k", [(W.SMALL_SCALE, 64), (12, 5)])
def test_sssp_batched_vs_oracle(scale, k):
    n, s, d = W.raw(scale)
    g = gm.Graph.from_coo(n, s, d, w=W.weights(scale), prep=P_DIR)
    S = srcs(scale, k)
    dist, _ = batched(g, gm.GM_PROG_SSSP, S, n, torch.int32)
    dist = dist.view(np.uint32)
    og = W.ograph(scale, "directed", True)
    for j, r in enumerate(S):
        assert np.array_equal(dist[:, j], oracle.sssp(og, r)), "column %d" % j


def test_sssp_batched_full_size():
    n, s, d = W.raw(BATCH_SCALE)
    g = gm.Graph.from_coo(n, s, d, w=W.weights(BATCH_SCALE), prep=P_DIR)
    S = srcs(BATCH_SCALE, 64)
    dist, it = batched(g, gm.GM_PROG_SSSP, S, n, torch.int32)
    dist = dist.view(np.uint32)
    og = W.ograph(BATCH_SCALE, "directed", True)
    for j in (0, 7, 63):
        assert np.array_equal(dist[:, j], oracle.sssp(og, S[j]))
    its = []
    for j, r in enumerate(S):
        ref, pit = plain_sssp(g, n, r)
        assert np.array_equal(dist[:, j], ref)
        its.append(pit)
    assert it <= max(its)


def l1_rel(got, ref):
    return float(np.abs(got - ref).sum() / np.abs(ref).sum())


@pytest.mark.parametrize("scale,k", [(12, 128), (10, 64), (10, 200)])
def test_ppr_batched_vs_oracle(scale, k):
    n, s, d = W.raw(scale)
    g = gm.Graph.from_coo(n, s, d)
    S = srcs(scale, k, gg.SEED_PPR_SEEDS)
    k = len(S)
    pr, it = batched(g, gm.GM_PROG_PPR, S, n, torch.float32, max_iters=20)
    assert it == 20
    og, ogin = W.ograph(scale, "directed"), W.otranspose(scale, "directed")
    for j, r in enumerate(S):
        ref = oracle.personalized_pagerank(og, int(r), 0.15, 20, g_in=ogin)
        assert l1_rel(pr[:, j], ref) <= 1e-5, "seed %d" % r


def test_ppr_batched_full_size_and_linearity():
    n, s, d = W.raw(BATCH_SCALE)
    g = gm.Graph.from_coo(n, s, d)
    S = srcs(BATCH_SCALE, 128, gg.SEED_PPR_SEEDS)
    pr, _ = batched(g, gm.GM_PROG_PPR, S, n, torch.float32, max_iters=20)
    og, ogin = W.ograph(BATCH_SCALE, "directed"), W.otranspose(BATCH_SCALE, "directed")
    for j in (0, 64, 127):
        ref = oracle.personalized_pagerank(og, int(S[j]), 0.15, 20, g_in=ogin)
        assert l1_rel(pr[:, j], ref) <= 1e-5
    # every column against the plain single-seed GPU run from its seed (each
    # within 1e-5 of the FP64 result, so within 2e-5 of each other); the
    # plain path is the one checked against the oracle above and in
    # test_gpu_pagerank.py
    col = torch.empty(n, dtype=torch.float32, device=DEV)
    worst = 0.0
    for j, seed in enumerate(S):
        col.zero_()
        col[int(seed)] = 1.0
        gm.run_vertex_program(g, gm.GM_PROG_PPR, dev([int(seed)]), 20, col)
        worst = max(worst, l1_rel(pr[:, j], col.cpu().numpy()))
    assert worst <= 2e-5, worst
    # every vertex as a seed: the columns sum to PageRank (teleports sum to 1)
    n2 = 200
    s2, d2 = gg.rmat(8, seed=5)[1:]
    keep = (s2 < n2) & (d2 < n2)
    g2 = gm.Graph.from_coo(n2, s2[keep], d2[keep])
    allp, _ = batched(g2, gm.GM_PROG_PPR, np.arange(n2), n2, torch.float32, max_iters=20)
    pr2 = oracle.pagerank(oracle.prepare(n2, s2[keep], d2[keep]), 0.15, 20)
    assert W.max_rel_err(allp.astype(np.float64).sum(1), pr2) <= 1e-5


def test_batched_duplicate_and_dangling_sources():
    n = 30
    s = np.array([0, 1, 2, 3, 10], np.int32)
    d = np.array([1, 2, 3, 4, 11], np.int32)
    g = gm.Graph.from_coo(n, s, d, w=np.array([3, 4, 5, 6, 7], np.uint32), prep=P_DIR)
    S = np.array([0, 0, 4, 20, 10], np.int32)  # repeated source, sink, isolated vertex
    dist, _ = batched(g, gm.GM_PROG_SSSP, S, n, torch.int32)
    dist = dist.view(np.uint32)
    og = oracle.prepare(n, s, d, w=np.array([3, 4, 5, 6, 7], np.uint32))
    for j, r in enumerate(S):
        assert np.array_equal(dist[:, j], oracle.sssp(og, r))


def test_batched_argument_errors():
    n, s, d = W.raw(8)
    g = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    blk = torch.empty((n, 65), dtype=torch.int32, device=DEV)
    with pytest.raises(gm.GmError) as e:
        gm.run_batched(g, gm.GM_PROG_BFS, dev(np.arange(65)), -1, blk)
    assert e.value.status == gm._lib.GM_EINVAL
    with pytest.raises(gm.GmError) as e:
        gm.run_batched(g, gm.GM_PROG_BFS, dev([0, n]), -1, blk)
    assert e.value.status == gm._lib.GM_EINVAL
    with pytest.raises(gm.GmError) as e:  # no weights
        gm.run_batched(g, gm.GM_PROG_SSSP, dev([0]), -1, blk)
    assert e.value.status == gm._lib.GM_EUNSUPPORTED


def test_batched_on_edgeless_graph():
    n = 300
    none = np.zeros(0, np.int32)
    S = [3, 299, 0, 3]
    g = gm.Graph.from_coo(n, none, none, prep=P_SYM)
    lv, _ = batched(g, gm.GM_PROG_BFS, S, n, torch.int32)
    gw = gm.Graph.from_coo(n, none, none, w=np.zeros(0, np.uint32), prep=P_DIR)
    dist, _ = batched(gw, gm.GM_PROG_SSSP, S, n, torch.int32)
    og = oracle.prepare(n, none, none, w=np.zeros(0, np.uint32), mode="directed")
    for j, r in enumerate(S):
        assert np.array_equal(lv[:, j], oracle.bfs(og, r))
        assert np.array_equal(dist[:, j].view(np.uint32), oracle.sssp(og, r))
    pr = torch.empty((n, len(S)), dtype=torch.float32, device=DEV)
    gm.run_batched(gw, gm.GM_PROG_PPR, dev(S), 20, pr)
    pr = pr.cpu().numpy()
    for j, r in enumerate(S):
        ref = oracle.personalized_pagerank(og, r, 0.15, 20)
        assert np.allclose(pr[:, j], ref, rtol=1e-6, atol=0)
