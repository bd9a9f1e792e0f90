"""GPU PageRank (Sec. 3 I, Eq. (1)) in FP32 against the FP64 oracle: relative
error <= 1e-5 per vertex after 20 supersteps."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_1503_07241_amd as gm
from tests import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL = 1e-5


def run_pr(g, n, T=20, kind=gm.GM_PROG_PAGERANK, seed=None, r=0.15):
    rank = torch.ones(n, dtype=torch.float32, device=DEV)
    fr = None
    if seed is not None:
        rank.zero_()
        rank[seed] = 1.0
        fr = torch.tensor([seed], dtype=torch.int32, device=DEV)
    it = gm.run_vertex_program(g, kind, fr, T, rank, r=r)
    assert it == T
    return rank.cpu().numpy()


@pytest.mark.parametrize("scale", [W.SMALL_SCALE, W.FULL_SCALE])
def test_pagerank_rmat(scale):
    n, s, d = W.raw(scale)
    g = gm.Graph.from_coo(n, s, d)
    got = run_pr(g, n)
    assert W.max_rel_err(got, W.pagerank(scale)) <= TOL


def test_pagerank_long_rows_split():
    """In-star with far more in-edges than one work item holds: the hub row is
    reduced in chunks; closed form of Eq. (1) for the hub and the leaves."""
    leaves = 50000
    n = leaves + 1
    s = np.arange(1, n, dtype=np.int32)
    d = np.zeros(leaves, dtype=np.int32)
    g = gm.Graph.from_coo(n, s, d)
    got = run_pr(g, n, T=3)
    r = 0.15
    assert abs(got[0] - (r + (1 - r) * r * leaves)) / got[0] <= TOL
    assert np.allclose(got[1:], r, rtol=TOL)
    # ragged sizes around the work-item boundaries
    for deg in (2047, 2048, 2049, 4097, 6000):
        n = deg + 3
        s = np.concatenate([np.arange(1, deg + 1), [0, 1]]).astype(np.int32)
        d = np.concatenate([np.zeros(deg), [deg + 1, deg + 2]]).astype(np.int32)
        g = gm.Graph.from_coo(n, s, d)
        ref = oracle.pagerank(oracle.prepare(n, s, d), 0.15, 20)
        assert W.max_rel_err(run_pr(g, n), ref) <= TOL


def _rows_graph(degrees, extra_sources, seed):
    """Row v (v < len(degrees)) gets degrees[v] in-edges from distinct random
    sources among all n vertices (no self loops)."""
    rng = np.random.default_rng(seed)
    nrows = len(degrees)
    n = nrows + extra_sources
    src, dst = [], []
    for v, k in enumerate(degrees):
        cand = rng.choice(n - 1, size=k, replace=False)
        cand = np.where(cand >= v, cand + 1, cand)
        src.append(cand)
        dst.append(np.full(k, v))
    return n, np.concatenate(src).astype(np.int32), np.concatenate(dst).astype(np.int32)


# In-degree multisets whose running sums, in decreasing order (the kernel's
# row order), put row ends exactly on, just before and just after multiples
# of the 1024-edge tile, rows spanning several tiles, and runs of in-degree-1
# rows; totals that fill the last tile exactly and that leave it ragged.
TILE_CASES = [
    [3072, 1024, 1000, 24] + [1] * 1024,
    [3072, 1024, 1000, 24] + [1] * 1023,
    [2049, 1023, 1, 1],
    [1025] + [2] * 600 + [1] * 5,
    [1024],
    [5] * 3 + [1] * 7,
    [700, 324] + [3] * 341 + [1],
    [5 * 1024 + 17],
    [512] * 4,
    list(np.sort(np.minimum((np.random.default_rng(3).pareto(1.2, 3000) * 3 + 1).astype(int),
                            9000))[::-1]),
]


@pytest.mark.parametrize("case", range(len(TILE_CASES)))
def test_pagerank_tile_boundaries(case):
    """The device-built layout (degree relabelling, row-start bitmap, first
    row of each tile, rows spanning tiles) through the pull superstep."""
    degrees = TILE_CASES[case]
    n, s, d = _rows_graph(degrees, max(4000, max(degrees) + 1), seed=100 + case)
    g = gm.Graph.from_coo(n, s, d)
    og = oracle.prepare(n, s, d)
    assert W.max_rel_err(run_pr(g, n), oracle.pagerank(og, 0.15, 20)) <= TOL
    wf = gg.weights_f32(s, d, 12 + case, 0.5, 1.5)
    gw = gm.Graph.from_coo(n, s, d, w=wf)
    ogw = oracle.prepare(n, s, d, w=wf)
    ref = oracle.pagerank(ogw, 0.15, 20, w=ogw.w.astype(np.float64))
    assert W.max_rel_err(run_pr(gw, n), ref) <= TOL
    for seed in (0, 1):
        got = run_pr(g, n, kind=gm.GM_PROG_PPR, seed=seed)
        ref = oracle.personalized_pagerank(og, seed, 0.15, 20)
        assert np.abs(got - ref).sum() / np.abs(ref).sum() <= TOL


def test_pagerank_closed_forms():
    n = 1000
    cyc = gm.Graph.from_coo(n, np.arange(n), (np.arange(n) + 1) % n)
    assert np.allclose(run_pr(cyc, n), 1.0, rtol=1e-6)
    path = gm.Graph.from_coo(25, np.arange(24), np.arange(1, 25))
    want = np.array([1 - 0.85 ** (k + 1) if k < 20 else 1.0 for k in range(25)])
    assert W.max_rel_err(run_pr(path, 25), want) <= TOL


def test_personalized_single_seed():
    scale = 12
    n, s, d = W.raw(scale)
    g = gm.Graph.from_coo(n, s, d)
    og = W.ograph(scale, "directed")
    for seed in (0, 17):
        got = run_pr(g, n, kind=gm.GM_PROG_PPR, seed=seed)
        ref = oracle.personalized_pagerank(og, seed, 0.15, 20)
        # PPR values can be 0: L1 relative error per seed
        assert np.abs(got - ref).sum() / np.abs(ref).sum() <= TOL


def test_weighted_pagerank():
    scale = 12
    n, s, d = W.raw(scale)
    wf = gg.weights_f32(s, d, 11, 0.5, 1.5)
    g = gm.Graph.from_coo(n, s, d, w=wf)
    og = oracle.prepare(n, s, d, w=wf)
    ref = oracle.pagerank(og, 0.15, 20, w=og.w.astype(np.float64))
    assert W.max_rel_err(run_pr(g, n), ref) <= TOL


def test_pagerank_empty_graph():
    g = gm.Graph.from_coo(7, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert np.allclose(run_pr(g, 7, T=4), 0.15)


def test_pagerank_deterministic():
    n, s, d = W.raw(16)
    g = gm.Graph.from_coo(n, s, d)
    a = run_pr(g, n)
    b = run_pr(g, n)
    assert np.array_equal(a, b)
