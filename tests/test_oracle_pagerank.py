"""Pins of the oracle's PageRank (Sec. 3 I, Eq. (1)), personalised PageRank and
the edge-weight gradient of the weighted form.

Independent of the oracle's code: closed forms (cycle, complete digraph,
directed path, in-star), networkx's PageRank fixed point, linearity of the
personalised form, torch float64 autograd of a dense unrolled iteration, and
central finite differences.
"""
import os

import networkx as nx
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
R = 0.15


def gp(n, pairs):
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    return oracle.prepare(n, pairs[:, 0], pairs[:, 1])


def test_cycle_and_complete_are_uniform():
    n = 13
    cyc = gp(n, [(i, (i + 1) % n) for i in range(n)])
    for t_row in oracle.pagerank_history(cyc, R, 20):
        assert np.allclose(t_row, 1.0, rtol=0, atol=1e-15)
    kn = gp(7, [(i, j) for i in range(7) for j in range(7) if i != j])
    assert np.allclose(oracle.pagerank(kn, R, 20), 1.0, rtol=0, atol=1e-14)


def test_directed_path_golden():
    """tests/golden/pagerank_directed_path.txt: hand-derived closed form of Eq. (1)."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "pagerank_directed_path.txt"))
            if l.strip() and not l.startswith("#")]
    exp = np.array([float(v) for _, v in rows])
    n = len(exp)
    g = gp(n, [(i, i + 1) for i in range(n - 1)])
    got = oracle.pagerank(g, R, 20)
    assert np.allclose(got, exp, rtol=1e-13, atol=0)
    hist = oracle.pagerank_history(g, R, 20)
    for t in range(21):
        for k in range(n):
            want = 1.0 if t <= k else 1 - (1 - R) ** (k + 1)
            assert abs(hist[t, k] - want) < 1e-13


def test_in_star_dangling_hub():
    """Leaves -> hub, hub has out-degree 0 (its mass leaks, Eq. (1) taken literally)."""
    n = 9
    g = gp(n, [(i, 0) for i in range(1, n)])
    h = oracle.pagerank_history(g, R, 5)
    assert abs(h[1, 0] - (R + (1 - R) * (n - 1))) < 1e-13
    for t in range(2, 6):
        assert abs(h[t, 0] - (R + (1 - R) * R * (n - 1))) < 1e-13
        assert np.allclose(h[t, 1:], R, atol=1e-15)
    # a vertex without in-edges takes r at every step >= 1 (dense APPLY reading)
    assert np.allclose(h[1:, 1:], R)


@pytest.mark.parametrize("seed", range(3))
def test_networkx_fixed_point_dangling_free(seed):
    """For graphs with no dangling vertex, n * networkx.pagerank(alpha=1-r) is the
    fixed point of Eq. (1)."""
    rng = np.random.default_rng(seed)
    n = 40
    s = np.concatenate([np.arange(n), rng.integers(0, n, 150)])
    d = np.concatenate([(np.arange(n) + 1) % n, rng.integers(0, n, 150)])
    g = oracle.prepare(n, s, d)
    assert (g.degree() > 0).all()
    G = nx.DiGraph()
    G.add_nodes_from(range(n))
    G.add_edges_from(zip(g.rows().tolist(), g.idx.tolist()))
    ref = nx.pagerank(G, alpha=1 - R, tol=1e-15, max_iter=10_000)
    got = oracle.pagerank(g, R, 400)
    assert np.allclose(got, n * np.array([ref[i] for i in range(n)]), rtol=1e-9, atol=0)


def dense_unrolled(n, rows, cols, w, r, T, c):
    """L = c . PR^T of the weighted Eq. (1) built with dense torch float64 ops."""
    wt = torch.tensor(w, dtype=torch.float64, requires_grad=True)
    deg = np.bincount(rows, minlength=n).astype(np.float64)
    M = torch.zeros(n, n, dtype=torch.float64)
    M = M.index_put((torch.tensor(cols), torch.tensor(rows)),
                    wt / torch.tensor(deg[rows]), accumulate=True)  # M[v, u] = w_uv / deg(u)
    pr = torch.ones(n, dtype=torch.float64)
    for _ in range(T):
        pr = r + (1 - r) * (M @ pr)
    L = (torch.tensor(c) * pr).sum()
    L.backward()
    return pr.detach().numpy(), wt.grad.numpy()


@pytest.mark.parametrize("seed", range(3))
def test_weighted_pagerank_and_gradient_vs_autograd(seed):
    n, s, d = gg.rmat(5, seed=20 + seed)
    g = oracle.prepare(n, s, d)
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.5, 1.5, g.m)
    c = rng.uniform(0, 1, n)
    T = 6
    pr_ref, gw_ref = dense_unrolled(n, g.rows(), g.idx.astype(np.int64), w, R, T, c)
    hist = oracle.pagerank_history(g, R, T, w=w)
    assert np.allclose(hist[-1], pr_ref, rtol=1e-12, atol=0)
    gw = oracle.pagerank_vjp_w(g, w, c, R, T, hist=hist)
    assert np.allclose(gw, gw_ref, rtol=1e-10, atol=1e-14)


def test_unit_weights_equal_eq1():
    n, s, d = gg.rmat(8)
    g = oracle.prepare(n, s, d)
    assert np.array_equal(oracle.pagerank(g, R, 20), oracle.pagerank(g, R, 20, w=np.ones(g.m)))


def test_gradient_T1_closed_form_and_cycle_symmetry():
    n, s, d = gg.rmat(6)
    g = oracle.prepare(n, s, d)
    c = np.random.default_rng(0).uniform(0, 1, n)
    gw = oracle.pagerank_vjp_w(g, np.ones(g.m), c, R, 1)
    deg = g.degree()[g.rows()]
    assert np.allclose(gw, (1 - R) * c[g.idx] / deg, rtol=1e-14)
    cyc = gp(10, [(i, (i + 1) % 10) for i in range(10)])
    gc = oracle.pagerank_vjp_w(cyc, np.ones(10), np.ones(10), R, 20)
    assert np.allclose(gc, gc[0], rtol=1e-13)


def test_gradient_central_difference():
    n, s, d = gg.rmat(6, seed=3)
    g = oracle.prepare(n, s, d)
    rng = np.random.default_rng(1)
    w = rng.uniform(0.5, 1.5, g.m)
    c = rng.uniform(0, 1, n)
    T = 20
    gw = oracle.pagerank_vjp_w(g, w, c, R, T)
    dirv = rng.normal(size=g.m)
    h = 1e-6
    Lp = c @ oracle.pagerank(g, R, T, w=w + h * dirv)
    Lm = c @ oracle.pagerank(g, R, T, w=w - h * dirv)
    fd = (Lp - Lm) / (2 * h)
    assert abs(fd - gw @ dirv) <= 1e-6 * abs(fd)


def test_personalized_linearity():
    """sum_s PPR_s^t = PR^t: the teleport vectors e_s sum to the all-ones vector."""
    n, s, d = gg.rmat(6, seed=5)
    g = oracle.prepare(n, s, d)
    gin = g.transpose()
    tot = sum(oracle.personalized_pagerank(g, v, R, 20, g_in=gin) for v in range(n))
    assert np.allclose(tot, oracle.pagerank(g, R, 20), rtol=1e-12)


def test_personalized_on_cycle_closed_form():
    """On a directed n-cycle PPR_0^t(k) for t >= 1 is r(1-r)^k/(1-(1-r)^n) at the
    fixed point; after t steps the mass that started at 0 sits at vertex t mod n."""
    n = 6
    g = gp(n, [(i, (i + 1) % n) for i in range(n)])
    ppr = oracle.personalized_pagerank(g, 0, R, 400)
    want = R * (1 - R) ** np.arange(n) / (1 - (1 - R) ** n)
    assert np.allclose(ppr, want, rtol=1e-12)


def test_pagerank_step_rows_is_one_superstep():
    """oracle.pagerank_step_rows (one superstep for sampled rows, used at full
    scale) reproduces step t -> t + 1 of the FP64 history, unweighted and
    weighted, including rows with no in-edge (value r)."""
    n, s, d = gg.rmat(10, seed=7)
    g = oracle.prepare(n, s, d)
    src, dst = g.rows(), g.idx.astype(np.int64)
    outdeg = g.degree()
    rows = np.array([0, 1, 2, 5, 17, 100, 511, n - 1])
    hist = oracle.pagerank_history(g, 0.15, 5)
    for t in range(5):
        got = oracle.pagerank_step_rows(hist[t], outdeg, src, dst, rows, 0.15)
        assert np.allclose(got, hist[t + 1][rows], rtol=1e-13, atol=0)
    w = gg.weights_f32(g.rows().astype(np.int32), g.idx, 3, 0.5, 1.5).astype(np.float64)
    hw = oracle.pagerank_history(g, 0.15, 3, w=w)
    got = oracle.pagerank_step_rows(hw[2], outdeg, src, dst, rows, 0.15, w=w)
    assert np.allclose(got, hw[3][rows], rtol=1e-13, atol=0)
    indeg = np.bincount(dst, minlength=n)
    z = np.flatnonzero(indeg == 0)[:3]
    assert np.allclose(oracle.pagerank_step_rows(hist[2], outdeg, src, dst, z), 0.15)


def test_edgeless_graph_closed_forms():
    # no in-edges anywhere: Eq. (1) gives r at every vertex from the first
    # superstep on; personalised, r at the seed and 0 elsewhere
    none = np.zeros(0, np.int32)
    g = oracle.prepare(7, none, none)
    for T in (1, 5):
        assert np.array_equal(oracle.pagerank(g, 0.15, T), np.full(7, 0.15))
        ppr = oracle.personalized_pagerank(g, 4, 0.15, T)
        assert np.array_equal(ppr, np.where(np.arange(7) == 4, 0.15, 0.0))
