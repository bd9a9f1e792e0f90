"""Pins of the oracle's BFS (Sec. 3 II, Eq. (2)) and SSSP (Sec. 3 V, Eq. (8)).

Each pin is independent of the oracle's own code: closed forms on small
graph families, scipy's csgraph routines, brute-force Bellman-Ford, and the
O(m) certificates that characterise BFS levels and shortest-path distances.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import graphgen as gg
import oracle

INF_I = oracle.INF_I32
INF_U = oracle.INF_U32


def graph_from_pairs(n, pairs, mode="directed", w=None):
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    return oracle.prepare(n, pairs[:, 0], pairs[:, 1], w=w, mode=mode)


def check_bfs_certificate(g, root, level):
    """levels are BFS levels iff: root 0; |dl| <= 1 on every edge with a finite
    end (so no finite-infinite edge); every reached v != root has a neighbour at
    level - 1 (symmetric graph)."""
    assert level[root] == 0
    rows = g.rows()
    lu, lv = level[rows].astype(np.int64), level[g.idx].astype(np.int64)
    fu, fv = lu != INF_I, lv != INF_I
    assert np.array_equal(fu, fv)
    assert (np.abs(lu[fu] - lv[fu]) <= 1).all()
    has_parent = np.zeros(g.n, dtype=bool)
    tight = fu & (lu == lv - 1)
    has_parent[g.idx[tight]] = True
    reached = level != INF_I
    reached[root] = False
    assert has_parent[reached].all()


def check_sssp_certificate(g, s, dist):
    """dist are shortest-path distances iff: dist(s) = 0; no edge can be relaxed
    (dist(v) <= dist(u) + w); every reached v != s has a tight in-edge from a
    reached u (weights are positive, so tight edges lead back to s)."""
    assert dist[s] == 0
    rows = g.rows()
    du = dist[rows].astype(np.uint64)
    dv = dist[g.idx].astype(np.uint64)
    fin = du != INF_U
    cand = du + g.w.astype(np.uint64)
    assert (dv[fin] <= cand[fin]).all()
    tight = fin & (dv == cand)
    has = np.zeros(g.n, dtype=bool)
    has[g.idx[tight]] = True
    reached = dist != INF_U
    reached[s] = False
    assert has[reached].all()


# --- BFS closed forms -------------------------------------------------------
def test_bfs_path():
    n = 9
    g = graph_from_pairs(n, [(i, i + 1) for i in range(n - 1)], "symmetric")
    assert oracle.bfs(g, 0).tolist() == list(range(n))
    assert oracle.bfs(g, 4).tolist() == [abs(i - 4) for i in range(n)]


def test_bfs_cycle_star_components():
    n = 11
    g = graph_from_pairs(n, [(i, (i + 1) % n) for i in range(n)], "symmetric")
    assert oracle.bfs(g, 0).tolist() == [min(i, n - i) for i in range(n)]
    star = graph_from_pairs(8, [(0, i) for i in range(1, 8)], "symmetric")
    assert oracle.bfs(star, 0).tolist() == [0] + [1] * 7
    assert oracle.bfs(star, 3).tolist() == [1, 2, 2, 0, 2, 2, 2, 2]
    two = graph_from_pairs(6, [(0, 1), (1, 2), (3, 4), (4, 5)], "symmetric")
    assert oracle.bfs(two, 0).tolist() == [0, 1, 2, INF_I, INF_I, INF_I]


def test_bfs_multi_root():
    g = graph_from_pairs(7, [(i, i + 1) for i in range(6)], "symmetric")
    assert oracle.bfs(g, [0, 6]).tolist() == [0, 1, 2, 3, 2, 1, 0]


@pytest.mark.parametrize("seed", range(6))
def test_bfs_matches_scipy_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 60))
    m = int(rng.integers(0, 3 * n))
    s, d = rng.integers(0, n, m), rng.integers(0, n, m)
    g = oracle.prepare(n, s, d, mode="symmetric")
    A = sp.csr_matrix((np.ones(g.m), g.idx, g.off), shape=(n, n))
    ref = csgraph.shortest_path(A, unweighted=True, indices=0)
    exp = np.where(np.isinf(ref), INF_I, ref).astype(np.int64)
    assert np.array_equal(oracle.bfs(g, 0).astype(np.int64), exp)


def test_bfs_rmat14_certificate_and_supersteps():
    n, s, d = gg.rmat(14)
    g = oracle.prepare(n, s, d, mode="symmetric")
    level = oracle.bfs(g, 0)
    check_bfs_certificate(g, 0, level)
    # Alg. 2 literally, BFS program: same levels; supersteps = max level + 1
    prop = np.full(n, INF_U, dtype=np.uint32)
    prop[0] = 0
    act = np.zeros(n, dtype=bool)
    act[0] = True
    out, _, iters = oracle.run_min_program(g, prop, act, weighted=False)
    exp = np.where(level == INF_I, INF_U, level).astype(np.uint32)
    assert np.array_equal(out, exp)
    assert iters == level[level != INF_I].max() + 1


def test_certificates_reject_planted_errors():
    """The certificate checks fail on a wrong level / distance."""
    n, s, d = gg.rmat(10)
    g = oracle.prepare(n, s, d, mode="symmetric")
    level = oracle.bfs(g, 0)
    bad = level.copy()
    v = int(np.flatnonzero((level != INF_I) & (level > 0))[5])
    bad[v] += 1
    with pytest.raises(AssertionError):
        check_bfs_certificate(g, 0, bad)
    w = gg.weights_u32(s, d)
    gd = oracle.prepare(n, s, d, w=w)
    dist = oracle.sssp(gd, 0)
    badd = dist.copy()
    v = int(np.flatnonzero((dist != INF_U) & (dist > 0))[3])
    badd[v] -= 1
    with pytest.raises(AssertionError):
        check_sssp_certificate(gd, 0, badd)


# --- SSSP --------------------------------------------------------------------
def bellman_ford_brute(n, rows, cols, w, s):
    dist = [None] * n
    dist[s] = 0
    for _ in range(n):
        for u, v, ww in zip(rows, cols, w):
            if dist[u] is not None and (dist[v] is None or dist[u] + ww < dist[v]):
                dist[v] = dist[u] + ww
    return [INF_U if x is None else x for x in dist]


@pytest.mark.parametrize("seed", range(6))
def test_sssp_brute_force_and_scipy(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 50))
    m = int(rng.integers(0, 4 * n))
    s, d = rng.integers(0, n, m), rng.integers(0, n, m)
    w = rng.integers(1, 256, m).astype(np.uint32)
    g = oracle.prepare(n, s, d, w=w)
    dist = oracle.sssp(g, 0)
    rows = g.rows()
    assert dist.tolist() == bellman_ford_brute(n, rows.tolist(), g.idx.tolist(), g.w.tolist(), 0)
    A = sp.csr_matrix((g.w.astype(float), g.idx, g.off), shape=(n, n))
    ref = csgraph.dijkstra(A, indices=0)
    assert np.array_equal(np.where(np.isinf(ref), INF_U, ref).astype(np.uint32), dist)


def test_sssp_duplicates_keep_min_weight():
    g = graph_from_pairs(3, [(0, 1), (0, 1), (1, 2)], w=np.array([9, 4, 1], dtype=np.uint32))
    assert g.m == 2 and g.w.tolist() == [4, 1]
    assert oracle.sssp(g, 0).tolist() == [0, 4, 5]


def test_sssp_unit_weights_is_directed_bfs():
    n, s, d = gg.rmat(12)
    g = oracle.prepare(n, s, d, w=np.ones(len(s), dtype=np.uint32))
    dist = oracle.sssp(g, 0)
    lvl = oracle.bfs(g, 0)
    assert np.array_equal(np.where(lvl == INF_I, INF_U, lvl).astype(np.uint32), dist)


def test_sssp_rmat14_certificate_and_bsp():
    n, s, d = gg.rmat(14)
    w = gg.weights_u32(s, d)
    g = oracle.prepare(n, s, d, w=w)
    dist = oracle.sssp(g, 0)
    check_sssp_certificate(g, 0, dist)
    A = sp.csr_matrix((g.w.astype(float), g.idx, g.off), shape=(n, n))
    ref = csgraph.dijkstra(A, indices=0)
    assert np.array_equal(np.where(np.isinf(ref), INF_U, ref).astype(np.uint32), dist)
    prop = np.full(n, INF_U, dtype=np.uint32)
    prop[0] = 0
    act = np.zeros(n, dtype=bool)
    act[0] = True
    out, act_out, iters = oracle.run_min_program(g, prop, act, weighted=True)
    assert np.array_equal(out, dist) and not act_out.any()
    assert 5 <= iters <= 40  # exact counts are pinned on the hand-worked trace below


def test_bsp_resume_equals_uninterrupted():
    """State between supersteps is (property, active); resuming continues exactly."""
    n, s, d = gg.rmat(11)
    g = oracle.prepare(n, s, d, w=gg.weights_u32(s, d))
    prop = np.full(n, INF_U, dtype=np.uint32)
    prop[0] = 0
    act = np.zeros(n, dtype=bool)
    act[0] = True
    full, _, it_full = oracle.run_min_program(g, prop, act, weighted=True)
    p1, a1, it1 = oracle.run_min_program(g, prop, act, weighted=True, max_iters=3)
    assert it1 == 3
    p2, _, it2 = oracle.run_min_program(g, p1, a1, weighted=True)
    assert np.array_equal(p2, full) and it1 + it2 == it_full


def test_oracle_bfs_certificate_function():
    """oracle.bfs_certificate (the linear-time check used at full scale)
    accepts true levels (oracle BFS and SciPy's unweighted shortest paths) and
    rejects each kind of planted error."""
    n, s, d = gg.rmat(11)
    g = oracle.prepare(n, s, d, mode="symmetric")
    rows = g.rows().astype(np.int32)
    level = oracle.bfs(g, 0)
    assert oracle.bfs_certificate(n, rows, g.idx, level, 0) == 0
    A = sp.csr_matrix((np.ones(g.m), g.idx, g.off), shape=(n, n))
    dsp = csgraph.shortest_path(A, unweighted=True, indices=0)
    sc = np.where(np.isinf(dsp), INF_I, dsp).astype(np.int32)
    assert oracle.bfs_certificate(n, rows, g.idx, sc, 0) == 0
    reached = np.flatnonzero((level != INF_I) & (level > 0))
    unreached = np.flatnonzero(level == INF_I)
    assert len(unreached) > 0
    bad = level.copy(); bad[0] = 1
    assert oracle.bfs_certificate(n, rows, g.idx, bad, 0) == 1
    bad = level.copy(); bad[reached[7]] += 1            # too far from a neighbour
    assert oracle.bfs_certificate(n, rows, g.idx, bad, 0) in (2, 4)
    bad = level.copy(); bad[reached[7]] -= 1            # no parent one level up
    assert oracle.bfs_certificate(n, rows, g.idx, bad, 0) in (2, 4)
    bad = level.copy(); bad[reached[3]] = INF_I          # reached vertex dropped
    assert oracle.bfs_certificate(n, rows, g.idx, bad, 0) == 3
    iso = np.flatnonzero(g.degree() == 0)
    bad = level.copy(); bad[iso[0]] = 2                  # isolated vertex "reached"
    assert oracle.bfs_certificate(n, rows, g.idx, bad, 0) == 4
    # a planted mistake the numpy certificate above also catches
    with pytest.raises(AssertionError):
        b2 = level.copy(); b2[reached[7]] += 1
        check_bfs_certificate(g, 0, b2)


# Path sums that reach 2^32 - 1: the distance is the sum clamped at
# UINT32_MAX (the saturating PROCESS of SSSP), worked out by hand.
SAT_PAIRS = [(0, 1), (1, 2), (0, 3), (3, 4), (0, 5), (5, 4)]
SAT_W = np.array([4_000_000_000, 4_000_000_000, INF_U - 1, 1, 2**31, 2**31 - 2], np.uint32)
SAT_DIST = [0, 4_000_000_000, INF_U, INF_U - 1, INF_U - 1, 2**31]


def test_sssp_saturates_at_uint32_max():
    g = graph_from_pairs(6, SAT_PAIRS, w=SAT_W)
    assert oracle.sssp(g, 0).tolist() == SAT_DIST


def test_sssp_superstep_trace_hand_worked():
    """Alg. 2 supersteps of SSSP on the hand-worked graph of
    golden/sssp_supersteps_hand.txt: distances and active set after every
    superstep, and the exact superstep count (5), which the GPU tests then
    require of the GPU run."""
    from tests import workloads as W
    n, s, d, w, src, trace, steps = W.sssp_hand_trace()
    g = oracle.prepare(n, s, d, w=w)
    prop = np.full(n, INF_U, dtype=np.uint32)
    prop[src] = 0
    act = np.zeros(n, dtype=bool)
    act[src] = True
    for k, (dist_k, act_k) in enumerate(trace, start=1):
        p, a, it = oracle.run_min_program(g, prop, act, weighted=True, max_iters=k)
        assert it == k and np.array_equal(p, dist_k) and np.array_equal(a, act_k), k
    p, a, it = oracle.run_min_program(g, prop, act, weighted=True)
    assert it == steps == 5 and not a.any()
    assert np.array_equal(p, oracle.sssp(g, src)) and np.array_equal(p, trace[-1][0])


def test_degree_program_hand_graph_and_closed_forms():
    """Fig. 1's degree-as-SpMV: on the hand-made digraph 0->1, 0->2, 2->1,
    1->3 the in-degrees are [0, 2, 1, 1] and out-degrees [2, 1, 1, 0]; on K_n
    every degree is n - 1 each way; a star's hub has degree n - 1."""
    g = graph_from_pairs(4, [(0, 1), (0, 2), (2, 1), (1, 3)])
    assert oracle.degree(g, "out").tolist() == [0, 2, 1, 1]
    assert oracle.degree(g, "in").tolist() == [2, 1, 1, 0]
    assert oracle.degree(g, "all").tolist() == [2, 3, 2, 1]
    n = 7
    kn = graph_from_pairs(n, [(i, j) for i in range(n) for j in range(n) if i != j])
    assert (oracle.degree(kn, "out") == n - 1).all() and (oracle.degree(kn, "all") == 2 * n - 2).all()
    star = graph_from_pairs(n, [(0, j) for j in range(1, n)])
    assert oracle.degree(star, "in")[0] == n - 1 and oracle.degree(star, "out")[0] == 0
