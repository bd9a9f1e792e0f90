"""GPU BFS (Sec. 3 II) and SSSP (Sec. 3 V) against the oracle: bit-exact
properties and the superstep counts of Alg. 2."""
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
DEG = gm._lib.GM_VARIANT_DEGREE_ORDER


def ids(*v):
    return torch.tensor(list(v), dtype=torch.int32, device=DEV)


def run_bfs(g, n, roots, max_iters=-1):
    level = torch.full((n,), gm.INF_LEVEL, dtype=torch.int32, device=DEV)
    level[torch.as_tensor(roots, dtype=torch.long)] = 0
    active = torch.zeros(n, dtype=torch.int32, device=DEV)
    it = gm.run_vertex_program(g, gm.GM_PROG_BFS, ids(*roots), max_iters, level, active)
    return level.cpu().numpy(), it, active.cpu().numpy()


def run_sssp(g, n, source, max_iters=-1, prop=None, frontier=None):
    if prop is None:
        prop = torch.full((n,), -1, dtype=torch.int32, device=DEV)  # UINT32_MAX bits
        prop[source] = 0
        frontier = ids(source)
    active = torch.zeros(n, dtype=torch.int32, device=DEV)
    it = gm.run_vertex_program(g, gm.GM_PROG_SSSP, frontier, max_iters, prop, active)
    return prop.cpu().numpy().view(np.uint32), it, active.cpu().numpy()


@pytest.mark.parametrize("scale", [W.SMALL_SCALE, W.FULL_SCALE])
def test_bfs_rmat(scale):
    n, s, d = W.raw(scale)
    g = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    level, it, active = run_bfs(g, n, [0])
    ref = W.bfs_levels(scale)
    assert np.array_equal(level, ref)
    assert it == int(ref[ref != oracle.INF_I32].max()) + 1
    assert not active.any()
    st = g.last_run_stats()
    # Alg. 1 traverses the out-edges of every vertex that sends: all reached ones
    og = W.ograph(scale, "symmetric")
    assert st.edges_scanned == int(og.degree()[ref != oracle.INF_I32].sum())


@pytest.mark.parametrize("scale", [W.SMALL_SCALE, W.FULL_SCALE])
def test_sssp_rmat(scale):
    n, s, d = W.raw(scale)
    g = gm.Graph.from_coo(n, s, d, w=W.weights(scale), prep=P_DIR)
    dist, it, active = run_sssp(g, n, 0)
    assert np.array_equal(dist, W.sssp_dist(scale))
    assert it == W.sssp_supersteps(scale)
    assert not active.any()


def test_sssp_resume_equals_uninterrupted():
    scale = 12
    n, s, d = W.raw(scale)
    g = gm.Graph.from_coo(n, s, d, w=W.weights(scale), prep=P_DIR)
    full, it_full, _ = run_sssp(g, n, 0)
    prop = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    prop[0] = 0
    d1, it1, act1 = run_sssp(g, n, 0, max_iters=3, prop=prop, frontier=ids(0))
    assert it1 == 3 and act1.any()
    fr = torch.tensor(np.flatnonzero(act1), dtype=torch.int32, device=DEV)
    d2, it2, _ = run_sssp(g, n, 0, prop=prop, frontier=fr)
    assert np.array_equal(d2, full) and it1 + it2 == it_full
    # the oracle's Alg. 2 agrees on the intermediate state after 3 supersteps
    og = W.ograph(scale, "directed", True)
    p0 = np.full(n, oracle.INF_U32, dtype=np.uint32)
    p0[0] = 0
    a0 = np.zeros(n, dtype=bool)
    a0[0] = True
    po, ao, _ = oracle.run_min_program(og, p0, a0, weighted=True, max_iters=3)
    assert np.array_equal(d1, po) and np.array_equal(act1.astype(bool), ao)


def test_bfs_multi_root_empty_and_isolated():
    n = 50
    s = np.arange(0, 20, dtype=np.int32)
    d = np.arange(1, 21, dtype=np.int32)  # path 0..20, vertices 21..49 isolated
    g = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    og = oracle.prepare(n, s, d, mode="symmetric")
    level, it, _ = run_bfs(g, n, [0, 20])
    assert np.array_equal(level, oracle.bfs(og, [0, 20]))
    assert it == 11
    level, it, _ = run_bfs(g, n, [30])
    assert it == 1 and level[30] == 0 and (np.delete(level, 30) == gm.INF_LEVEL).all()
    # empty frontier: nothing runs, nothing changes
    lv = torch.full((n,), 5, dtype=torch.int32, device=DEV)
    assert gm.run_vertex_program(g, gm.GM_PROG_BFS, ids(), -1, lv) == 0
    assert (lv.cpu().numpy() == 5).all()


def test_hub_chunks_and_long_path():
    """A star whose centre has far more out-edges than the hub chunk, plus a
    long path (many supersteps, one vertex each)."""
    leaves = 20000
    n = leaves + 1 + 3000
    s = np.concatenate([np.zeros(leaves, np.int32), np.arange(leaves + 1, n - 1, dtype=np.int32),
                        np.array([5], np.int32)])
    d = np.concatenate([np.arange(1, leaves + 1, dtype=np.int32),
                        np.arange(leaves + 2, n, dtype=np.int32), np.array([leaves + 1], np.int32)])
    w = gg.weights_u32(s, d)
    g = gm.Graph.from_coo(n, s, d, w=w, prep=P_DIR)
    og = oracle.prepare(n, s, d, w=w)
    dist, it, _ = run_sssp(g, n, 0)
    assert np.array_equal(dist, oracle.sssp(og, 0))
    gs = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    level, it, _ = run_bfs(gs, n, [0])
    ref = oracle.bfs(oracle.prepare(n, s, d, mode="symmetric"), 0)
    assert np.array_equal(level, ref) and it == ref[ref != oracle.INF_I32].max() + 1


def test_bfs_deterministic_repeats():
    n, s, d = W.raw(16)
    g = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    first = run_bfs(g, n, [0])[0]
    for _ in range(3):
        assert np.array_equal(run_bfs(g, n, [0])[0], first)


def test_sssp_unit_weights_equal_directed_bfs():
    n, s, d = W.raw(12)
    g = gm.Graph.from_coo(n, s, d, w=np.ones(len(s), np.uint32), prep=P_DIR)
    dist, _, _ = run_sssp(g, n, 0)
    lvl = oracle.bfs(oracle.prepare(n, s, d), 0)
    assert np.array_equal(dist, np.where(lvl == oracle.INF_I32, oracle.INF_U32, lvl).astype(np.uint32))


def test_argument_errors_on_device():
    n, s, d = W.raw(10)
    g = gm.Graph.from_coo(n, s, d, prep=P_DIR)
    lv = torch.zeros(n, dtype=torch.int32, device=DEV)
    with pytest.raises(gm.GmError) as e:
        gm.run_vertex_program(g, gm.GM_PROG_BFS, ids(n + 5), -1, lv)
    assert e.value.status == gm._lib.GM_EINVAL
    with pytest.raises(gm.GmError) as e:  # SSSP on an unweighted graph
        gm.run_vertex_program(g, gm.GM_PROG_SSSP, ids(0), -1, lv)
    assert e.value.status == gm._lib.GM_EUNSUPPORTED
    with pytest.raises(gm.GmError) as e:  # PageRank needs max_iters > 0
        gm.run_vertex_program(g, gm.GM_PROG_PAGERANK, None, 0, lv.float())
    assert e.value.status == gm._lib.GM_EINVAL


def test_binding_checks_device_buffers():
    n, s, d = W.raw(8)
    g = gm.Graph.from_coo(n, s, d, prep=P_DIR)
    lv = torch.zeros(n, dtype=torch.int32, device=DEV)
    with pytest.raises(ValueError, match="elements"):  # shorter than n
        gm.run_vertex_program(g, gm.GM_PROG_BFS, ids(0), -1, lv[: n - 1])
    with pytest.raises(ValueError, match="dtype"):  # ranks are float32
        gm.run_vertex_program(g, gm.GM_PROG_PAGERANK, None, 2, lv)
    with pytest.raises(ValueError, match="device tensor"):
        gm.run_vertex_program(g, gm.GM_PROG_BFS, ids(0), -1, lv.cpu())
    with pytest.raises(ValueError, match="dtype"):  # frontier ids are int32
        gm.run_vertex_program(g, gm.GM_PROG_BFS, ids(0).long(), -1, lv)
    with pytest.raises(ValueError, match="elements"):  # n x k block for k = 2
        gm.run_batched(g, gm.GM_PROG_BFS, ids(0, 1), -1, lv)
    with pytest.raises(ValueError, match="elements"):
        gm.pagerank_forward_w(g, torch.ones(g.m, device=DEV), 0.15, 3,
                              torch.empty((3, n), dtype=torch.float32, device=DEV))
    R = gg.cf_ratings(n_users=50, n_items=20, total=400, dmin=2)
    rg = gm.RatingGraph.from_coo(R.n_users, R.n_items, R.user, R.item, R.rating)
    loss = torch.empty(1, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError, match="rows"):  # P_V must have one row per item
        gm.cf_forward(rg, torch.zeros((50, 4), device=DEV), torch.zeros((19, 4), device=DEV),
                      0.05, loss)
    # nothing above reached a kernel: the same buffers still work
    lv[0] = 0
    lv[1:] = gm.INF_LEVEL
    assert gm.run_vertex_program(g, gm.GM_PROG_BFS, ids(0), -1, lv) >= 1


def test_sssp_saturating_weights():
    # path sums beyond 2^32 - 1 clamp to UINT32_MAX, as in the oracle
    from tests.test_oracle_bfs_sssp import SAT_DIST, SAT_PAIRS, SAT_W
    s = np.array([p[0] for p in SAT_PAIRS], np.int32)
    d = np.array([p[1] for p in SAT_PAIRS], np.int32)
    g = gm.Graph.from_coo(6, s, d, w=SAT_W, prep=P_DIR)
    dist, _, _ = run_sssp(g, 6, 0)
    assert dist.tolist() == SAT_DIST
    block = torch.empty((6, 2), dtype=torch.int32, device=DEV)
    gm.run_batched(g, gm.GM_PROG_SSSP, ids(0, 5), -1, block)
    out = block.cpu().numpy().view(np.uint32)
    og = oracle.prepare(6, s, d, w=SAT_W)
    assert out[:, 0].tolist() == SAT_DIST
    assert np.array_equal(out[:, 1], oracle.sssp(og, 5))


def test_sssp_superstep_trace_hand_worked():
    """The hand-worked trace of golden/sssp_supersteps_hand.txt: after k
    supersteps (a run capped at k, from the initial state) the GPU holds the
    hand-derived distances and active set; the full run takes exactly 5."""
    n, s, d, w, src, trace, steps = W.sssp_hand_trace()
    g = gm.Graph.from_coo(n, s, d, w=w, prep=P_DIR)
    for k, (dist_k, act_k) in enumerate(trace, start=1):
        dist, it, active = run_sssp(g, n, src, max_iters=k)
        assert it == k and np.array_equal(dist, dist_k), k
        assert np.array_equal(active.astype(bool), act_k), k
    dist, it, active = run_sssp(g, n, src)
    assert it == steps and np.array_equal(dist, trace[-1][0]) and not active.any()


def tile_edge_graph():
    """A graph for the SSSP pull's tile layout: vertex 0 has an edge to every
    vertex with in-edges; in-degrees are picked so that rows end one edge
    before, on and one edge after multiples of the 1,024-edge tile, one row
    has 5,001 in-edges (spanning several tiles), every third vertex has no
    in-edge at all (interspersed empty rows), and the edge count is not a
    multiple of the tile. No duplicate edges and no self-loops, so the
    in-offsets are the cumulative sums of the in-degrees below."""
    rng = np.random.default_rng(1234)
    n = 6000
    empty = np.arange(n) % 3 == 2
    empty[0] = True
    targets = np.flatnonzero(~empty)
    deg = rng.integers(0, 40, size=len(targets))  # in-edges besides the one from 0
    deg[1500] = 5000
    for t, delta in ((2048, -1), (6144, 0), (9216, 1)):
        off = np.cumsum(deg + 1)
        i = int(np.searchsorted(off, t))
        deg[i] -= off[i] - (t + delta)  # row i now ends at t + delta
        assert deg[i] >= 0
    src, dst = [], []
    pool = np.arange(1, n)
    for v, k in zip(targets, deg):
        u = rng.choice(pool[pool != v], size=int(k), replace=False)
        src.append(np.concatenate([[0], u]))
        dst.append(np.full(int(k) + 1, v))
    return n, np.concatenate(src).astype(np.int32), np.concatenate(dst).astype(np.int32)


@pytest.mark.parametrize("pull_div", [1, 128, 65536])
def test_sssp_pull_tile_layout_cases(pull_div):
    """Every superstep's distances and frontier against the oracle's Alg. 2
    superstep loop, pushing only, by default, and pulling almost always."""
    n, s, d = tile_edge_graph()
    w = gg.weights_u32(s, d)
    g = gm.Graph.from_coo(n, s, d, w=w, prep=P_DIR)
    g.set_tuning(pull_div=pull_div)
    og = oracle.prepare(n, s, d, w=w)
    m = og.off[-1]
    assert m % 1024 != 0 and g.m == m
    prop0 = np.full(n, oracle.INF_U32, np.uint32)
    prop0[0] = 0
    act0 = np.zeros(n, bool)
    act0[0] = True
    _, _, steps = oracle.run_min_program(og, prop0, act0, True)
    for k in range(1, steps + 1):
        ref_p, ref_a, it = oracle.run_min_program(og, prop0, act0, True, max_iters=k)
        dist, it_g, active = run_sssp(g, n, 0, max_iters=k)
        assert it_g == it and np.array_equal(dist, ref_p), k
        assert np.array_equal(active.astype(bool), ref_a), k
    dist, it_g, _ = run_sssp(g, n, 0)
    assert it_g == steps and np.array_equal(dist, oracle.sssp(og, 0))
    st = g.last_run_stats()
    if pull_div == 1:
        assert st.pull_supersteps == 0
    if pull_div == 65536:
        assert st.pull_supersteps > 0


@pytest.mark.parametrize("name", ["sssp_rmat24_a50", "sssp_grid2048"])
def test_paper_sssp_workloads(name):
    """The paper's SSSP graphs (f3): RMAT scale 24 with a = .50, b = c = .10
    (Sec. 5.1, Table 1) and a long-diameter 2048 x 2048 grid; every distance
    against the oracle's Dijkstra (SHA-256 of the whole array in the
    oracle-written golden file) and the superstep count of its Alg. 2 loop."""
    from tests.golden import make_sssp_goldens as G
    ref = G.read(name)
    n, s, d, w, _ = G.workload(name)
    g = gm.Graph.from_coo(n, s, d, w=w, prep=P_DIR)
    assert g.m == ref["m"]
    dist, it, active = run_sssp(g, n, 0)
    assert it == ref["supersteps"] and not active.any()
    reached = dist != oracle.INF_U32
    assert int(reached.sum()) == ref["reached"] and int(dist[reached].max()) == ref["max_dist"]
    import hashlib
    assert hashlib.sha256(np.ascontiguousarray(dist, dtype="<u4").tobytes()).hexdigest() == \
        ref["dist_sha256"]


@pytest.mark.parametrize("labels", [0, DEG])
def test_orders_in_and_all(labels):
    """Messages along in-edges (GM_ORDER_IN) equal the run on the transposed
    graph; along both (GM_ORDER_ALL) the run on the union of the graph and its
    transpose (a pair in both directions keeps the smaller weight): BFS and
    SSSP from several sources against the oracle, on the caller's labels and on
    the degree-ordered copy of each adjacency."""
    scale = 12
    n, s, d = W.raw(scale)
    w = W.weights(scale)
    g = gm.Graph.from_coo(n, s, d, w=w, prep=P_DIR)
    g.set_tuning(variant=labels)
    og_in = oracle.prepare(n, d, s, w=w)                      # transposed
    og_all = oracle.prepare(n, np.concatenate([s, d]), np.concatenate([d, s]),
                            w=np.concatenate([w, w]))          # both directions
    for src in (0, 7, 1234):
        for order, og in ((gm.GM_ORDER_IN, og_in), (gm.GM_ORDER_ALL, og_all)):
            lv = torch.full((n,), gm.INF_LEVEL, dtype=torch.int32, device=DEV)
            lv[src] = 0
            gm.run_vertex_program(g, gm.GM_PROG_BFS, ids(src), -1, lv, order=order)
            assert np.array_equal(lv.cpu().numpy(), oracle.bfs(og, src)), (order, src)
            dist = torch.full((n,), -1, dtype=torch.int32, device=DEV)
            dist[src] = 0
            gm.run_vertex_program(g, gm.GM_PROG_SSSP, ids(src), -1, dist, order=order)
            assert np.array_equal(dist.cpu().numpy().view(np.uint32), oracle.sssp(og, src))


@pytest.mark.parametrize("labels", [0, DEG])
def test_degree_program_all_orders(labels):
    """Fig. 1: degree as one generalized SpMV with a ones vector, along out-,
    in- and both directions, against the oracle's counts (RMAT scale 14 and
    a graph with isolated and edgeless vertices)."""
    for n, s, d in (W.raw(W.SMALL_SCALE), (50, np.array([3, 3, 4], np.int32),
                                           np.array([4, 5, 3], np.int32))):
        g = gm.Graph.from_coo(n, s, d)
        g.set_tuning(variant=labels)
        og = oracle.prepare(n, s, d)
        for order, name in ((gm.GM_ORDER_OUT, "out"), (gm.GM_ORDER_IN, "in"),
                            (gm.GM_ORDER_ALL, "all")):
            deg = torch.full((n,), 77, dtype=torch.int32, device=DEV)  # overwritten from 0
            it = gm.run_vertex_program(g, gm.GM_PROG_DEGREE, None, 1, deg, order=order)
            assert it == (1 if n > 0 else 0)
            assert np.array_equal(deg.cpu().numpy().astype(np.int64), oracle.degree(og, name))


def test_order_errors():
    n, s, d = W.raw(8)
    g = gm.Graph.from_coo(n, s, d, layouts=gm.GM_LAYOUT_OUT)
    lv = torch.zeros(n, dtype=torch.int32, device=DEV)
    with pytest.raises(gm.GmError) as e:  # IN needs the in-layout
        gm.run_vertex_program(g, gm.GM_PROG_BFS, ids(0), -1, lv, order=gm.GM_ORDER_IN)
    assert e.value.status == gm._lib.GM_EUNSUPPORTED
    g2 = gm.Graph.from_coo(n, s, d)
    pr = torch.ones(n, dtype=torch.float32, device=DEV)
    with pytest.raises(gm.GmError) as e:  # PageRank runs along out-edges only
        gm.run_vertex_program(g2, gm.GM_PROG_PAGERANK, None, 20, pr, order=gm.GM_ORDER_IN)
    assert e.value.status == gm._lib.GM_EUNSUPPORTED
    with pytest.raises(gm.GmError) as e:
        gm.run_vertex_program(g2, gm.GM_PROG_BFS, ids(0), -1, lv, order=9)
    assert e.value.status == gm._lib.GM_EINVAL
    with pytest.raises(gm.GmError) as e:  # the degree program takes no frontier
        gm.run_vertex_program(g2, gm.GM_PROG_DEGREE, ids(0), 1, lv)
    assert e.value.status == gm._lib.GM_EINVAL
