"""Mixed batches (block-diagonal unions of graphs), captured plans (runs
recorded as one HIP graph and replayed by a single launch) and the autotuner.

Every result is compared with the FP64/integer oracle or with the plain GPU
call it stands for: bit-exact for BFS, SSSP, TC and batched BFS/SSSP; PageRank
max relative error <= 1e-5, PPR per-seed L1 relative <= 1e-5. Plans are
replayed several times with eager work and synchronisations in between, and
every replay is checked."""
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
P_DAG = gm.GM_PREP_UPPER_DAG


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.int32, device=DEV)


def l1_rel(got, ref):
    return float(np.abs(got - ref).sum() / np.abs(ref).sum())


# ---------------------------------------------------------------- union ----
def small_parts():
    specs = [(8, 21), (6, 22), (10, 23)]
    return [(sc, seed) + gg.rmat(sc, seed=seed) for sc, seed in specs]


def test_union_edges_are_parts_shifted():
    parts = small_parts()
    gs = [gm.Graph.from_coo(n, s, d, prep=P_SYM) for _, _, n, s, d in parts]
    u = gm.Graph.union(gs)
    base = gm.union_bases(gs)
    us, ud = u.edges()
    es = np.concatenate([g.edges()[0] + b for g, b in zip(gs, base)])
    ed = np.concatenate([g.edges()[1] + b for g, b in zip(gs, base)])
    assert np.array_equal(us, es) and np.array_equal(ud, ed)
    info = u.info()
    assert info.n == base[-1] and info.m == sum(g.m for g in gs)
    assert info.max_out == max(g.info().max_out for g in gs)


def test_union_bfs_and_pagerank_equal_solo_oracle():
    parts = small_parts()
    gsym = [gm.Graph.from_coo(n, s, d, prep=P_SYM) for _, _, n, s, d in parts]
    gdir = [gm.Graph.from_coo(n, s, d) for _, _, n, s, d in parts]
    usym, udir = gm.Graph.union(gsym), gm.Graph.union(gdir)
    base = gm.union_bases(gsym)
    N = int(base[-1])
    lv = torch.full((N,), gm.INF_LEVEL, dtype=torch.int32, device=DEV)
    lv[torch.tensor(base[:-1], device=DEV)] = 0
    it = gm.run_vertex_program(usym, gm.GM_PROG_BFS, dev(base[:-1]), -1, lv)
    pr = torch.ones(N, dtype=torch.float32, device=DEV)
    gm.run_vertex_program(udir, gm.GM_PROG_PAGERANK, None, 20, pr)
    lv, pr = lv.cpu().numpy(), pr.cpu().numpy()
    maxlev = 0
    for (_, _, n, s, d), b in zip(parts, base):
        ref = oracle.bfs(oracle.prepare(n, s, d, mode="symmetric"), 0)
        assert np.array_equal(lv[b:b + n], ref)
        maxlev = max(maxlev, int(ref[ref != oracle.INF_I32].max()))
        assert W.max_rel_err(pr[b:b + n], oracle.pagerank(oracle.prepare(n, s, d), 0.15, 20)) <= 1e-5
    assert it == maxlev + 1


def test_union_argument_errors():
    n, s, d = W.raw(8)
    a = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    b = gm.Graph.from_coo(n, s, d, prep=P_DIR)
    with pytest.raises(gm.GmError) as e:
        gm.Graph.union([a, b])
    assert e.value.status == gm._lib.GM_EINVAL
    R = gg.cf_ratings(n_users=50, n_items=20, total=400, dmin=2)
    rg = gm.RatingGraph.from_coo(R.n_users, R.n_items, R.user, R.item, R.rating)
    with pytest.raises(gm.GmError) as e:
        gm.Graph.union([rg])
    assert e.value.status == gm._lib.GM_EUNSUPPORTED


# ---------------------------------------------------------------- plans ----
def test_plan_single_source_programs_replayed():
    """BFS, SSSP, PageRank and TC recorded in one plan; three launches with
    eager work in between, the sources changed between launches."""
    sc = W.SMALL_SCALE
    n, s, d = W.raw(sc)
    gsym = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    gdir = gm.Graph.from_coo(n, s, d, w=W.weights(sc), prep=P_DIR)
    gdag = gm.Graph.from_coo(n, s, d, prep=P_DAG)
    src = dev([0])
    lv = torch.empty(n, dtype=torch.int32, device=DEV)
    dist = torch.empty(n, dtype=torch.int32, device=DEV)
    pr = torch.empty(n, dtype=torch.float32, device=DEV)
    tri = torch.empty(n, dtype=torch.int64, device=DEV)
    plan = gm.Plan([gm.PlanRun(gsym, gm.GM_PROG_BFS, lv, src, max_iters=16),
                    gm.PlanRun(gdir, gm.GM_PROG_SSSP, dist, src, max_iters=40),
                    gm.PlanRun(gdir, gm.GM_PROG_PAGERANK, pr, max_iters=20),
                    gm.PlanRun(gdag, gm.GM_PROG_TC, tri)])
    osym, odir = W.ograph(sc, "symmetric"), W.ograph(sc, "directed", True)
    ref_pr = W.pagerank(sc)
    odag = W.ograph(sc, "dag")
    ref_tri = oracle.triangles_at(odag.transpose(), np.arange(n))
    for rep, root in enumerate([0, 0, 17]):
        src.fill_(root)
        plan.launch()
        res = plan.results()
        ref_lv = oracle.bfs(osym, root)
        assert np.array_equal(lv.cpu().numpy(), ref_lv), "replay %d" % rep
        assert res[0][0] == int(ref_lv[ref_lv != oracle.INF_I32].max()) + 1 and res[0][1] == 1
        ref_d = oracle.sssp(odir, root)
        assert np.array_equal(dist.cpu().numpy().view(np.uint32), ref_d)
        assert res[1][1] == 1
        assert W.max_rel_err(pr.cpu().numpy(), ref_pr) <= 1e-5
        assert np.array_equal(tri.cpu().numpy().astype(np.uint64), ref_tri)
        assert res[2] == (20, 1, 20 * gdir.m) and res[3][0] == 1
        # eager work between replays: the plain calls on the same graphs
        lv2 = torch.full((n,), gm.INF_LEVEL, dtype=torch.int32, device=DEV)
        lv2[root] = 0
        it = gm.run_vertex_program(gsym, gm.GM_PROG_BFS, dev([root]), -1, lv2)
        assert np.array_equal(lv2.cpu().numpy(), ref_lv) and it == res[0][0]
        torch.cuda.synchronize()


def test_plan_min_programs_match_plain_edges_and_supersteps():
    sc = 12
    n, s, d = W.raw(sc)
    gdir = gm.Graph.from_coo(n, s, d, w=W.weights(sc), prep=P_DIR)
    dist = torch.empty(n, dtype=torch.int32, device=DEV)
    plan = gm.Plan([gm.PlanRun(gdir, gm.GM_PROG_SSSP, dist, dev([3]), max_iters=64)])
    plan.launch()
    it, conv, edges = plan.results()[0]
    ref = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    ref[3] = 0
    pit = gm.run_vertex_program(gdir, gm.GM_PROG_SSSP, dev([3]), -1, ref)
    assert np.array_equal(dist.cpu().numpy(), ref.cpu().numpy())
    assert (it, conv, edges) == (pit, 1, gdir.last_run_stats().edges_scanned)


def test_plan_not_converged_is_reported():
    sc = W.SMALL_SCALE
    n, s, d = W.raw(sc)
    gsym = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    lv = torch.empty(n, dtype=torch.int32, device=DEV)
    plan = gm.Plan([gm.PlanRun(gsym, gm.GM_PROG_BFS, lv, dev([0]), max_iters=2)])
    plan.launch()
    assert plan.results()[0][:2] == (2, 0)
    ref = torch.full((n,), gm.INF_LEVEL, dtype=torch.int32, device=DEV)
    ref[0] = 0
    gm.run_vertex_program(gsym, gm.GM_PROG_BFS, dev([0]), 2, ref)
    assert np.array_equal(lv.cpu().numpy(), ref.cpu().numpy())
    # the next launch starts clean (no frontier left over)
    plan.launch()
    assert np.array_equal(lv.cpu().numpy(), ref.cpu().numpy())


def test_plan_batched_runs_equal_gm_run_batched():
    sc = W.SMALL_SCALE
    n, s, d = W.raw(sc)
    gsym = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    gdir = gm.Graph.from_coo(n, s, d, w=W.weights(sc), prep=P_DIR)
    S = dev(gg.sources(n, s, d, 64, gg.SEED_BATCH_SOURCES))
    P = dev(gg.sources(n, s, d, 100, gg.SEED_PPR_SEEDS))
    bl = torch.empty((n, 64), dtype=torch.int32, device=DEV)
    bd = torch.empty((n, 64), dtype=torch.int32, device=DEV)
    bp = torch.empty((n, P.numel()), dtype=torch.float32, device=DEV)
    plan = gm.Plan([gm.PlanRun(gsym, gm.GM_PROG_BFS, bl, S, max_iters=16, batched=True),
                    gm.PlanRun(gdir, gm.GM_PROG_SSSP, bd, S, max_iters=48, batched=True),
                    gm.PlanRun(gdir, gm.GM_PROG_PPR, bp, P, max_iters=20, batched=True)])
    for rep in range(2):
        plan.launch()
        res = plan.results()
        rl = torch.empty_like(bl)
        it = gm.run_batched(gsym, gm.GM_PROG_BFS, S, -1, rl)
        assert np.array_equal(bl.cpu().numpy(), rl.cpu().numpy()) and res[0][:2] == (it, 1)
        rd = torch.empty_like(bd)
        it = gm.run_batched(gdir, gm.GM_PROG_SSSP, S, -1, rd)
        assert np.array_equal(bd.cpu().numpy(), rd.cpu().numpy()) and res[1][:2] == (it, 1)
        og, ogin = W.ograph(sc, "directed"), W.otranspose(sc, "directed")
        got = bp.cpu().numpy()
        for j in (0, 50, P.numel() - 1):
            ref = oracle.personalized_pagerank(og, int(P[j]), 0.15, 20, g_in=ogin)
            assert l1_rel(got[:, j], ref) <= 1e-5
        torch.cuda.synchronize()


def test_plan_goes_stale_when_the_workspace_changes():
    n, s, d = W.raw(10)
    g = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    lv = torch.empty(n, dtype=torch.int32, device=DEV)
    plan = gm.Plan([gm.PlanRun(g, gm.GM_PROG_BFS, lv, dev([0]), max_iters=8)])
    plan.launch()
    g.set_tuning(pull_div=7)
    with pytest.raises(gm.GmError) as e:
        plan.launch()
    assert e.value.status == gm._lib.GM_ESTATE
    # a new plan works
    plan2 = gm.Plan([gm.PlanRun(g, gm.GM_PROG_BFS, lv, dev([0]), max_iters=8)])
    plan2.launch()
    assert np.array_equal(lv.cpu().numpy(), oracle.bfs(W.ograph(10, "symmetric"), 0))


def test_plan_argument_errors():
    n, s, d = W.raw(8)
    g = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    lv = torch.empty(n, dtype=torch.int32, device=DEV)
    for bad in (0, 65):
        with pytest.raises(gm.GmError) as e:
            gm.Plan([gm.PlanRun(g, gm.GM_PROG_BFS, lv, dev([0]), max_iters=bad)])
        assert e.value.status == gm._lib.GM_EINVAL
    with pytest.raises(gm.GmError) as e:
        gm.Plan([gm.PlanRun(g, gm.GM_PROG_BFS, lv, dev([n]), max_iters=8)])
    assert e.value.status == gm._lib.GM_EINVAL
    with pytest.raises(gm.GmError) as e:
        gm.Plan([gm.PlanRun(g, gm.GM_PROG_PPR, lv.float(), dev([0]), max_iters=8)])
    assert e.value.status == gm._lib.GM_EUNSUPPORTED


# ------------------------------------------------------------ mixed batch --
MIXED = gg.mixed_batch_specs()


@pytest.fixture(scope="module")
def mixed():
    raws = [gg.rmat(sc, seed=seed) for sc, seed in MIXED]
    gsym = [gm.Graph.from_coo(n, s, d, prep=P_SYM) for n, s, d in raws]
    gdir = [gm.Graph.from_coo(n, s, d) for n, s, d in raws]
    return raws, gsym, gdir


def test_mixed_batch_one_launch_equals_solo_runs(mixed):
    """32 RMAT graphs of scales 12-18 (2,142,208 vertices): BFS from each
    graph's vertex 0 and 20 PageRank supersteps, all in one plan launch."""
    raws, gsym, gdir = mixed
    usym, udir = gm.Graph.union(gsym), gm.Graph.union(gdir)
    base = gm.union_bases(gsym)
    N = int(base[-1])
    assert N == 2_142_208
    roots = dev(base[:-1])
    lv = torch.empty(N, dtype=torch.int32, device=DEV)
    pr = torch.empty(N, dtype=torch.float32, device=DEV)
    plan = gm.Plan([gm.PlanRun(usym, gm.GM_PROG_BFS, lv, roots, max_iters=32),
                    gm.PlanRun(udir, gm.GM_PROG_PAGERANK, pr, max_iters=20)])
    plan.launch()
    res = plan.results()
    assert res[0][1] == 1
    lv, pr = lv.cpu().numpy(), pr.cpu().numpy()
    its = []
    for i, ((n, s, d), gs, gd) in enumerate(zip(raws, gsym, gdir)):
        b = int(base[i])
        ref = torch.full((n,), gm.INF_LEVEL, dtype=torch.int32, device=DEV)
        ref[0] = 0
        its.append(gm.run_vertex_program(gs, gm.GM_PROG_BFS, dev([0]), -1, ref))
        assert np.array_equal(lv[b:b + n], ref.cpu().numpy()), "graph %d" % i
        rp = torch.ones(n, dtype=torch.float32, device=DEV)
        gm.run_vertex_program(gd, gm.GM_PROG_PAGERANK, None, 20, rp)
        assert W.max_rel_err(pr[b:b + n], rp.cpu().numpy()) <= 2e-6, "graph %d" % i
        if i % 7 in (0, 6):  # the oracle on one graph of the smallest and largest scale
            assert np.array_equal(lv[b:b + n], oracle.bfs(oracle.prepare(n, s, d, mode="symmetric"), 0))
            assert W.max_rel_err(pr[b:b + n], oracle.pagerank(oracle.prepare(n, s, d), 0.15, 20)) <= 1e-5
    assert res[0][0] == max(its)


# -------------------------------------------------------------- autotune ---
def test_autotune_keeps_results_and_sets_values():
    sc = W.SMALL_SCALE
    n, s, d = W.raw(sc)
    gsym = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    t = gm.autotune(gsym, gm.GM_PROG_BFS, dev([0]), trials=2)
    assert t == gsym.tuning()
    assert t["pull_div"] in (16, 32, 64, 128, 256, 512)
    lv = torch.full((n,), gm.INF_LEVEL, dtype=torch.int32, device=DEV)
    lv[0] = 0
    gm.run_vertex_program(gsym, gm.GM_PROG_BFS, dev([0]), -1, lv)
    assert np.array_equal(lv.cpu().numpy(), W.bfs_levels(sc))
    gdir = gm.Graph.from_coo(n, s, d, w=W.weights(sc), prep=P_DIR)
    P = dev(gg.sources(n, s, d, 64, gg.SEED_PPR_SEEDS))
    t = gm.autotune(gdir, gm.GM_PROG_PPR, P, batched=True, max_iters=20, trials=2)
    assert t["ppr_chunk"] in (128, 256, 512, 1024, 2048, 4096)
    bp = torch.empty((n, 64), dtype=torch.float32, device=DEV)
    gm.run_batched(gdir, gm.GM_PROG_PPR, P, 20, bp)
    og, ogin = W.ograph(sc, "directed"), W.otranspose(sc, "directed")
    ref = oracle.personalized_pagerank(og, int(P[5]), 0.15, 20, g_in=ogin)
    assert l1_rel(bp.cpu().numpy()[:, 5], ref) <= 1e-5
    t = gm.autotune(gdir, gm.GM_PROG_SSSP, dev([0]), trials=2)
    assert t["pull_div"] in (64, 128, 256, 512, 1024)
    dist = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    dist[0] = 0
    assert gm.run_vertex_program(gdir, gm.GM_PROG_SSSP, dev([0]), -1, dist) == W.sssp_supersteps(sc)
    assert np.array_equal(dist.cpu().numpy().view(np.uint32), W.sssp_dist(sc))
    gdag = gm.Graph.from_coo(n, s, d, prep=P_DAG)
    t = gm.autotune(gdag, gm.GM_PROG_TC, trials=1)
    assert gm.triangle_count(gdag) == oracle.triangle_count(W.ograph(sc, "dag"))


def test_tuning_range_checks():
    n, s, d = W.raw(8)
    g = gm.Graph.from_coo(n, s, d)
    with pytest.raises(gm.GmError):
        g.set_tuning(superstep_batch=0)
    with pytest.raises(gm.GmError):
        g.set_tuning(tc_wave_max=2048)
    g.set_tuning(push_blocks=1024)
    assert g.tuning()["push_blocks"] == 1024
