"""GPU tests of the boundary's frontier forms, preparation and release, the
multi-graph run and the autotuner cache (through the C ABI), each against
the oracle or the plain single-graph run."""
import json
import os

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


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.int32, device=DEV)


def bitmap_of(n, verts):
    words = np.zeros((n + 31) // 32, dtype=np.uint32)
    for v in verts:
        words[v >> 5] |= np.uint32(1 << (v & 31))
    return torch.tensor(words.view(np.int32), device=DEV)


@pytest.mark.parametrize("labels", [0, gm._lib.GM_VARIANT_DEGREE_ORDER])
def test_bitmap_frontier_equals_ids(labels):
    """The bitvector sparse vector of Sec. 4.4.2 as the first frontier: BFS and
    SSSP from several sources equal the oracle and the id-list runs; bits at or
    past n are ignored; an empty bitmap runs no superstep. On the caller's
    labels and on the degree-ordered copy of the adjacency."""
    scale = 12
    n, s, d = W.raw(scale)
    srcs = [0, 5, 77, n - 1]
    g = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    g.set_tuning(variant=labels)
    lv = torch.full((n,), gm.INF_LEVEL, dtype=torch.int32, device=DEV)
    lv[srcs] = 0
    bm = bitmap_of(n + 40, srcs + [n + 3, n + 39])  # stray bits past n
    it = gm.run_vertex_program(g, gm.GM_PROG_BFS, None, -1, lv, bitmap=bm)
    ref = oracle.bfs(W.ograph(scale, "symmetric"), srcs)
    assert np.array_equal(lv.cpu().numpy(), ref)
    lv2 = torch.full((n,), gm.INF_LEVEL, dtype=torch.int32, device=DEV)
    lv2[srcs] = 0
    assert gm.run_vertex_program(g, gm.GM_PROG_BFS, dev(srcs), -1, lv2) == it
    assert torch.equal(lv, lv2)
    gw = gm.Graph.from_coo(n, s, d, w=W.weights(scale), prep=P_DIR)
    gw.set_tuning(variant=labels)
    dist = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    dist[srcs] = 0
    gm.run_vertex_program(gw, gm.GM_PROG_SSSP, None, -1, dist, bitmap=bitmap_of(n, srcs))
    refd = oracle.sssp(W.ograph(scale, "directed", True), srcs)
    assert np.array_equal(dist.cpu().numpy().view(np.uint32), refd)
    empty = torch.zeros((n + 31) // 32, dtype=torch.int32, device=DEV)
    keep = lv.clone()
    assert gm.run_vertex_program(g, gm.GM_PROG_BFS, None, -1, lv, bitmap=empty) == 0
    assert torch.equal(lv, keep)


def test_bitmap_frontier_errors():
    n, s, d = W.raw(8)
    g = gm.Graph.from_coo(n, s, d)
    lv = torch.zeros(n, dtype=torch.float32, device=DEV)
    bm = bitmap_of(n, [0])
    with pytest.raises(gm.GmError) as e:  # PPR takes its seed from ids
        gm.run_vertex_program(g, gm.GM_PROG_PPR, None, 20, lv, bitmap=bm)
    assert e.value.status == gm._lib.GM_EINVAL
    with pytest.raises(ValueError):
        gm.run_vertex_program(g, gm.GM_PROG_BFS, dev([0]), -1, lv, bitmap=bm)


def test_prepare_and_release():
    """Runs after gm_graph_prepare and after gm_graph_release equal a first
    run (results never depend on the schedules' lifetime)."""
    scale = 12
    n, s, d = W.raw(scale)
    gdag = gm.Graph.from_coo(n, s, d, prep=gm.GM_PREP_UPPER_DAG)
    gdag.prepare(gm.GM_PROG_TC)
    c1 = torch.zeros(n, dtype=torch.int64, device=DEV)
    t1 = gm.triangle_count(gdag, c1)
    gdag.release()
    c2 = torch.zeros(n, dtype=torch.int64, device=DEV)
    t2 = gm.triangle_count(gdag, c2)
    dag = W.ograph(scale, "dag")
    assert t1 == t2 == oracle.triangle_count(dag)
    assert torch.equal(c1, c2)
    gdir = gm.Graph.from_coo(n, s, d)
    for prep_first in (True, False):
        gdir.release()
        if prep_first:
            gdir.prepare(gm.GM_PROG_PAGERANK)
        pr = torch.ones(n, dtype=torch.float32, device=DEV)
        gm.run_vertex_program(gdir, gm.GM_PROG_PAGERANK, None, 20, pr)
        assert W.max_rel_err(pr.cpu().numpy(), W.pagerank(scale)) <= 1e-5
    gsym = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    gsym.prepare(gm.GM_PROG_BFS)
    lv = torch.full((n,), gm.INF_LEVEL, dtype=torch.int32, device=DEV)
    lv[0] = 0
    gm.run_vertex_program(gsym, gm.GM_PROG_BFS, dev([0]), -1, lv)
    assert np.array_equal(lv.cpu().numpy(), W.bfs_levels(scale))
    with pytest.raises(gm.GmError) as e:
        gsym.prepare(gm.GM_PROG_TC)
    assert e.value.status == gm._lib.GM_EUNSUPPORTED


def test_multi_graph_run_equals_solo_runs():
    """gm_run_multi_graph over graphs of uneven sizes (scales 8-12, one
    without edges): each graph's part equals its solo run and the oracle."""
    specs = [(8, 201), (12, 202), (10, 203), (9, 204)]
    raws = [gg.rmat(sc, seed=sd) for sc, sd in specs]
    none = np.zeros(0, np.int32)
    raws.append((37, none, none))
    sym = [gm.Graph.from_coo(a, b, c, prep=P_SYM, layouts=gm.GM_LAYOUT_OUT) for a, b, c in raws]
    srcs = [0, 3, -1, 7, 36]
    lvs = []
    for (a, _, _), sv in zip(raws, srcs):
        t = torch.full((a,), gm.INF_LEVEL, dtype=torch.int32, device=DEV)
        if sv >= 0:
            t[sv] = 0
        lvs.append(t)
    it = gm.run_multi_graph(sym, gm.GM_PROG_BFS, srcs, lvs, -1)
    its = []
    for (a, b, c), sv, lv in zip(raws, srcs, lvs):
        og = oracle.prepare(a, b, c, mode="symmetric")
        ref = oracle.bfs(og, sv) if sv >= 0 else np.full(a, oracle.INF_I32, np.int32)
        assert np.array_equal(lv.cpu().numpy(), ref)
        if sv >= 0:
            its.append(int(ref[ref != oracle.INF_I32].max()) + 1)
    assert it == max(its)
    # PageRank and triangle counts over the same graphs
    dirs = [gm.Graph.from_coo(a, b, c) for a, b, c in raws]
    prs = [torch.ones(a, dtype=torch.float32, device=DEV) for a, _, _ in raws]
    assert gm.run_multi_graph(dirs, gm.GM_PROG_PAGERANK, None, prs, 20) == 20
    for (a, b, c), pr in zip(raws, prs):
        ref = oracle.pagerank(oracle.prepare(a, b, c), 0.15, 20)
        assert W.max_rel_err(pr.cpu().numpy(), ref) <= 1e-5
    dags = [gm.Graph.from_coo(a, b, c, prep=gm.GM_PREP_UPPER_DAG) for a, b, c in raws]
    cnts = [torch.zeros(a, dtype=torch.int64, device=DEV) for a, _, _ in raws]
    gm.run_multi_graph(dags, gm.GM_PROG_TC, None, cnts, 1)
    for (a, b, c), cn in zip(raws, cnts):
        din = oracle.dag_in_lists(oracle.prepare(a, b, c, mode="dag"))
        assert np.array_equal(cn.cpu().numpy().view(np.uint64),
                              oracle.triangles_at(din, np.arange(a)))


def test_multi_graph_errors():
    n, s, d = W.raw(8)
    a = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    b = gm.Graph.from_coo(n, s, d)  # differs in prep
    lv = [torch.zeros(n, dtype=torch.int32, device=DEV) for _ in range(2)]
    with pytest.raises(gm.GmError) as e:
        gm.run_multi_graph([a, b], gm.GM_PROG_BFS, [0, 0], lv, -1)
    assert e.value.status == gm._lib.GM_EINVAL
    with pytest.raises(gm.GmError) as e:
        gm.run_multi_graph([a, a], gm.GM_PROG_BFS, [0, n], lv, -1)
    assert e.value.status == gm._lib.GM_EINVAL


def test_autotune_cache_roundtrip(tmp_path):
    """The autotuner writes its choice to the cache file under the key of
    (architecture, program, graph shape); a later call with the same key sets
    those values without timing, and results are unchanged."""
    scale = 12
    n, s, d = W.raw(scale)
    g = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    path = str(tmp_path / "tune.json")
    t1 = gm.autotune(g, gm.GM_PROG_BFS, dev([0]), trials=1, cache=path)
    entries = json.load(open(path))
    assert len(entries) == 1
    key, val = next(iter(entries.items()))
    assert "|bfs|batched=0|k=1|log2n=12|" in key and val == t1
    # a stored entry is taken as it is: make it recognisable, then read it back
    val2 = dict(val, pull_div=32, push_blocks=1024)
    json.dump({key: val2}, open(path, "w"))
    g2 = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    t2 = gm.autotune(g2, gm.GM_PROG_BFS, dev([0]), trials=1, cache=path)
    assert t2 == val2 and g2.tuning() == val2
    lv = torch.full((n,), gm.INF_LEVEL, dtype=torch.int32, device=DEV)
    lv[0] = 0
    gm.run_vertex_program(g2, gm.GM_PROG_BFS, dev([0]), -1, lv)
    assert np.array_equal(lv.cpu().numpy(), W.bfs_levels(scale))
    # another program adds an entry; a damaged file is refused
    gd = gm.Graph.from_coo(n, s, d)
    gm.autotune(gd, gm.GM_PROG_PAGERANK, None, max_iters=20, trials=1, cache=path)
    assert len(json.load(open(path))) == 2
    open(path, "w").write("{\"x\": [1, 2]}")
    with pytest.raises(gm.GmError) as e:
        gm.autotune(gd, gm.GM_PROG_PAGERANK, None, max_iters=20, trials=1, cache=path)
    assert e.value.status == gm._lib.GM_EINVAL
    os.remove(path)
