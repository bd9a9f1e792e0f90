"""Error paths on the GPU: an allocation that fails inside a call reports
GM_ENOMEM and leaves the graph intact, so the same call succeeds afterwards
with results equal to the oracle's. Failures are injected through the
library's GM_FAULT_ALLOC hook (the k-th device allocation after the
variable is set fails), which is read at every allocation."""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1503_07241_amd as gm
from tests import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda"


class fault_at:
    def __init__(self, k):
        self.k = k

    def __enter__(self):
        os.environ["GM_FAULT_ALLOC"] = str(self.k)

    def __exit__(self, *exc):
        os.environ.pop("GM_FAULT_ALLOC", None)


@pytest.mark.parametrize("k", [1, 2, 5])
def test_enomem_in_pagerank_layout_leaves_graph_intact(k):
    scale = 10
    n, s, d = W.raw(scale)
    g = gm.Graph.from_coo(n, s, d)
    rank = torch.ones(n, dtype=torch.float32, device=DEV)
    with fault_at(k):
        with pytest.raises(gm.GmError) as e:
            gm.run_vertex_program(g, gm.GM_PROG_PAGERANK, None, 20, rank)
    assert e.value.status == gm._lib.GM_ENOMEM
    rank.fill_(1.0)
    gm.run_vertex_program(g, gm.GM_PROG_PAGERANK, None, 20, rank)
    ref = oracle.pagerank(W.ograph(scale, "directed"), 0.15, 20)
    assert W.max_rel_err(rank.cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("k", [1, 4, 9])
def test_enomem_in_triangle_plan_leaves_graph_intact(k):
    scale = 10
    n, s, d = W.raw(scale)
    g = gm.Graph.from_coo(n, s, d, prep=gm.GM_PREP_UPPER_DAG)
    counts = torch.zeros(n, dtype=torch.int64, device=DEV)
    with fault_at(k):
        with pytest.raises(gm.GmError) as e:
            gm.triangle_count(g, counts)
    assert e.value.status == gm._lib.GM_ENOMEM
    counts.zero_()
    total = gm.triangle_count(g, counts)
    dag_in = oracle.dag_in_lists(W.ograph(scale, "dag"))
    assert total == oracle.triangle_count(W.ograph(scale, "dag"), dag_in)
    assert np.array_equal(counts.cpu().numpy().view(np.uint64),
                          oracle.triangles_at(dag_in, np.arange(n)))


def test_enomem_in_graph_load_and_frontier_workspace():
    scale = 10
    n, s, d = W.raw(scale)
    with fault_at(2):
        with pytest.raises(gm.GmError) as e:
            gm.Graph.from_coo(n, s, d, prep=gm.GM_PREP_DROP_SELF_LOOPS | gm.GM_PREP_SYMMETRIZE)
    assert e.value.status == gm._lib.GM_ENOMEM
    g = gm.Graph.from_coo(n, s, d, prep=gm.GM_PREP_DROP_SELF_LOOPS | gm.GM_PREP_SYMMETRIZE)
    lv = torch.full((n,), gm.INF_LEVEL, dtype=torch.int32, device=DEV)
    lv[0] = 0
    root = torch.zeros(1, dtype=torch.int32, device=DEV)
    with fault_at(1):
        with pytest.raises(gm.GmError) as e:
            gm.run_vertex_program(g, gm.GM_PROG_BFS, root, -1, lv)
    assert e.value.status == gm._lib.GM_ENOMEM
    lv.fill_(gm.INF_LEVEL)
    lv[0] = 0
    gm.run_vertex_program(g, gm.GM_PROG_BFS, root, -1, lv)
    assert np.array_equal(lv.cpu().numpy(), W.bfs_levels(scale))
