"""The ablation variants of the paper's design choices (Sec. 5.4, Fig. 7),
selected through gm_tuning.variant and the direction/LDS parameters: each
must leave every result unchanged. BFS and SSSP bit-exact against the
oracle, PageRank within 1e-5, at RMAT scale 14 and (BFS, SSSP) scale 22."""
import numpy as np
import pytest
import torch

import oracle
import paper_1503_07241_amd as gm
from tests import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda"
P_DIR = gm.GM_PREP_DROP_SELF_LOOPS
P_SYM = gm.GM_PREP_DROP_SELF_LOOPS | gm.GM_PREP_SYMMETRIZE
LIST, VPUSH, ROWPULL, DEG = (gm._lib.GM_VARIANT_LIST_FRONTIER, gm._lib.GM_VARIANT_VERTEX_PUSH,
                              gm._lib.GM_VARIANT_ROW_PULL, gm._lib.GM_VARIANT_DEGREE_ORDER)
VARIANTS = [0, LIST, VPUSH, LIST | VPUSH, DEG, DEG | LIST, DEG | VPUSH]


def ids(*v):
    return torch.tensor(list(v), dtype=torch.int32, device=DEV)


@pytest.mark.parametrize("scale", [W.SMALL_SCALE, W.FULL_SCALE])
@pytest.mark.parametrize("variant", VARIANTS)
def test_min_program_variants(scale, variant):
    n, s, d = W.raw(scale)
    gs = gm.Graph.from_coo(n, s, d, prep=P_SYM)
    gd = gm.Graph.from_coo(n, s, d, w=W.weights(scale), prep=P_DIR)
    ref_lv, ref_d = W.bfs_levels(scale), W.sssp_dist(scale)
    for pull_div in (128, 1):  # with pull supersteps for large frontiers, and push only
        gs.set_tuning(variant=variant, pull_div=pull_div)
        lv = torch.full((n,), gm.INF_LEVEL, dtype=torch.int32, device=DEV)
        lv[0] = 0
        it = gm.run_vertex_program(gs, gm.GM_PROG_BFS, ids(0), -1, lv)
        assert np.array_equal(lv.cpu().numpy(), ref_lv)
        assert it == int(ref_lv[ref_lv != oracle.INF_I32].max()) + 1
    for pull_div in (128, 1, 65536):  # pull supersteps for frontiers with many edges,
        gd.set_tuning(variant=variant, pull_div=pull_div)  # push only, pull almost always
        dist = torch.full((n,), -1, dtype=torch.int32, device=DEV)
        dist[0] = 0
        it = gm.run_vertex_program(gd, gm.GM_PROG_SSSP, ids(0), -1, dist)
        assert np.array_equal(dist.cpu().numpy().view(np.uint32), ref_d)
        assert it == W.sssp_supersteps(scale)


@pytest.mark.parametrize("pull_div", [128, 65536])
@pytest.mark.parametrize("variant", VARIANTS)
def test_min_program_variants_resume_and_hand_trace(variant, pull_div):
    n, s, d, w, src, trace, steps = W.sssp_hand_trace()
    g = gm.Graph.from_coo(n, s, d, w=w, prep=P_DIR)
    g.set_tuning(variant=variant, pull_div=pull_div)
    for k, (dist_k, act_k) in enumerate(trace, start=1):
        dist = torch.full((n,), -1, dtype=torch.int32, device=DEV)
        dist[src] = 0
        act = torch.zeros(n, dtype=torch.int32, device=DEV)
        assert gm.run_vertex_program(g, gm.GM_PROG_SSSP, ids(src), k, dist, act) == k
        assert np.array_equal(dist.cpu().numpy().view(np.uint32), dist_k)
        assert np.array_equal(act.cpu().numpy().astype(bool), act_k)


@pytest.mark.parametrize("hot", [0, 40960])
def test_pagerank_row_pull_and_lds_variants(hot):
    scale = W.SMALL_SCALE
    n, s, d = W.raw(scale)
    g = gm.Graph.from_coo(n, s, d)
    for variant in (0, ROWPULL):
        g.set_tuning(variant=variant, pr_hot=hot)
        pr = torch.ones(n, dtype=torch.float32, device=DEV)
        gm.run_vertex_program(g, gm.GM_PROG_PAGERANK, None, 20, pr)
        assert W.max_rel_err(pr.cpu().numpy(), W.pagerank(scale)) <= 1e-5
        ppr = torch.zeros(n, dtype=torch.float32, device=DEV)
        ppr[3] = 1.0
        gm.run_vertex_program(g, gm.GM_PROG_PPR, ids(3), 20, ppr)
        ref = oracle.personalized_pagerank(W.ograph(scale, "directed"), 3, 0.15, 20)
        got = ppr.cpu().numpy()
        assert np.abs(got - ref).sum() / np.abs(ref).sum() <= 1e-5
