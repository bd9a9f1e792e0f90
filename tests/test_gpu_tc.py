"""GPU triangle counting (Sec. 3 IV, Eq. (7); two-program form of Sec. 4.2) against
the oracle: exact totals and exact per-vertex counts (APPLY output)."""
import hashlib
import itertools

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_1503_07241_amd as gm
from tests import workloads as W
from tests.golden import make_tc_goldens

pytestmark = pytest.mark.gpu
DEV = "cuda"


def gpu_tc(n, s, d):
    g = gm.Graph.from_coo(n, np.asarray(s, np.int32), np.asarray(d, np.int32),
                          prep=gm.GM_PREP_UPPER_DAG, layouts=gm.GM_LAYOUT_OUT | gm.GM_LAYOUT_IN)
    counts = torch.zeros(n, dtype=torch.int64, device=DEV)
    total = gm.triangle_count(g, counts)
    return g, total, counts.cpu().numpy().view(np.uint64)


def pairs(lst):
    a = np.asarray(lst, dtype=np.int64).reshape(-1, 2)
    return a[:, 0], a[:, 1]


def test_closed_forms():
    for n in (3, 4, 7, 40):
        s, d = pairs(list(itertools.combinations(range(n), 2)))
        assert gpu_tc(n, s, d)[1] == n * (n - 1) * (n - 2) // 6
    for n in (5, 9):
        s, d = pairs([(i, (i + 1) % n) for i in range(n)])
        assert gpu_tc(n, s, d)[1] == 0
    n = 12
    s, d = pairs([(0, i) for i in range(1, n)] + [(i, i % (n - 1) + 1) for i in range(1, n)])
    assert gpu_tc(n, s, d)[1] == n - 1
    s, d = pairs([(i, j) for i in range(5) for j in range(5, 12)])
    assert gpu_tc(12, s, d)[1] == 0


@pytest.mark.parametrize("scale", [W.SMALL_SCALE, 16])
def test_rmat_total_and_per_vertex(scale):
    n, s, d = W.raw(scale)
    _, total, counts = gpu_tc(n, s, d)
    dag = W.ograph(scale, "dag")
    dag_in = oracle.dag_in_lists(dag)
    assert total == oracle.triangle_count(dag, dag_in)
    assert np.array_equal(counts, oracle.triangles_at(dag_in, np.arange(n)))
    assert int(counts.sum()) == total


def test_hub_receivers_large_lists():
    """Receivers whose in-list exceeds one wavefront's and the LDS limit:
    a dense core of 2000 vertices plus a sparse fringe."""
    rng = np.random.default_rng(7)
    core = 2000
    n = core + 30000
    s = rng.integers(0, core, 800_000)
    d = rng.integers(0, core, 800_000)
    s2 = rng.integers(0, n, 200_000)
    d2 = rng.integers(0, core, 200_000)
    s3 = rng.choice(n - 1, 17000, replace=False)  # in-list longer than the LDS stage
    d3 = np.full(17000, n - 1)
    S = np.concatenate([s, s2, np.arange(core - 1), s3])
    D = np.concatenate([d, d2, np.arange(1, core), d3])
    _, total, counts = gpu_tc(n, S, D)
    dag = oracle.prepare(n, S, D, mode="dag")
    dag_in = oracle.dag_in_lists(dag)
    assert total == oracle.triangle_count(dag, dag_in)
    assert np.array_equal(counts, oracle.triangles_at(dag_in, np.arange(n)))


def golden_check(name, total, counts):
    """Total and every receiver's count against the oracle-written golden file
    (total and SHA-256 of the whole per-vertex uint64 array)."""
    ref = make_tc_goldens.read(name)
    assert len(counts) == ref["n"]
    assert total == ref["total"]
    digest = hashlib.sha256(np.ascontiguousarray(counts, dtype="<u8").tobytes()).hexdigest()
    assert digest == ref["counts_sha256"]


def test_full_size_sampled_vertices():
    """RMAT scale 22: the exact total and every receiver's count against the
    oracle's (golden/tc_rmat22.txt), plus sampled receivers computed one by
    one by the oracle here."""
    n, s, d = W.raw(W.FULL_SCALE)
    _, total, counts = gpu_tc(n, s, d)
    assert int(counts.sum()) == total
    golden_check("tc_rmat22", total, counts)
    dag_in = oracle.dag_in_lists(W.ograph(W.FULL_SCALE, "dag"))
    indeg = np.diff(dag_in.off)
    rng = np.random.default_rng(11)
    cand = np.flatnonzero(indeg > 0)
    sample = rng.choice(cand, 300, replace=False)
    mid = np.flatnonzero((indeg > 1500) & (indeg < 2500))[:4]  # workgroup-path receivers
    verts = np.concatenate([sample, mid]).astype(np.int32)
    assert np.array_equal(counts[verts], oracle.triangles_at(dag_in, verts))


def test_run_vertex_program_tc_apply_accumulates():
    n, s, d = W.raw(10)
    g = gm.Graph.from_coo(n, s, d, prep=gm.GM_PREP_UPPER_DAG, layouts=3)
    counts = torch.full((n,), 5, dtype=torch.int64, device=DEV)
    it = gm.run_vertex_program(g, gm.GM_PROG_TC, None, 1, counts)
    assert it == 1
    ref = oracle.triangles_at(oracle.dag_in_lists(W.ograph(10, "dag")), np.arange(n))
    assert np.array_equal(counts.cpu().numpy().view(np.uint64), ref + 5)


def test_tc_needs_dag():
    n, s, d = W.raw(8)
    g = gm.Graph.from_coo(n, s, d, prep=gm.GM_PREP_DROP_SELF_LOOPS | gm.GM_PREP_SYMMETRIZE)
    with pytest.raises(gm.GmError) as e:
        gm.triangle_count(g)
    assert e.value.status == gm._lib.GM_EUNSUPPORTED


def test_edgeless_dag():
    g, total, counts = gpu_tc(9, [], [])
    assert total == 0 and not counts.any()
    tri = torch.full((9,), 3, dtype=torch.int64, device=DEV)  # APPLY adds nothing
    assert gm.run_vertex_program(g, gm.GM_PROG_TC, None, 1, tri) == 1
    assert np.array_equal(tri.cpu().numpy(), np.full(9, 3))


def test_paper_tc_workload_rmat20_a45():
    """The paper's triangle-counting graph (Sec. 5.1, Table 1): RMAT scale 20
    with a = .45, b = c = .15; exact total and every receiver's count against
    the oracle (golden/tc_rmat20_a45.txt), sampled receivers recomputed here."""
    n, s, d = gg.rmat(20, a=0.45, b=0.15, c=0.15)
    g, total, counts = gpu_tc(n, s, d)
    assert g.m == make_tc_goldens.read("tc_rmat20_a45")["m_dag"]
    golden_check("tc_rmat20_a45", total, counts)
    dag_in = oracle.dag_in_lists(oracle.prepare(n, s, d, mode="dag"))
    verts = np.random.default_rng(45).choice(n, 200, replace=False).astype(np.int32)
    assert np.array_equal(counts[verts], oracle.triangles_at(dag_in, verts))


@pytest.mark.parametrize("tuning", [
    {"tc_wave_max": 64},                                   # per-wavefront tables up to 64 keys only
    {"tc_wave_max": 128, "tc_wave_work": 256},             # class 0 only, tiny wavefront items
    {"tc_wave_max": 300, "tc_block_work": 4096},           # class 1 boundary off a power of two
    {"tc_wave_max": 512, "tc_wave_work": 1 << 20, "tc_block_work": 256},
])
def test_tuning_keeps_counts_exact(tuning):
    """Table classes, work-item sizes and the split into pieces move with the
    tuning; the total and every receiver's count stay exact (Eq. (7))."""
    n, s, d = W.raw(16)
    g = gm.Graph.from_coo(n, s, d, prep=gm.GM_PREP_UPPER_DAG,
                          layouts=gm.GM_LAYOUT_OUT | gm.GM_LAYOUT_IN)
    g.set_tuning(**tuning)
    counts = torch.zeros(n, dtype=torch.int64, device=DEV)
    total = gm.triangle_count(g, counts)
    dag_in = oracle.dag_in_lists(W.ograph(16, "dag"))
    assert total == oracle.triangle_count(W.ograph(16, "dag"), dag_in)
    assert np.array_equal(counts.cpu().numpy().view(np.uint64),
                          oracle.triangles_at(dag_in, np.arange(n)))
