"""Pins of the oracle's triangle count (Sec. 3 IV, Eq. (7); two-program form of
Sec. 4.2) and collaborative-filtering loss/gradients (Sec. 3 III, Eqs. (3)-(6)).
"""
import itertools
import os

import networkx as nx
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def dag_of(n, pairs):
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    return oracle.prepare(n, pairs[:, 0], pairs[:, 1], mode="dag")


def brute_triangles(n, pairs):
    """Eq. (7) written out: count u < v < w with all three edges present."""
    E = set()
    for a, b in pairs:
        if a != b:
            E.add((min(a, b), max(a, b)))
    return sum(1 for u, v, w in itertools.combinations(range(n), 3)
               if (u, v) in E and (v, w) in E and (u, w) in E)


def test_tc_closed_forms():
    for n in (3, 4, 5, 8):
        assert oracle.triangle_count(dag_of(n, list(itertools.combinations(range(n), 2)))) == \
            n * (n - 1) * (n - 2) // 6
    for n in (4, 5, 9):
        assert oracle.triangle_count(dag_of(n, [(i, (i + 1) % n) for i in range(n)])) == 0
    for n in (5, 6, 10):  # wheel: hub 0 + cycle over 1..n-1
        rim = [(i, i % (n - 1) + 1) for i in range(1, n)]
        assert oracle.triangle_count(dag_of(n, [(0, i) for i in range(1, n)] + rim)) == n - 1
    k4 = [p for p in itertools.combinations(range(4), 2) if p != (0, 1)]
    assert oracle.triangle_count(dag_of(4, k4)) == 2
    bip = [(i, j) for i in range(4) for j in range(4, 9)]
    assert oracle.triangle_count(dag_of(9, bip)) == 0


@pytest.mark.parametrize("seed", range(5))
def test_tc_brute_force_trace_networkx(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 40))
    m = int(rng.integers(0, 5 * n))
    s, d = rng.integers(0, n, m), rng.integers(0, n, m)
    dag = oracle.prepare(n, s, d, mode="dag")
    got = oracle.triangle_count(dag)
    assert got == brute_triangles(n, zip(s.tolist(), d.tolist()))
    A = np.zeros((n, n), dtype=np.int64)
    sym = oracle.prepare(n, s, d, mode="symmetric")
    A[sym.rows(), sym.idx] = 1
    assert got == np.trace(A @ A @ A) // 6
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from(zip(sym.rows().tolist(), sym.idx.tolist()))
    assert got == sum(nx.triangles(G).values()) // 3
    per = oracle.triangles_at(oracle.dag_in_lists(dag), np.arange(n))
    assert int(per.sum()) == got


def test_tc_rmat10_networkx():
    n, s, d = gg.rmat(10)
    dag = oracle.prepare(n, s, d, mode="dag")
    sym = oracle.prepare(n, s, d, mode="symmetric")
    G = nx.Graph()
    G.add_edges_from(zip(sym.rows().tolist(), sym.idx.tolist()))
    assert oracle.triangle_count(dag) == sum(nx.triangles(G).values()) // 3


def test_tc_per_vertex_is_max_corner_count():
    """count(v) = #triangles whose largest vertex is v (each counted at (mid, max))."""
    n, s, d = gg.rmat(7)
    dag = oracle.prepare(n, s, d, mode="dag")
    per = oracle.triangles_at(oracle.dag_in_lists(dag), np.arange(n))
    sym = oracle.prepare(n, s, d, mode="symmetric")
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from(zip(sym.rows().tolist(), sym.idx.tolist()))
    want = np.zeros(n, dtype=np.int64)
    for tri in nx.enumerate_all_cliques(G):
        if len(tri) == 3:
            want[max(tri)] += 1
        elif len(tri) > 3:
            break
    assert np.array_equal(per.astype(np.int64), want)


# --- collaborative filtering -------------------------------------------------
def read_golden(name):
    kv = {}
    for line in open(os.path.join(HERE, "golden", name)):
        if line.startswith("#") or not line.strip() or line.startswith("key"):
            continue
        k, v = line.split()
        kv[k] = float(v)
    return kv


def test_cf_hand_example_golden():
    kv = read_golden("cf_hand_example.txt")
    L, gU, gV = oracle.cf_loss_grad(
        1, 1, np.array([0]), np.array([0]), np.array([int(kv["G"])]),
        np.array([[kv["p_u"]]], dtype=np.float32), np.array([[kv["p_v"]]], dtype=np.float32),
        kv["lambda"])
    assert abs(L - kv["L"]) < 1e-12
    assert abs(gU[0, 0] - kv["g_u"]) < 1e-12 and abs(gV[0, 0] - kv["g_v"]) < 1e-12


def small_ratings(seed=0):
    R = gg.cf_ratings(n_users=300, n_items=40, total=3000, dmin=3)
    rng = np.random.default_rng(seed)
    PU = rng.normal(0, 0.4, (R.n_users, 8)).astype(np.float32)
    PV = rng.normal(0, 0.4, (R.n_items, 8)).astype(np.float32)
    return R, PU, PV


def test_cf_zero_factors():
    R, PU, PV = small_ratings()
    L, gU, gV = oracle.cf_loss_grad(R.n_users, R.n_items, R.user, R.item, R.rating,
                                    np.zeros_like(PU), np.zeros_like(PV), 0.05)
    assert L == float((R.rating.astype(np.int64) ** 2).sum())
    assert not gU.any() and not gV.any()


def test_cf_vs_torch_autograd_and_fd():
    R, PU, PV = small_ratings(1)
    lam = 0.05
    L, gU, gV = oracle.cf_loss_grad(R.n_users, R.n_items, R.user, R.item, R.rating, PU, PV, lam)
    pu = torch.tensor(PU, dtype=torch.float64, requires_grad=True)
    pv = torch.tensor(PV, dtype=torch.float64, requires_grad=True)
    u = torch.tensor(R.user.astype(np.int64))
    v = torch.tensor(R.item.astype(np.int64))
    e = torch.tensor(R.rating, dtype=torch.float64) - (pu[u] * pv[v]).sum(1)
    Lt = (e * e).sum() + lam * (pu * pu).sum() + lam * (pv * pv).sum()
    Lt.backward()
    assert abs(L - Lt.item()) <= 1e-12 * abs(L)
    assert np.allclose(gU, pu.grad.numpy(), rtol=1e-10, atol=1e-12)
    assert np.allclose(gV, pv.grad.numpy(), rtol=1e-10, atol=1e-12)
    # central difference along a random direction (float32 factors: step in
    # the float32 grid is exact, so use the float64 torch loss for the values)
    rng = np.random.default_rng(2)
    du, dv = rng.normal(size=PU.shape), rng.normal(size=PV.shape)
    h = 1e-6

    def loss_at(a, b):
        e = torch.tensor(R.rating, dtype=torch.float64) - (a[u] * b[v]).sum(1)
        return ((e * e).sum() + lam * (a * a).sum() + lam * (b * b).sum()).item()

    p0u, p0v = torch.tensor(PU, dtype=torch.float64), torch.tensor(PV, dtype=torch.float64)
    fd = (loss_at(p0u + h * torch.tensor(du), p0v + h * torch.tensor(dv))
          - loss_at(p0u - h * torch.tensor(du), p0v - h * torch.tensor(dv))) / (2 * h)
    assert abs(fd - ((gU * du).sum() + (gV * dv).sum())) <= 1e-6 * abs(fd)


def test_cf_gradient_matches_gd_update():
    """Eqs. (5)-(6): p* = p + gamma (sum e p' - lambda p) = p - (gamma/2) dL/dp."""
    R, PU, PV = small_ratings(3)
    lam, gamma = 0.05, 0.01
    _, gU, gV = oracle.cf_loss_grad(R.n_users, R.n_items, R.user, R.item, R.rating, PU, PV, lam)
    PU64, PV64 = PU.astype(np.float64), PV.astype(np.float64)
    e = R.rating - (PU64[R.user] * PV64[R.item]).sum(1)
    su = np.zeros_like(PU64)
    sv = np.zeros_like(PV64)
    np.add.at(su, R.user, e[:, None] * PV64[R.item])
    np.add.at(sv, R.item, e[:, None] * PU64[R.user])
    assert np.allclose(PU64 + gamma * (su - lam * PU64), PU64 - gamma / 2 * gU, rtol=1e-12)
    assert np.allclose(PV64 + gamma * (sv - lam * PV64), PV64 - gamma / 2 * gV, rtol=1e-12)


def test_cf_without_ratings_is_the_l2_term():
    # Eq. (3) with no rating: loss = lambda (|P_U|^2 + |P_V|^2), gradients 2 lambda P
    rng = np.random.default_rng(4)
    PU = rng.normal(size=(3, 5)).astype(np.float32)
    PV = rng.normal(size=(2, 5)).astype(np.float32)
    none = np.zeros(0, np.int32)
    L, gU, gV = oracle.cf_loss_grad(3, 2, none, none, np.zeros(0, np.uint8), PU, PV, 0.05)
    l2 = float((PU.astype(np.float64) ** 2).sum() + (PV.astype(np.float64) ** 2).sum())
    assert L == pytest.approx(0.05 * l2, rel=1e-12)
    assert np.allclose(gU, 0.1 * PU.astype(np.float64), rtol=1e-12, atol=0)
    assert np.allclose(gV, 0.1 * PV.astype(np.float64), rtol=1e-12, atol=0)


def test_cf_gd_hand_worked_and_against_one_pass_gradients():
    """The oracle's GD loop (Eqs. (5)-(6)) on the hand-worked 1 x 1 example of
    golden/cf_gd_hand.txt (two steps), and each step's gradients against the
    C oracle's one-pass gradients at the same (float32-representable) point."""
    import os
    kv = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "cf_gd_hand.txt")):
        if line.startswith("#") or not line.strip() or line.startswith("key"):
            continue
        k, v = line.split()
        kv[k] = float(v)
    P = np.array([[kv["p0"]]])
    pu, pv, L = oracle.cf_gd(1, 1, [0], [0], [int(kv["G"])], P, P, kv["lambda"], kv["gamma"], 2)
    assert abs(L[0] - kv["L0"]) < 1e-12 and abs(L[1] - kv["L1"]) < 1e-12
    assert abs(pu[0, 0] - kv["p2"]) < 1e-12 and abs(pv[0, 0] - kv["p2"]) < 1e-12
    pu1, _, _ = oracle.cf_gd(1, 1, [0], [0], [int(kv["G"])], P, P, kv["lambda"], kv["gamma"], 1)
    assert abs(pu1[0, 0] - kv["p1"]) < 1e-12
    R = gg.cf_ratings(n_users=300, n_items=40, total=6000, dmin=5)
    PU, PV = gg.cf_point(300, 40, 8)
    L0, gu, gv = oracle.cf_loss_grad(300, 40, R.user, R.item, R.rating, PU, PV, 0.05)
    L64, gu64, gv64 = oracle._cf_loss_grad64(300, 40, R.user, R.item, R.rating,
                                             PU.astype(np.float64), PV.astype(np.float64), 0.05)
    assert abs(L0 - L64) <= 1e-12 * L0
    assert np.allclose(gu, gu64, rtol=1e-12, atol=1e-12)
    assert np.allclose(gv, gv64, rtol=1e-12, atol=1e-12)
