"""Adjoint (transpose-direction) products on the GPU against the FP64 oracle:
collaborative-filtering loss and factor gradients (Sec. 3 III, Eqs. (3)-(6))
and the edge-weight gradient of PageRank (Eq. (1) with weights).

Tolerances: loss relative error <= 1e-5; gradients ||g - g_ref|| / ||g_ref||
<= 1e-5 (Frobenius / 2-norm)."""
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
HERE = os.path.dirname(os.path.abspath(__file__))
LAM = 0.05


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cf_setup(n_users, n_items, total, K=32, seed=gg.SEED_CF_POINT, dmin=gg.CF_DMIN):
    R = gg.cf_ratings(n_users=n_users, n_items=n_items, total=total, dmin=dmin)
    PU, PV = gg.cf_point(R.n_users, R.n_items, K, seed)
    g = gm.RatingGraph.from_coo(R.n_users, R.n_items, R.user, R.item, R.rating)
    return R, PU, PV, g


def gpu_cf(g, PU, PV, lam=LAM, scale=1.0):
    pu = torch.tensor(PU, device=DEV)
    pv = torch.tensor(PV, device=DEV)
    loss = torch.empty(1, dtype=torch.float64, device=DEV)
    gm.cf_forward(g, pu, pv, lam, loss)
    gu, gv = torch.empty_like(pu), torch.empty_like(pv)
    gm.cf_backward(g, pu, pv, lam, scale, gu, gv)
    return float(loss.item()), gu.cpu().numpy(), gv.cpu().numpy()


def test_cf_hand_example():
    kv = {}
    for line in open(os.path.join(HERE, "golden", "cf_hand_example.txt")):
        if line.startswith("#") or not line.strip() or line.startswith("key"):
            continue
        k, v = line.split()
        kv[k] = float(v)
    g = gm.RatingGraph.from_coo(1, 1, [0], [0], [int(kv["G"])])
    L, gu, gv = gpu_cf(g, np.array([[kv["p_u"]]], np.float32), np.array([[kv["p_v"]]], np.float32),
                       kv["lambda"])
    # lambda crosses the ABI as float32 (0.05f = 0.05 + 7.5e-10), hence 1e-7
    assert abs(L - kv["L"]) < 1e-7
    assert abs(gu[0, 0] - kv["g_u"]) < 1e-6 and abs(gv[0, 0] - kv["g_v"]) < 1e-6


@pytest.mark.parametrize("shape,K", [((3000, 500, 120_000), 32), ((3000, 3000, 600_000), 32),
                                     ((2000, 20, 30_000), 16), ((500, 400, 20_000), 7)])
def test_cf_loss_and_gradients(shape, K):
    """Includes long rows and columns (more than one work item) and K not a
    power of two."""
    nu, ni, tot = shape
    R, PU, PV, g = cf_setup(nu, ni, tot, K, dmin=min(gg.CF_DMIN, ni))
    L, gu, gv = gpu_cf(g, PU, PV)
    Lr, gur, gvr = oracle.cf_loss_grad(R.n_users, R.n_items, R.user, R.item, R.rating, PU, PV, LAM)
    assert abs(L - Lr) <= 1e-5 * abs(Lr)
    assert rel(gu, gur) <= 1e-5 and rel(gv, gvr) <= 1e-5


def test_cf_full_size():
    """The 480,189 x 17,770 rating graph with 100M ratings, K = 32."""
    R, PU, PV, g = cf_setup(gg.NETFLIX_USERS, gg.NETFLIX_ITEMS, gg.NETFLIX_RATINGS)
    L, gu, gv = gpu_cf(g, PU, PV)
    Lr, gur, gvr = oracle.cf_loss_grad(R.n_users, R.n_items, R.user, R.item, R.rating, PU, PV, LAM)
    assert abs(L - Lr) <= 1e-5 * abs(Lr)
    assert rel(gu, gur) <= 1e-5 and rel(gv, gvr) <= 1e-5
    # per-row maxima, reported for information
    print("cf full: loss rel %.2e, gU rel %.2e, gV rel %.2e" % (
        abs(L - Lr) / Lr, rel(gu, gur), rel(gv, gvr)))


def test_cf_autograd_and_finite_difference():
    R, PU, PV, g = cf_setup(2000, 300, 60_000)
    pu = torch.tensor(PU, device=DEV, requires_grad=True)
    pv = torch.tensor(PV, device=DEV, requires_grad=True)
    loss = gm.CFLoss.apply(pu, pv, g, LAM)
    (3.0 * loss).backward()
    Lr, gur, gvr = oracle.cf_loss_grad(R.n_users, R.n_items, R.user, R.item, R.rating, PU, PV, LAM)
    assert rel(pu.grad.cpu().numpy(), 3.0 * gur) <= 1e-5
    assert rel(pv.grad.cpu().numpy(), 3.0 * gvr) <= 1e-5
    # central difference of the GPU loss along a random direction; the
    # direction is taken from the float32-rounded perturbed points
    rng = np.random.default_rng(3)
    du, dv = rng.normal(size=PU.shape), rng.normal(size=PV.shape)
    h = 1e-3
    Up, Um = (PU + h * du).astype(np.float32), (PU - h * du).astype(np.float32)
    Vp, Vm = (PV + h * dv).astype(np.float32), (PV - h * dv).astype(np.float32)
    Lp = gpu_cf(g, Up, Vp)[0]
    Lm = gpu_cf(g, Um, Vm)[0]
    fd = (Lp - Lm) / (2 * h)
    du_eff = (Up.astype(np.float64) - Um) / (2 * h)
    dv_eff = (Vp.astype(np.float64) - Vm) / (2 * h)
    _, gu0, gv0 = oracle.cf_loss_grad(R.n_users, R.n_items, R.user, R.item, R.rating,
                                      (Up.astype(np.float64) + Um) / 2, (Vp.astype(np.float64) + Vm) / 2,
                                      LAM)
    ana = (gu0 * du_eff).sum() + (gv0 * dv_eff).sum()
    assert abs(fd - ana) <= 1e-5 * abs(ana)


def test_cf_rejects_plain_graph_and_bad_k():
    n, s, d = W.raw(8)
    g = gm.Graph.from_coo(n, s, d)
    x = torch.zeros((n, 4), device=DEV)
    loss = torch.empty(1, dtype=torch.float64, device=DEV)
    with pytest.raises(gm.GmError) as e:
        gm.cf_forward(g, x, x, LAM, loss)
    assert e.value.status == gm._lib.GM_EUNSUPPORTED
    R, PU, PV, rg = cf_setup(200, 50, 3000)
    big = torch.zeros((200, 65), device=DEV)
    with pytest.raises(gm.GmError) as e:
        gm.cf_forward(rg, big, torch.zeros((50, 65), device=DEV), LAM, loss)
    assert e.value.status == gm._lib.GM_EINVAL


# --- PageRank edge-weight gradient ------------------------------------------
def pr_setup(n, s, d, seed=11):
    og = oracle.prepare(n, s, d)
    w = gg.weights_f32(og.rows().astype(np.int32), og.idx, seed, 0.5, 1.5)
    c = gg.uniform_f32(n, gg.SEED_PR_UPSTREAM)
    g = gm.Graph.from_coo(n, s, d)
    return og, w, c, g


def gpu_pr_grad(g, n, w, c, T, r=0.15):
    wt = torch.tensor(w, device=DEV)
    hist = torch.empty((T + 1, n), dtype=torch.float32, device=DEV)
    hist[0].fill_(1.0)
    gm.pagerank_forward_w(g, wt, r, T, hist)
    gw = torch.empty_like(wt)
    gm.pagerank_vjp_w(g, wt, r, T, hist, torch.tensor(c, device=DEV), gw)
    return hist.cpu().numpy(), gw.cpu().numpy()


@pytest.mark.parametrize("scale,T", [(12, 20), (W.SMALL_SCALE, 20), (10, 1), (W.SMALL_SCALE, 3),
                                     (W.FULL_SCALE, 20)])
def test_pagerank_weight_gradient(scale, T):
    """Every edge's gradient against the FP64 oracle (2-norm relative <= 1e-5),
    up to the full-size scale-22 graph (65.2M edges) at T = 20."""
    n, s, d = W.raw(scale)
    og, w, c, g = pr_setup(n, s, d)
    hist, gw = gpu_pr_grad(g, n, w, c, T)
    ref_hist = oracle.pagerank_history(og, 0.15, T, w=w.astype(np.float64))
    assert W.max_rel_err(hist[T], ref_hist[T]) <= 1e-5
    ref = oracle.pagerank_vjp_w(og, w, c, 0.15, T, hist=ref_hist)
    assert rel(gw, ref) <= 1e-5
    if T == 1:  # closed form: 0.85 * c_v / outdeg(u)
        deg = og.degree()[og.rows()]
        assert rel(gw, 0.85 * c[og.idx].astype(np.float64) / deg) <= 1e-6


def test_pagerank_weight_gradient_long_rows():
    """Out-degree and in-degree far above one work item (split rows)."""
    hub = 0
    n = 12000
    s = np.concatenate([np.zeros(n - 1), np.arange(1, n), np.arange(1, n - 1)]).astype(np.int32)
    d = np.concatenate([np.arange(1, n), np.zeros(n - 1), np.arange(2, n)]).astype(np.int32)
    og, w, c, g = pr_setup(n, s, d)
    hist, gw = gpu_pr_grad(g, n, w, c, 20)
    ref_hist = oracle.pagerank_history(og, 0.15, 20, w=w.astype(np.float64))
    assert W.max_rel_err(hist[20], ref_hist[20]) <= 1e-5
    assert rel(gw, oracle.pagerank_vjp_w(og, w, c, 0.15, 20, hist=ref_hist)) <= 1e-5


# Out-degree multisets for the reverse pass's edge tiles (its rows are the
# sources, relabelled by decreasing out-degree): row ends on, just before and
# just after 1024-edge tile boundaries, rows spanning several tiles, a last
# tile filled exactly and one left ragged.
OUT_TILE_CASES = [
    [3072, 1024, 1000, 24] + [1] * 1024,
    [2049, 1023, 1, 1],
    [1025] + [2] * 600 + [1] * 5,
    [700, 324] + [3] * 341 + [1],
]


@pytest.mark.parametrize("case", range(len(OUT_TILE_CASES)))
def test_pagerank_weight_gradient_tile_boundaries(case):
    rng = np.random.default_rng(200 + case)
    degrees = OUT_TILE_CASES[case]
    n = len(degrees) + 3000
    src, dst = [], []
    for u, k in enumerate(degrees):
        cand = rng.choice(n - 1, size=k, replace=False)
        dst.append(np.where(cand >= u, cand + 1, cand))
        src.append(np.full(k, u))
    s = np.concatenate(src).astype(np.int32)
    d = np.concatenate(dst).astype(np.int32)
    og, w, c, g = pr_setup(n, s, d)
    for T in (1, 20):
        hist, gw = gpu_pr_grad(g, n, w, c, T)
        ref_hist = oracle.pagerank_history(og, 0.15, T, w=w.astype(np.float64))
        assert rel(gw, oracle.pagerank_vjp_w(og, w, c, 0.15, T, hist=ref_hist)) <= 1e-5


def test_pagerank_weight_gradient_autograd_fd():
    n, s, d = W.raw(10)
    og, w, c, g = pr_setup(n, s, d)
    wt = torch.tensor(w, device=DEV, requires_grad=True)
    out = gm.PageRankW.apply(wt, g, 0.15, 20)
    (out * torch.tensor(c, device=DEV)).sum().backward()
    ref = oracle.pagerank_vjp_w(og, w, c, 0.15, 20)
    assert rel(wt.grad.cpu().numpy(), ref) <= 1e-5
    # FP64 central difference of the oracle along a random direction
    rng = np.random.default_rng(5)
    dirv = rng.normal(size=og.m)
    h = 1e-6
    Lp = c @ oracle.pagerank(og, 0.15, 20, w=w + h * dirv)
    Lm = c @ oracle.pagerank(og, 0.15, 20, w=w - h * dirv)
    fd = (Lp - Lm) / (2 * h)
    assert abs(wt.grad.cpu().numpy().astype(np.float64) @ dirv - fd) <= 1e-5 * abs(fd)


def test_cf_unrated_rows_columns_and_no_ratings():
    """Users 1 and 3 and item 2 have no rating: their gradient rows are the
    L2 term of Eq. (3) alone; a rating graph without ratings leaves only it."""
    user = np.array([0, 0, 2, 4], np.int32)
    item = np.array([0, 1, 3, 1], np.int32)
    rating = np.array([5, 3, 1, 4], np.uint8)
    rng = np.random.default_rng(11)
    PU = (0.3 * rng.normal(size=(5, 8))).astype(np.float32)
    PV = (0.3 * rng.normal(size=(4, 8))).astype(np.float32)
    for nu, ni, u, i, v in ((5, 4, user, item, rating),
                            (5, 4, user[:0], item[:0], rating[:0])):
        g = gm.RatingGraph.from_coo(nu, ni, u, i, v)
        L, gu, gv = gpu_cf(g, PU, PV)
        Lr, gur, gvr = oracle.cf_loss_grad(nu, ni, u, i, v, PU, PV, LAM)
        assert abs(L - Lr) <= 1e-5 * abs(Lr)
        assert rel(gu, gur) <= 1e-5 and rel(gv, gvr) <= 1e-5
        assert np.allclose(gu[[1, 3]], 2 * LAM * PU[[1, 3]], rtol=1e-6, atol=0)
        assert np.allclose(gv[2], 2 * LAM * PV[2], rtol=1e-6, atol=0)


def test_pagerank_weight_gradient_edgeless_graph():
    n = 40
    none = np.zeros(0, np.int32)
    g = gm.Graph.from_coo(n, none, none)
    wt = torch.zeros(0, device=DEV, requires_grad=True)  # its address is NULL
    out = gm.PageRankW.apply(wt, g, 0.15, 3)
    ref = oracle.pagerank(oracle.prepare(n, none, none), 0.15, 3, w=np.zeros(0))
    assert np.allclose(out.detach().cpu().numpy(), ref, rtol=1e-6, atol=0)
    out.sum().backward()
    assert wt.grad.shape == (0,)


def test_cf_gradient_descent_hand_and_oracle():
    """gm_cf_gd (Eqs. (5)-(6)): the hand-worked two steps of
    golden/cf_gd_hand.txt, and five steps on a 2,000 x 300 rating graph
    against the oracle's float64 descent (losses relative <= 1e-5, factors
    Frobenius relative <= 1e-5)."""
    kv = {}
    for line in open(os.path.join(HERE, "golden", "cf_gd_hand.txt")):
        if line.startswith("#") or not line.strip() or line.startswith("key"):
            continue
        k, v = line.split()
        kv[k] = float(v)
    g = gm.RatingGraph.from_coo(1, 1, [0], [0], [int(kv["G"])])
    pu = torch.full((1, 1), kv["p0"], dtype=torch.float32, device=DEV)
    pv = pu.clone()
    hist = torch.empty(3, dtype=torch.float64, device=DEV)
    gm.cf_gd(g, pu, pv, kv["lambda"], kv["gamma"], 2, hist)
    assert abs(float(pu.item()) - kv["p2"]) < 1e-6 and abs(float(pv.item()) - kv["p2"]) < 1e-6
    assert abs(float(hist[0]) - kv["L0"]) < 1e-6 and abs(float(hist[1]) - kv["L1"]) < 1e-5
    R, PU, PV, rg = cf_setup(2000, 300, 60_000)
    pu, pv = torch.tensor(PU, device=DEV), torch.tensor(PV, device=DEV)
    hist = torch.empty(6, dtype=torch.float64, device=DEV)
    gm.cf_gd(rg, pu, pv, LAM, 0.002, 5, hist)
    rpu, rpv, rL = oracle.cf_gd(R.n_users, R.n_items, R.user, R.item, R.rating, PU, PV, LAM,
                                0.002, 5)
    assert np.max(np.abs(hist.cpu().numpy() - rL) / rL) <= 1e-5
    assert rL[-1] < rL[0]  # descent
    assert rel(pu.cpu().numpy(), rpu) <= 1e-5 and rel(pv.cpu().numpy(), rpv) <= 1e-5
