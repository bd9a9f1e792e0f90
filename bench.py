"""Benchmark of the generalized-SpMSpV hot path on one MI355X.

One step = one pass of every program of the full-size single-source workload
on RMAT scale 22 (4,194,304 vertices, edge factor 16, a/b/c = .57/.19/.19,
self-loops and duplicates removed):
  BFS from vertex 0 on the symmetrised graph (int32 levels),
  SSSP from vertex 0 on the directed graph, uint32 weights in [1, 255],
  PageRank, 20 supersteps, FP32 (r = 0.15),
  triangle counting on the upper-triangle DAG of the symmetrised graph (uint64).
Each program's property array is re-initialised inside the step.

value = edges traversed by the step / step time, in GTEPS, where "edges
traversed" counts, per superstep, the out-edges of every vertex that sent a
message (Alg. 1's column walk): BFS and SSSP report it from the library's
counters, PageRank traverses all m edges per superstep, triangle counting
sends one message along each of the m_dag DAG edges.

After the timed steps (and outside them) the batched and adjoint forms are
measured against the plain runs they replace, on the same GPU, together
with the paper's own triangle-counting and SSSP graphs (RMAT scale 20 with
a = .45 and RMAT scale 24 with a = .50, Table 1) and a 2048 x 2048 grid:
  RMAT scale 20: 64-source BFS and SSSP, 128-seed personalised PageRank
  (20 supersteps) against 64 / 128 plain runs; the mixed batch of 32 RMAT
  graphs of scales 12-18 (BFS from each vertex 0 + 20 PageRank supersteps)
  as one captured launch against the 32 solo runs;
  collaborative filtering on 480,189 x 17,770 users x items with 100M
  ratings, K = 32: loss (forward) against both factor gradients (adjoint);
  weighted PageRank on RMAT scale 22, T = 20: forward against the
  edge-weight gradient (adjoint);
  RMAT scale 26 (67,108,864 vertices): PageRank per superstep (GB/s against
  the HBM peak: its vectors no longer fit the caches), BFS from vertex 0,
  32-source batched BFS against 32 plain runs, and the weight gradient
  (T = 20) against its forward pass.

Prints one JSON line. Inputs are generated and loaded before the timed region
(graph loading is excluded, as in the paper's measurements).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS per generalized-SpMV iteration + % HBM peak; batched/adjoint vs plain"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
PR_SOURCES = [os.path.join(ROOT, "paper_1503_07241_amd", "csrc", f)
              for f in ("pagerank.hip", "tiles.h")]


def pr_source_sha():
    """SHA-256 of the PageRank superstep kernel's sources, in order."""
    h = hashlib.sha256()
    for f in PR_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pr_pull_rmat22_traffic.txt")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def ensure_built():
    from paper_1503_07241_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()


class Timer:
    """HIP events on torch's current stream (the stream the library launches on)."""

    def __init__(self):
        import torch
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)

    def ms(self, fn, reps=3):
        import torch
        fn()  # warm-up
        out = []
        for _ in range(reps):
            self.a.record()
            fn()
            self.b.record()
            torch.cuda.synchronize()
            out.append(self.a.elapsed_time(self.b))
        out.sort()
        return out[len(out) // 2]


def measured_traffic():
    """HBM bytes per PageRank superstep from the committed counter summary,
    or None when pagerank.hip changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source sha256") != pr_source_sha() or "hbm bytes per superstep" not in kv:
        return None
    return int(float(kv["hbm bytes per superstep"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the batched/adjoint comparisons")
    ap.add_argument("--no-scale26", action="store_true", help="skip the RMAT scale-26 measurements")
    ap.add_argument("--pr-only", type=int, default=0, metavar="K",
                    help="only run K PageRank passes (20 supersteps) and a 1 GiB copy, for "
                         "hardware-counter runs")
    ap.add_argument("--tc-only", type=int, default=0, metavar="K",
                    help="only run K triangle counts, for hardware-counter runs")
    ap.add_argument("--ablation", action="store_true",
                    help="only the ablation of the paper's design choices (Sec. 5.4, Fig. 7) on "
                         "RMAT scale 22: frontier as bitvector or sorted list, equal-edge or "
                         "thread-per-vertex push, push vs pull, PageRank tiles and LDS copy")
    ap.add_argument("--tc-cold", action="store_true",
                    help="with --tc-only: free the work plan before each count (cold calls)")
    ap.add_argument("--sssp-pull-div", type=int, default=0, metavar="D",
                    help="with --sssp-only: the pull_div tuning value (1: push only)")
    ap.add_argument("--sssp-only", type=int, default=0, metavar="K",
                    help="only run K SSSP runs from vertex 0 on the scale-22 directed graph, "
                         "for hardware-counter runs")
    ap.add_argument("--cf-only", type=int, default=0, metavar="K",
                    help="only run K CF forward + backward passes on the 100M-rating graph, "
                         "for hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    ensure_built()
    import numpy as np
    import torch

    import graphgen as gg
    import paper_1503_07241_amd as gm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.cf_only:
        R = gg.cf_ratings()
        PU, PV = gg.cf_point(R.n_users, R.n_items)
        rg = gm.RatingGraph.from_coo(R.n_users, R.n_items, R.user, R.item, R.rating)
        pu, pv = torch.tensor(PU, device=dev), torch.tensor(PV, device=dev)
        loss = torch.empty(1, dtype=torch.float64, device=dev)
        gu, gv = torch.empty_like(pu), torch.empty_like(pv)
        for _ in range(args.cf_only):
            gm.cf_forward(rg, pu, pv, 0.05, loss)
            gm.cf_backward(rg, pu, pv, 0.05, 1.0, gu, gv)
        torch.cuda.synchronize()
        print(json.dumps({"cf_runs": args.cf_only, "ratings": int(R.m)}), flush=True)
        return
    scale = args.scale
    t0 = time.time()
    n, s, d = gg.rmat(scale)
    w = gg.weights_u32(s, d)
    log("generated RMAT scale %d in %.1fs" % (scale, time.time() - t0))
    if args.pr_only:
        pr_counter_run(gm, torch, n, s, d, args.pr_only)
        return
    if args.ablation:
        print(json.dumps(run_ablation(gm, gg, torch, np, n, s, d, w)), flush=True)
        return
    if args.sssp_only:
        g = gm.Graph.from_coo(n, s, d, w=w, prep=gm.GM_PREP_DROP_SELF_LOOPS)
        if args.sssp_pull_div:
            g.set_tuning(pull_div=args.sssp_pull_div)
        root = torch.zeros(1, dtype=torch.int32, device=dev)
        dist = torch.empty(n, dtype=torch.int32, device=dev)
        for _ in range(args.sssp_only):
            dist.fill_(-1)
            dist[0] = 0
            it = gm.run_vertex_program(g, gm.GM_PROG_SSSP, root, -1, dist)
        torch.cuda.synchronize()
        print(json.dumps({"sssp_runs": args.sssp_only, "supersteps": it,
                          "edges": g.last_run_stats().edges_scanned}), flush=True)
        return
    if args.tc_only:
        g = gm.Graph.from_coo(n, s, d, prep=gm.GM_PREP_UPPER_DAG)
        tri = torch.empty(n, dtype=torch.int64, device=dev)
        for _ in range(args.tc_only):
            if args.tc_cold:
                g.release()
            tri.zero_()
            gm.run_vertex_program(g, gm.GM_PROG_TC, None, 1, tri)
        torch.cuda.synchronize()
        print(json.dumps({"tc_runs": args.tc_only, "m_dag": g.m}), flush=True)
        return
    t0 = time.time()  # graph loads: host edge lists in, device layouts out
    g_sym = gm.Graph.from_coo(n, s, d, prep=gm.GM_PREP_DROP_SELF_LOOPS | gm.GM_PREP_SYMMETRIZE,
                              layouts=gm.GM_LAYOUT_OUT)
    g_dir = gm.Graph.from_coo(n, s, d, w=w, prep=gm.GM_PREP_DROP_SELF_LOOPS,
                              layouts=gm.GM_LAYOUT_OUT | gm.GM_LAYOUT_IN)
    g_dag = gm.Graph.from_coo(n, s, d, prep=gm.GM_PREP_UPPER_DAG,
                              layouts=gm.GM_LAYOUT_OUT | gm.GM_LAYOUT_IN)
    m_dir, m_sym, m_dag = g_dir.m, g_sym.m, g_dag.m
    log("graphs loaded: m_dir=%d m_sym=%d m_dag=%d (%.1fs)" % (m_dir, m_sym, m_dag,
                                                            time.time() - t0))

    level = torch.empty(n, dtype=torch.int32, device=dev)
    dist = torch.empty(n, dtype=torch.int32, device=dev)
    rank = torch.empty(n, dtype=torch.float32, device=dev)
    tri = torch.empty(n, dtype=torch.int64, device=dev)
    root = torch.zeros(1, dtype=torch.int32, device=dev)
    T_PR = 20
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for k in ("bfs", "sssp", "pr", "tc")}
    acc = {k: 0.0 for k in ev}
    edges = {}
    steps_sssp = [0]

    def step(record: bool):
        e = ev["bfs"]
        if record:
            e[0].record()
        level.fill_(gm.INF_LEVEL)
        level[0] = 0
        gm.run_vertex_program(g_sym, gm.GM_PROG_BFS, root, -1, level)
        if record:
            e[1].record()
        edges["bfs"] = g_sym.last_run_stats().edges_scanned
        e = ev["sssp"]
        if record:
            e[0].record()
        dist.fill_(-1)
        dist[0] = 0
        gm.run_vertex_program(g_dir, gm.GM_PROG_SSSP, root, -1, dist)
        if record:
            e[1].record()
        edges["sssp"] = g_dir.last_run_stats().edges_scanned
        steps_sssp[0] = g_dir.last_run_stats().supersteps
        e = ev["pr"]
        if record:
            e[0].record()
        rank.fill_(1.0)
        gm.run_vertex_program(g_dir, gm.GM_PROG_PAGERANK, None, T_PR, rank)
        if record:
            e[1].record()
        edges["pr"] = T_PR * m_dir
        e = ev["tc"]
        if record:
            e[0].record()
        tri.zero_()
        gm.run_vertex_program(g_dag, gm.GM_PROG_TC, None, 1, tri)
        if record:
            e[1].record()
        edges["tc"] = m_dag
        if record:
            torch.cuda.synchronize()
            for k, (a, b) in ev.items():
                acc[k] += a.elapsed_time(b)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    log("timed %d steps in %.2fs" % (args.steps, wall))
    ms_step = 1e3 * wall / args.steps
    edges_step = sum(edges.values())
    gteps = edges_step / (wall / args.steps) / 1e9
    programs = {}
    for k in ev:
        ms = acc[k] / args.steps
        programs[k] = {"ms": round(ms, 4), "edges": int(edges[k]),
                       "gteps": round(edges[k] / (ms * 1e-3) / 1e9, 2)}
    # algorithmic bytes of the BFS and SSSP runs: BFS reads each symmetric
    # edge's index once (4 m_sym) and 20 B per vertex (offsets, level,
    # frontier bits); SSSP 8 B per relaxed edge (index + weight) plus 12 B
    # per vertex and superstep
    alg = {"bfs": 4 * m_sym + 20 * n,
           "sssp": 8 * edges["sssp"] + 12 * n * steps_sssp[0]}
    for k, b in alg.items():
        gbs = b / (acc[k] / args.steps * 1e-3) / 1e9
        programs[k].update({"algorithmic_bytes": int(b), "algorithmic_gbs": round(gbs, 1),
                            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)})
    # First-call costs: the triangle count's work plan (built on the device)
    # and the PageRank pull layout, each from a released graph, next to the
    # warm per-call times above.
    ea, eb, ec = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    tc_plan, tc_cold, pr_layout, sssp_layout = [], [], [], []
    for _ in range(3):
        g_dag.release()
        ea.record()
        g_dag.prepare(gm.GM_PROG_TC)
        eb.record()
        tri.zero_()
        gm.run_vertex_program(g_dag, gm.GM_PROG_TC, None, 1, tri)
        ec.record()
        torch.cuda.synchronize()
        tc_plan.append(ea.elapsed_time(eb))
        tc_cold.append(ea.elapsed_time(ec))
        g_dir.release()
        ea.record()
        g_dir.prepare(gm.GM_PROG_PAGERANK)
        eb.record()
        g_dir.prepare(gm.GM_PROG_SSSP)
        ec.record()
        torch.cuda.synchronize()
        pr_layout.append(ea.elapsed_time(eb))
        sssp_layout.append(eb.elapsed_time(ec))
    med = lambda a: sorted(a)[len(a) // 2]  # noqa: E731
    programs["tc"].update({"warm_ms": programs["tc"]["ms"], "plan_ms": round(med(tc_plan), 3),
                           "cold_ms": round(med(tc_cold), 3)})
    programs["pr"]["layout_ms"] = round(med(pr_layout), 3)
    programs["sssp"]["layout_ms"] = round(med(sssp_layout), 3)
    step(False)  # rebuild the released schedules before anything else is timed
    torch.cuda.synchronize()
    log("programs: %s" % json.dumps(programs))

    # Dominant SpMV kernel: the PageRank superstep (pr_pull + the combine of
    # split rows). Its time per superstep is the difference of a 21- and a
    # 1-superstep run over 20, which removes the per-run set-up kernels.
    # Algorithmic bytes per superstep (a pull SpMV over a CSC with 64-bit
    # offsets): every in-edge index (4 m), the row offsets (8 N), the gathered
    # message of every vertex (4 N), 1/outdeg (4 N), the new rank and the new
    # message written (4 N each): 4 m + 24 N. The count for this library's
    # own layout (32-bit offsets, rows without in-edges written once per run,
    # messages of vertices without out-edges never read) is reported beside it.
    tm = Timer()

    def pr_run(T):
        def f():
            rank.fill_(1.0)
            gm.run_vertex_program(g_dir, gm.GM_PROG_PAGERANK, None, T, rank)
        return f

    t21, t1 = tm.ms(pr_run(21), 5), tm.ms(pr_run(1), 5)
    pr_ms_launch = (t21 - t1) / 20
    info = g_dir.info()
    pr_bytes = 4 * m_dir + 24 * n
    layout_bytes = 4 * m_dir + 12 * info.n_dst + 4 * info.n_src
    achieved = pr_bytes / (pr_ms_launch * 1e-3) / 1e9
    # the committed counter summary is of the scale-22 workload's kernel
    traffic = measured_traffic() if scale == 22 else None

    forms = None
    if not args.no_forms:
        forms = measure_forms(gm, gg, torch, np, tm, g_dir, n, m_dir)
    if not args.no_forms:
        forms["paper_workloads"] = measure_paper_workloads(gm, gg, torch, np, tm)
    if not args.no_scale26:
        for g in (g_sym, g_dir, g_dag):
            g.close()
        torch.cuda.empty_cache()
        forms = forms or {}
        forms["rmat26"] = measure_scale26(gm, gg, torch, np, tm)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(n, s, d, w, programs)

    out = {
        "metric": METRIC,
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32/u32 (BFS, SSSP), f32 (PageRank), u64 (TC)",
        "data": "synthetic",
        "config": {"workload": "RMAT scale %d: BFS + SSSP + PageRank x20 + triangle count, "
                               "single source 0" % scale,
                   "scale": scale, "n": n, "m_dir": m_dir, "m_sym": m_sym, "m_dag": m_dag,
                   "edges_per_step": int(edges_step),
                   "schedules": "warm: per-graph schedules (triangle-count work plan, PageRank "
                                "pull layout, SSSP pull layout) are built by the warm-up steps; "
                                "their first-call costs are programs.tc.plan_ms / cold_ms, "
                                "programs.pr.layout_ms and programs.sssp.layout_ms, and "
                                "value_cold_schedules counts them in every step"},
        "value_cold_schedules": round(edges_step / ((ms_step - programs["tc"]["warm_ms"]
                                                     + programs["tc"]["cold_ms"]
                                                     + programs["pr"]["layout_ms"]
                                                     + programs["sssp"]["layout_ms"]) * 1e-3)
                                      / 1e9, 3),
        "programs": programs,
        "roofline": {"kernel": "pr_pull (PageRank superstep)", "bound": "hbm",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_counts": "rocprofv3 FETCH_SIZE + WRITE_SIZE per superstep, "
                                       "calibrated on a 1 GiB copy: L2 fills from and "
                                       "write-backs to the memory fabric, Infinity Cache "
                                       "hits included",
                     "algorithmic_bytes_per_launch": int(pr_bytes),
                     "algorithmic_bytes_formula": "4 m + 24 N",
                     "layout_bytes_per_launch": int(layout_bytes),
                     "launch_ms": round(pr_ms_launch, 5),
                     "pr_gteps": round(m_dir / (pr_ms_launch * 1e-3) / 1e9, 2)},
        "forms": forms,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def measure_forms(gm, gg, torch, np, tm, g22, n22, m22):
    """Batched and adjoint forms against the plain runs they stand for."""
    dev = torch.device("cuda:0")
    res = {}
    t0 = time.time()

    def ids(a):
        return torch.tensor(np.asarray(a), dtype=torch.int32, device=dev)

    # ---- batched sources, RMAT scale 20 ----
    n, s, d = gg.rmat(20)
    w = gg.weights_u32(s, d)
    gs = gm.Graph.from_coo(n, s, d, prep=gm.GM_PREP_DROP_SELF_LOOPS | gm.GM_PREP_SYMMETRIZE,
                           layouts=gm.GM_LAYOUT_OUT)
    gd = gm.Graph.from_coo(n, s, d, w=w, prep=gm.GM_PREP_DROP_SELF_LOOPS)
    S = gg.sources(n, s, d, 64, gg.SEED_BATCH_SOURCES)
    P = gg.sources(n, s, d, 128, gg.SEED_PPR_SEEDS)
    Sd, Pd = ids(S), ids(P)
    one = [ids([v]) for v in S]
    onep = [ids([v]) for v in P]
    prop = torch.empty(n, dtype=torch.int32, device=dev)
    prank = torch.empty(n, dtype=torch.float32, device=dev)
    blk64 = torch.empty((n, 64), dtype=torch.int32, device=dev)
    blk128 = torch.empty((n, 128), dtype=torch.float32, device=dev)
    plain_edges = {"bfs": 0, "sssp": 0}

    def plain_min(kind, g, inf):
        def f():
            tot = 0
            for r in one:
                prop.fill_(inf)
                prop[r] = 0
                gm.run_vertex_program(g, kind, r, -1, prop)
                tot += g.last_run_stats().edges_scanned
            plain_edges["bfs" if kind == gm.GM_PROG_BFS else "sssp"] = tot
        return f

    def plain_ppr():
        for r in onep:
            prank.zero_()
            prank[r] = 1.0
            gm.run_vertex_program(gd, gm.GM_PROG_PPR, r, 20, prank)

    entries = [
        ("bfs64", lambda: gm.run_batched(gs, gm.GM_PROG_BFS, Sd, -1, blk64),
         plain_min(gm.GM_PROG_BFS, gs, gm.INF_LEVEL), "bfs"),
        ("sssp64", lambda: gm.run_batched(gd, gm.GM_PROG_SSSP, Sd, -1, blk64),
         plain_min(gm.GM_PROG_SSSP, gd, -1), "sssp"),
        ("ppr128", lambda: gm.run_batched(gd, gm.GM_PROG_PPR, Pd, 20, blk128), plain_ppr, None),
    ]
    for name, batched, plain, ek in entries:
        tb = tm.ms(batched, 3)
        tp = tm.ms(plain, 1)
        e = plain_edges[ek] if ek else 20 * len(P) * gd.m
        res[name] = {"batched_ms": round(tb, 3), "plain_ms": round(tp, 3),
                     "speedup": round(tp / tb, 2),
                     "batched_gteps": round(e / (tb * 1e-3) / 1e9, 2),
                     "plain_gteps": round(e / (tp * 1e-3) / 1e9, 2)}
    log("batched forms: %s (%.1fs)" % (json.dumps(res), time.time() - t0))
    del blk64, blk128

    # ---- mixed batch: 32 graphs, one captured launch ----
    raws = [gg.rmat(sc, seed=seed) for sc, seed in gg.mixed_batch_specs()]
    msym = [gm.Graph.from_coo(a, b, c, prep=gm.GM_PREP_DROP_SELF_LOOPS | gm.GM_PREP_SYMMETRIZE,
                              layouts=gm.GM_LAYOUT_OUT) for a, b, c in raws]
    mdir = [gm.Graph.from_coo(a, b, c) for a, b, c in raws]
    usym, udir = gm.Graph.union(msym), gm.Graph.union(mdir)
    base = gm.union_bases(msym)
    N = int(base[-1])
    roots = ids(base[:-1])
    ulv = torch.empty(N, dtype=torch.int32, device=dev)
    upr = torch.empty(N, dtype=torch.float32, device=dev)
    plan = gm.Plan([gm.PlanRun(usym, gm.GM_PROG_BFS, ulv, roots, max_iters=32),
                    gm.PlanRun(udir, gm.GM_PROG_PAGERANK, upr, max_iters=20)])
    zero = ids([0])
    solo = [(torch.empty(a, dtype=torch.int32, device=dev),
             torch.empty(a, dtype=torch.float32, device=dev)) for a, _, _ in raws]

    def solo_runs():
        for gsy, gdi, (lv, pr) in zip(msym, mdir, solo):
            lv.fill_(gm.INF_LEVEL)
            lv[0] = 0
            gm.run_vertex_program(gsy, gm.GM_PROG_BFS, zero, -1, lv)
            pr.fill_(1.0)
            gm.run_vertex_program(gdi, gm.GM_PROG_PAGERANK, None, 20, pr)

    tb = tm.ms(plan.launch, 5)
    tp = tm.ms(solo_runs, 3)
    conv = plan.results()[0][1]
    res["mixed32"] = {"graphs": len(raws), "vertices": N, "one_launch_ms": round(tb, 3),
                      "solo_runs_ms": round(tp, 3), "speedup": round(tp / tb, 2),
                      "bfs_converged": bool(conv)}
    plan.close()
    log("mixed batch: %s (%.1fs)" % (json.dumps(res["mixed32"]), time.time() - t0))

    # ---- adjoint: collaborative filtering, 100M ratings ----
    R = gg.cf_ratings()
    PU, PV = gg.cf_point(R.n_users, R.n_items)
    rg = gm.RatingGraph.from_coo(R.n_users, R.n_items, R.user, R.item, R.rating)
    del R
    pu, pv = torch.tensor(PU, device=dev), torch.tensor(PV, device=dev)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    gu, gv = torch.empty_like(pu), torch.empty_like(pv)
    tf = tm.ms(lambda: gm.cf_forward(rg, pu, pv, 0.05, loss), 5)
    tbk = tm.ms(lambda: gm.cf_backward(rg, pu, pv, 0.05, 1.0, gu, gv), 5)
    tu = tm.ms(lambda: gm.cf_backward(rg, pu, pv, 0.05, 1.0, gu, None), 5)
    tv = tm.ms(lambda: gm.cf_backward(rg, pu, pv, 0.05, 1.0, None, gv), 5)
    ratings, K = 100_000_000, 32
    nu, ni = pu.shape[0], pv.shape[0]
    # Algorithmic bytes and flops. Forward (loss): each rating's index and
    # value (5 B) and both factor matrices read once; 2 K flops for the dot
    # product and 3 for the squared error. Backward (both gradients, one pass
    # per direction): per pass 5 B per rating, both factor matrices read and
    # one gradient matrix written; per rating and pass 2 K + 2 flops for the
    # residual and 2 K for the accumulation.
    fbytes = 5 * ratings + 4 * K * (nu + ni)
    bbytes = 2 * 5 * ratings + 2 * 4 * K * (nu + ni) + 4 * K * (nu + ni)
    fflops = (2 * K + 3) * ratings
    bflops = 2 * (4 * K + 2) * ratings

    def frac(b, f, ms):
        return {"gbs": round(b / (ms * 1e-3) / 1e9, 1),
                "hbm_frac": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "tflops": round(f / (ms * 1e-3) / 1e12, 2),
                "fp32_frac": round(f / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4)}

    res["cf_100M_k32"] = {"forward_ms": round(tf, 3), "backward_ms": round(tbk, 3),
                          "row_pass_ms": round(tu, 3), "transpose_pass_ms": round(tv, 3),
                          "backward_over_forward": round(tbk / tf, 2),
                          "forward_gratings_s": round(ratings / (tf * 1e-3) / 1e9, 2),
                          "transpose_gratings_s": round(ratings / (tv * 1e-3) / 1e9, 2),
                          "forward_bytes": fbytes, "forward_flops": fflops,
                          "backward_bytes": bbytes, "backward_flops": bflops,
                          "forward_roofline": frac(fbytes, fflops, tf),
                          "backward_roofline": frac(bbytes, bflops, tbk)}
    del rg, pu, pv, gu, gv
    log("cf: %s (%.1fs)" % (json.dumps(res["cf_100M_k32"]), time.time() - t0))

    # ---- adjoint: PageRank edge-weight gradient, RMAT scale 22, T = 20 ----
    T = 20
    wt = torch.ones(m22, dtype=torch.float32, device=dev)
    hist = torch.empty((T + 1, n22), dtype=torch.float32, device=dev)
    hist[0].fill_(1.0)
    c = torch.tensor(gg.uniform_f32(n22, gg.SEED_PR_UPSTREAM), device=dev)
    gw = torch.empty_like(wt)
    tf = tm.ms(lambda: gm.pagerank_forward_w(g22, wt, 0.15, T, hist), 3)
    tbk = tm.ms(lambda: gm.pagerank_vjp_w(g22, wt, 0.15, T, hist, c, gw), 3)
    res["pr_weight_grad_rmat22_T20"] = {
        "forward_ms": round(tf, 3), "vjp_ms": round(tbk, 3), "vjp_over_forward": round(tbk / tf, 2),
        "forward_gteps": round(T * m22 / (tf * 1e-3) / 1e9, 2),
        "vjp_gteps": round(T * m22 / (tbk * 1e-3) / 1e9, 2)}
    log("pr grad: %s (%.1fs)" % (json.dumps(res["pr_weight_grad_rmat22_T20"]), time.time() - t0))
    return res


def measure_paper_workloads(gm, gg, torch, np, tm):
    """The paper's own triangle-counting and SSSP graphs (Sec. 5.1, Table 1)
    and a long-diameter graph: triangle counting on RMAT scale 20 with
    a = .45, b = c = .15 (cold: work plan built inside the call; warm: plan
    kept); SSSP from vertex 0 on RMAT scale 24 with a = .50, b = c = .10 and
    on a 2048 x 2048 grid (thousands of supersteps: the per-superstep cost)."""
    dev = torch.device("cuda:0")
    res = {}
    t0 = time.time()
    n, s, d = gg.rmat(20, a=0.45, b=0.15, c=0.15)
    g = gm.Graph.from_coo(n, s, d, prep=gm.GM_PREP_UPPER_DAG)
    cnt = torch.empty(n, dtype=torch.int64, device=dev)

    def tc_cold():
        g.release()
        cnt.zero_()
        gm.run_vertex_program(g, gm.GM_PROG_TC, None, 1, cnt)

    def tc_warm():
        cnt.zero_()
        gm.run_vertex_program(g, gm.GM_PROG_TC, None, 1, cnt)

    tcold, twarm = tm.ms(tc_cold, 3), tm.ms(tc_warm, 5)
    res["tc_rmat20_a45"] = {"m_dag": g.m, "cold_ms": round(tcold, 3), "warm_ms": round(twarm, 3),
                            "gteps_warm": round(g.m / (twarm * 1e-3) / 1e9, 2),
                            "gteps_cold": round(g.m / (tcold * 1e-3) / 1e9, 2)}
    g.close()
    root = torch.zeros(1, dtype=torch.int32, device=dev)
    for name, (n, s, d) in (("sssp_rmat24_a50", gg.rmat(24, a=0.50, b=0.10, c=0.10)),
                            ("sssp_grid2048", gg.grid2d(2048, 2048))):
        w = gg.weights_u32(s, d)
        g = gm.Graph.from_coo(n, s, d, w=w, prep=gm.GM_PREP_DROP_SELF_LOOPS)
        dist = torch.empty(n, dtype=torch.int32, device=dev)
        info = {}

        def run():
            dist.fill_(-1)
            dist[0] = 0
            info["it"] = gm.run_vertex_program(g, gm.GM_PROG_SSSP, root, -1, dist)
            info["edges"] = g.last_run_stats().edges_scanned
            info["pull"] = g.last_run_stats().pull_supersteps

        ms = tm.ms(run, 3)
        res[name] = {"n": n, "m": g.m, "ms": round(ms, 3), "supersteps": info["it"],
                     "pull_supersteps": info["pull"],
                     "us_per_superstep": round(1e3 * ms / max(info["it"], 1), 2),
                     "edges_relaxed": int(info["edges"]),
                     "gteps": round(info["edges"] / (ms * 1e-3) / 1e9, 2),
                     "m_per_s_gteps": round(g.m / (ms * 1e-3) / 1e9, 2)}
        g.close()
        del dist
    torch.cuda.empty_cache()
    log("paper workloads: %s (%.1fs)" % (json.dumps(res), time.time() - t0))
    return res


def measure_scale26(gm, gg, torch, np, tm):
    """RMAT scale 26: PageRank per superstep, BFS, 32-source batched BFS and
    the PageRank weight gradient, each after a warm-up run."""
    dev = torch.device("cuda:0")
    t0 = time.time()
    n, s, d = gg.rmat(26)
    res = {"n": n}
    g = gm.Graph.from_coo(n, s, d)
    info = g.info()
    m = info.m
    res["m_dir"] = m
    log("scale 26 directed graph: m=%d (%.1fs)" % (m, time.time() - t0))
    rank = torch.empty(n, dtype=torch.float32, device=dev)

    def pr(T):
        def f():
            rank.fill_(1.0)
            gm.run_vertex_program(g, gm.GM_PROG_PAGERANK, None, T, rank)
        return f

    per = (tm.ms(pr(21), 3) - tm.ms(pr(1), 3)) / 20
    alg = 4 * m + 24 * n  # as at scale 22: 4 m + 24 N per superstep
    res["pagerank"] = {"ms_per_superstep": round(per, 4),
                       "gteps": round(m / (per * 1e-3) / 1e9, 2),
                       "algorithmic_bytes": int(alg),
                       "algorithmic_gbs": round(alg / (per * 1e-3) / 1e9, 1),
                       "hbm_frac": round(alg / (per * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    T = 20
    w = torch.ones(m, dtype=torch.float32, device=dev)
    hist = torch.empty((T + 1, n), dtype=torch.float32, device=dev)
    hist[0].fill_(1.0)
    c = torch.tensor(gg.uniform_f32(n, gg.SEED_PR_UPSTREAM), device=dev)
    gw = torch.empty_like(w)
    tf = tm.ms(lambda: gm.pagerank_forward_w(g, w, 0.15, T, hist), 1)
    tb = tm.ms(lambda: gm.pagerank_vjp_w(g, w, 0.15, T, hist, c, gw), 1)
    res["pr_weight_grad_T20"] = {"forward_ms": round(tf, 2), "vjp_ms": round(tb, 2),
                                 "vjp_over_forward": round(tb / tf, 2),
                                 "vjp_gteps": round(T * m / (tb * 1e-3) / 1e9, 2)}
    del w, hist, gw, rank
    g.close()
    torch.cuda.empty_cache()
    log("scale 26 PageRank: %s (%.1fs)" % (json.dumps(res), time.time() - t0))
    gs = gm.Graph.from_coo(n, s, d, prep=gm.GM_PREP_DROP_SELF_LOOPS | gm.GM_PREP_SYMMETRIZE,
                           layouts=gm.GM_LAYOUT_OUT)
    S = gg.sources(n, s, d, 32, gg.SEED_BATCH_SOURCES)
    del s, d
    Sd = torch.tensor(S, dtype=torch.int32, device=dev)
    one = [torch.tensor([v], dtype=torch.int32, device=dev) for v in S]
    lv = torch.empty(n, dtype=torch.int32, device=dev)
    edges = {}

    def bfs(r):
        def f():
            lv.fill_(gm.INF_LEVEL)
            lv[r] = 0
            gm.run_vertex_program(gs, gm.GM_PROG_BFS, r, -1, lv)
            edges[int(r[0])] = gs.last_run_stats().edges_scanned
        return f

    tb0 = tm.ms(bfs(one[0]), 3)
    res["bfs"] = {"ms": round(tb0, 3), "gteps": round(edges[int(S[0])] / (tb0 * 1e-3) / 1e9, 2)}

    def plain_all():
        for r in one:
            bfs(r)()

    tp = tm.ms(plain_all, 1)
    blk = torch.empty((n, 32), dtype=torch.int32, device=dev)
    tbb = tm.ms(lambda: gm.run_batched(gs, gm.GM_PROG_BFS, Sd, -1, blk), 2)
    e_all = sum(edges.values())
    res["bfs32"] = {"batched_ms": round(tbb, 2), "plain_ms": round(tp, 2),
                    "speedup": round(tp / tbb, 2),
                    "batched_gteps": round(e_all / (tbb * 1e-3) / 1e9, 2),
                    "plain_gteps": round(e_all / (tp * 1e-3) / 1e9, 2)}
    del blk, lv
    gs.close()
    torch.cuda.empty_cache()
    log("scale 26: %s (%.1fs)" % (json.dumps(res), time.time() - t0))
    return res


def run_ablation(gm, gg, torch, np, n, s, d, w):
    """Each design choice of the paper's Fig. 7 (Sec. 5.4) swapped for its
    alternative on the scale-22 workload, results asserted equal to the
    default schedule's (BFS, SSSP bit-exact; PageRank within 2e-5 relative):
      frontier: bitvector (default) vs sorted list of distinct ids;
      load balance: equal edge ranges per wavefront (default) vs one thread
        per active vertex;
      direction (BFS, SSSP): push with pull supersteps for large frontiers
        (default) vs push only;
      vertex order (BFS, SSSP): the caller's labels (default) vs a copy
        relabelled by decreasing in-degree, on the generator's labels and on
        a seeded random permutation of them (scrambled_labels);
      PageRank: edge tiles + LDS copy of the hottest messages (default),
        tiles without the LDS copy, one thread per row."""
    dev = torch.device("cuda:0")
    LIST, VPUSH, ROWPULL, DEG = (gm._lib.GM_VARIANT_LIST_FRONTIER,
                                  gm._lib.GM_VARIANT_VERTEX_PUSH, gm._lib.GM_VARIANT_ROW_PULL,
                                  gm._lib.GM_VARIANT_DEGREE_ORDER)
    tm = Timer()
    g_sym = gm.Graph.from_coo(n, s, d, prep=gm.GM_PREP_DROP_SELF_LOOPS | gm.GM_PREP_SYMMETRIZE,
                              layouts=gm.GM_LAYOUT_OUT)
    g_dir = gm.Graph.from_coo(n, s, d, w=w, prep=gm.GM_PREP_DROP_SELF_LOOPS)
    root = torch.zeros(1, dtype=torch.int32, device=dev)
    lv = torch.empty(n, dtype=torch.int32, device=dev)
    dist = torch.empty(n, dtype=torch.int32, device=dev)
    rank = torch.empty(n, dtype=torch.float32, device=dev)
    out, ref = {"bfs": {}, "sssp": {}, "pagerank": {}}, {}

    def bfs():
        lv.fill_(gm.INF_LEVEL)
        lv[0] = 0
        gm.run_vertex_program(g_sym, gm.GM_PROG_BFS, root, -1, lv)

    def sssp():
        dist.fill_(-1)
        dist[0] = 0
        gm.run_vertex_program(g_dir, gm.GM_PROG_SSSP, root, -1, dist)

    def pr(T):
        def f():
            rank.fill_(1.0)
            gm.run_vertex_program(g_dir, gm.GM_PROG_PAGERANK, None, T, rank)
        return f

    frontier_variants = [("bitvector_frontier+equal_edge_push", 0), ("list_frontier", LIST),
                         ("thread_per_vertex_push", VPUSH),
                         ("list_frontier+thread_per_vertex_push", LIST | VPUSH),
                         ("degree_ordered_labels", DEG)]
    for name, var in frontier_variants:
        # pull supersteps once more than n / pull_div vertices are active: 1
        # never pulls, 128 is the default switch
        for dname, pull_div in (("push_pull", 128), ("push_only", 1)):
            g_sym.set_tuning(variant=var, pull_div=pull_div)
            ms = tm.ms(bfs, 3)
            e = g_sym.last_run_stats().edges_scanned
            got = lv.cpu().numpy()
            if "bfs" not in ref:
                ref["bfs"] = got.copy()
            assert np.array_equal(got, ref["bfs"]), (name, dname)
            out["bfs"][name + "/" + dname] = {"ms": round(ms, 3), "gteps": round(e / ms / 1e6, 2)}
        for dname, pull_div in (("push_pull", 128), ("push_only", 1)):
            g_dir.set_tuning(variant=var, pull_div=pull_div)
            ms = tm.ms(sssp, 3)
            e = g_dir.last_run_stats().edges_scanned
            got = dist.cpu().numpy()
            if "sssp" not in ref:
                ref["sssp"] = got.copy()
            assert np.array_equal(got, ref["sssp"]), (name, dname)
            out["sssp"][name + "/" + dname] = {"ms": round(ms, 3),
                                               "gteps": round(e / ms / 1e6, 2)}
    g_dir.set_tuning(variant=0, pull_div=128)
    # The same graphs with the vertex labels scrambled (seeded permutation):
    # results are the unscrambled ones, permuted.
    perm = gg.label_permutation(n)
    sg_sym = gm.Graph.from_coo(n, perm[s], perm[d],
                               prep=gm.GM_PREP_DROP_SELF_LOOPS | gm.GM_PREP_SYMMETRIZE,
                               layouts=gm.GM_LAYOUT_OUT)
    sg_dir = gm.Graph.from_coo(n, perm[s], perm[d], w=w, prep=gm.GM_PREP_DROP_SELF_LOOPS)
    sroot = torch.tensor([int(perm[0])], dtype=torch.int32, device=dev)
    out["scrambled_labels"] = {}
    for name, var in (("caller_labels", 0), ("degree_ordered_labels", DEG)):
        sg_sym.set_tuning(variant=var)
        sg_dir.set_tuning(variant=var)

        def sbfs():
            lv.fill_(gm.INF_LEVEL)
            lv[int(perm[0])] = 0
            gm.run_vertex_program(sg_sym, gm.GM_PROG_BFS, sroot, -1, lv)

        def ssssp():
            dist.fill_(-1)
            dist[int(perm[0])] = 0
            gm.run_vertex_program(sg_dir, gm.GM_PROG_SSSP, sroot, -1, dist)
        bms = tm.ms(sbfs, 3)
        be = sg_sym.last_run_stats().edges_scanned
        assert np.array_equal(lv.cpu().numpy()[perm], ref["bfs"]), name
        sms = tm.ms(ssssp, 3)
        se = sg_dir.last_run_stats().edges_scanned
        assert np.array_equal(dist.cpu().numpy()[perm], ref["sssp"]), name
        out["scrambled_labels"][name] = {
            "bfs": {"ms": round(bms, 3), "gteps": round(be / bms / 1e6, 2)},
            "sssp": {"ms": round(sms, 3), "gteps": round(se / sms / 1e6, 2)}}
    sg_sym.close()
    sg_dir.close()
    m = g_dir.m
    for name, var, hot in (("tiles+lds_hot_set", 0, 40960), ("tiles_no_lds", 0, 0),
                           ("row_per_thread", ROWPULL, 40960)):
        g_dir.set_tuning(variant=var, pr_hot=hot)
        per = (tm.ms(pr(21), 3) - tm.ms(pr(1), 3)) / 20
        pr(20)()
        torch.cuda.synchronize()
        got = rank.cpu().numpy().astype(np.float64)
        if "pr" not in ref:
            ref["pr"] = got.copy()
        err = float(np.max(np.abs(got - ref["pr"]) / ref["pr"]))
        assert err <= 2e-5, (name, err)
        out["pagerank"][name] = {"ms_per_superstep": round(per, 4),
                                 "gteps": round(m / per / 1e6, 2),
                                 "gbs_4m_24n": round((4 * m + 24 * n) / per / 1e6, 1),
                                 "max_rel_diff_vs_default": err}
    out["config"] = {"workload": "RMAT scale 22 (BFS symmetrised, SSSP/PageRank directed), "
                                 "source 0", "n": n, "m_dir": m, "m_sym": g_sym.m}
    return out


def pr_counter_run(gm, torch, n, s, d, K):
    """K PageRank runs (20 supersteps each) on the scale-22 directed graph and
    one copy of 1 GiB (256 Mi floats) for calibrating the byte counters."""
    g = gm.Graph.from_coo(n, s, d)
    rank = torch.empty(n, dtype=torch.float32, device="cuda")
    for _ in range(K):
        rank.fill_(1.0)
        gm.run_vertex_program(g, gm.GM_PROG_PAGERANK, None, 20, rank)
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    info = g.info()
    print(json.dumps({"pr_runs": K, "m": info.m, "n_dst": info.n_dst, "n_src": info.n_src,
                      "copy_bytes": 1 << 30}), flush=True)


def host_info():
    """The host's CPU count (as the OS reports it and as this process may use)
    and CPU model."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def cpu_baseline(n, s, d, w, programs):
    """The oracle (single-threaded C) on a bounded sample of the same step:
    queue BFS and Dijkstra SSSP from vertex 0 in full, 2 of the 20 PageRank
    supersteps, and the triangle count's per-receiver counts on a stratified
    sample of receivers (for each in-degree class [2^b, 2^(b+1)) up to
    max(4, 2^(16 - b)) receivers, timed together and scaled by the class
    size). The oracle's step time is BFS + SSSP + 20 x (one PageRank
    superstep) + the triangle-count estimate, and value = the step's edges
    (the GPU run's counts, so both figures count the same work) over it."""
    import numpy as np

    import oracle
    t0 = time.time()
    gs = oracle.prepare(n, s, d, mode="symmetric")
    gd = oracle.prepare(n, s, d, w=w)
    gin = oracle.Graph(gd.n, gd.off, gd.idx).transpose()
    dag_in = oracle.dag_in_lists(oracle.prepare(n, s, d, mode="dag"))
    log("oracle graphs prepared in %.1fs" % (time.time() - t0))
    t = time.perf_counter()
    oracle.bfs(gs, 0)
    t_bfs = time.perf_counter() - t
    t = time.perf_counter()
    oracle.sssp(gd, 0)
    t_sssp = time.perf_counter() - t
    t = time.perf_counter()
    oracle.pagerank(gd, 0.15, 2, g_in=gin)
    t_pr = (time.perf_counter() - t) / 2
    indeg = np.diff(dag_in.off)
    cls = np.where(indeg > 0, np.floor(np.log2(np.maximum(indeg, 1))), -1).astype(np.int64)
    rng = np.random.default_rng(0)
    t_tc, t_tc_sample, sampled = 0.0, 0.0, 0
    for b in range(int(cls.max()) + 1):
        members = np.flatnonzero(cls == b)
        if len(members) == 0:
            continue
        k = min(len(members), max(4, 1 << max(0, 16 - b)))
        pick = np.sort(rng.choice(members, k, replace=False)).astype(np.int32)
        t = time.perf_counter()
        oracle.triangles_at(dag_in, pick)
        dt = time.perf_counter() - t
        t_tc_sample += dt
        t_tc += dt / k * len(members)
        sampled += k
    times = {"bfs": t_bfs, "sssp": t_sssp, "pr": 20 * t_pr, "tc": t_tc}
    step_s = sum(times.values())
    edges = sum(programs[k]["edges"] for k in times)
    per = {k: {"s": round(v, 3), "gteps": round(programs[k]["edges"] / v / 1e9, 4)}
           for k, v in times.items()}
    per["pr"]["s_per_superstep"] = round(t_pr, 4)
    per["tc"]["estimated"] = True
    return {"value": round(edges / step_s / 1e9, 4), "unit": "GTEPS", "cores": 1,
            "kind": "oracle", "step_s": round(step_s, 2), "programs": per,
            "host": host_info(),
            "sample": "RMAT scale-%d step on the oracle: queue BFS (%.3fs) + Dijkstra SSSP "
                      "(%.3fs) + 2 of 20 PageRank supersteps in FP64 (%.4fs each) + triangle "
                      "counts of %d receivers stratified by in-degree (%.2fs, scaled to an "
                      "estimated %.1fs for all)" % (int(n).bit_length() - 1, t_bfs, t_sssp, t_pr,
                                                    sampled, t_tc_sample, t_tc)}


if __name__ == "__main__":
    main()
