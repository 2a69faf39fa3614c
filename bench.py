"""Benchmark of the MI355X keyword-search hot path.

Default workload (the largest single-GPU batched configuration with
d_max = 3): R-MAT(.57,.19,.19,.05) with 2^24 vertices and 2^28 sampled
edges (263,429,032 after dropping loops and repeats), labels the leaves of
a complete 8-ary type tree of depth 6 (Zipf(1.0), 1-3 per vertex), and a
batch of 512 queries of 2-6 type keywords (a keyword matches its type and
every type below it), d_max = 3, top-50. One step = one batched pass of the
whole hot path (plan, seed, level expansion, finalize, root filter and
score, top-k, answer graphs, result copy) over those 512 queries; inputs
(graph, labels, type tree) are resident in HBM before timing starts. By
default the steps are pipelined: batch i + 1 is submitted (planned,
uploaded, enqueued) before batch i is collected, so host planning and
result unpacking overlap device time; --pipeline 0 times one synchronous
call per step instead.

Printed as one JSON line: queries/s of the batched path (value), GTEPS,
per-step latency percentiles, the plain one-query-per-call path on the same
queries (qps, p50/p99 latency, speedup, and whether every answer equals the
batched one), the roofline of the dominant kernel from HIP events recorded
on the library's stream during the timed steps, and the CPU oracle timed on
bounded samples of the same queries: one thread pinned to one core, and
one query per worker across the host's cores.

Other workloads: --workload rmat20_batch256 --autotune 1 is the 256-query
mixed batch (2-8 keywords, d_max 2-4) on the 2^20-vertex graph, tuned by the
library's autotuner first; rmat20_q4 (100 four-keyword queries on the same
graph), chunglu10k, rmat26_serve (the serving loop) and peel_rmat24 (parallel
peeling) are also available.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "keyword queries/sec + GTEPS (% of HBM roofline) at d_max=3; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str, scale: int | None, nq: int | None):
    from synth import workloads as W
    if name == "rmat20_q4":
        g, qs = W.rmat20_q4(scale or 20, nq or 100)
        desc = dict(graph="R-MAT(.57,.19,.19,.05) 2^%d vertices, 2^%d sampled edges" % (scale or 20, (scale or 20) + 4),
                    labels="10000 labels Zipf(1.0), 1-3 per vertex", keywords=4, d_max=3, k=20)
    elif name == "rmat20_batch256":
        g, qs = W.rmat20_batch256(scale or 20, nq or 256)
        desc = dict(graph="R-MAT 2^%d vertices" % (scale or 20), keywords="2-8", d_max="2-4", k=20)
    elif name == "chunglu10k":
        g = W.chunglu10k()
        qs = W.chunglu10k_queries(nq or 101)
        desc = dict(graph="Chung-Lu 2.1, 10k vertices, 50k edges", keywords=2, d_max=3, k=10)
    elif name == "rmat24_hier":
        g, qs = W.rmat24_hier(scale or 24, nq or 512)
        desc = dict(graph="R-MAT 2^%d vertices, type tree 8^6" % (scale or 24), keywords="2-6", d_max=3, k=50)
    elif name == "rmat26_serve":
        g, qs = W.rmat26_serve(scale or 26, nq or 4096)
        desc = dict(graph="R-MAT 2^%d vertices, 2^%d sampled edges" % (scale or 26, (scale or 26) + 4),
                    keywords="2-8", d_max="2-4", k=20)
    else:
        raise SystemExit(f"unknown workload {name}")
    return g, qs, desc


def byte_model(st: dict, n: int, kernel: str, launches: float = 0.0, fused: bool = True) -> float:
    """Algorithmic bytes of all launches of one kernel class in one step.

    expansion (push or pull) of level l, with U_l the frontier vertices,
    E_l their in-edges and T_l the vertices that gain a lane (= U_{l+1}),
    W the 64-lane words: 8|U_l| + 4E_l + 8W|U_l| + 16W|T_l|. A pull with the
    finalize fused in also writes, for every vertex, its next-frontier row
    when a level follows (8 Wp n) and each distance plane whose first level
    this is (8 Wp n per plane).
    finalize: one streaming pass over n*Wp words reading nxt and vis and
    writing the next frontier: 24 bytes per vertex-word, for every level
    not finalized inside a fused pull (level 0 has none when seeding by
    vertex, which writes it itself).
    score: 8*W*n*(2 + planes) (vis, the planes and, for the last level's
    arrivals it merges, nxt).
    """
    W, Wp, L = st["words"], st["words_padded"], st["levels"]
    f, fe, pulled = st["frontier"], st["frontier_edges"], st["pulled"]
    if kernel in ("pull", "push"):
        want = 1 if kernel == "pull" else 0
        tot = 0.0
        for lv in range(L):
            if (pulled[lv] == 1) != (want == 1) or f[lv] == 0:
                continue
            tot += 8 * f[lv] + 4 * fe[lv] + 8 * W * f[lv] + 16 * W * f[lv + 1]
            if want and fused:
                first_planes = sum(1 for b in range(4) if (1 << b) == lv + 1 and (1 << b) <= L)
                tot += 8.0 * Wp * n * ((1 if lv + 1 < L else 0) + first_planes)
        return tot
    if kernel == "finalize":
        if fused:
            return 24.0 * n * Wp * sum(1 for lv in range(L) if not pulled[lv])
        return 24.0 * n * Wp * launches
    if kernel == "score":
        planes = max(1, int(np.ceil(np.log2(L + 1)))) if L > 0 else 0
        return 8.0 * W * n * (2 + planes)
    return 0.0


def measured_traffic(kernel: str, workload: str, kernel_name: str | None = None):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when there is none, the
    kernel's source file changed since the counters were taken, or the
    summary was taken on another kernel of the class than `kernel_name` (the
    pull class runs as k_pull<T> or, finalize fused, as k_pull_fin<T>)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        line = line.strip().strip("`")
        if ":" in line:
            k, _, v = line.partition(":")
            fields[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2504_09311_amd", "csrc", fields.get("source", "kernels.hip"))
    if not os.path.exists(src):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if fields.get("source_sha256") != digest or "traffic_bytes_per_launch" not in fields:
        return None
    if kernel_name and fields.get("kernel_name", kernel_name) != kernel_name:
        return None
    return int(float(fields["traffic_bytes_per_launch"]))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, qs, budget_s: float, max_workers: int = 16):
    """The oracle on the host's cores, search only (its graph set-up is not
    timed): (a) one thread pinned to one core, queries in order until the
    budget is spent; (b) one query per worker on every core this process may
    use (at most max_workers), all started together, timed to the last."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    o = oracle.Oracle(g)
    cores = sorted(os.sched_getaffinity(0))
    workers = max(1, min(max_workers, len(cores)))
    os.sched_setaffinity(0, {cores[0]})
    try:
        t0 = time.perf_counter()
        done = 0
        for q in qs:
            o.search(q.kw, q.d_max, q.k)
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt1 = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, set(cores))
    par = qs[:workers]
    with ThreadPoolExecutor(max_workers=workers) as ex:
        t0 = time.perf_counter()
        list(ex.map(lambda q: o.search(q.kw, q.d_max, q.k), par))
        dtp = time.perf_counter() - t0
    o.close()
    host = dict(nproc=os.cpu_count(), usable_cores=len(cores), cpu_model=cpu_model())
    single = dict(value=round(done / dt1, 4), unit="queries/s", cores=1, kind="oracle",
                  sample=f"first {done} of the {len(qs)} queries, one thread pinned to core {cores[0]} "
                         f"({dt1:.1f} s)")
    return dict(value=round(len(par) / dtp, 4), unit="queries/s", cores=workers, kind="oracle",
                sample=f"first {len(par)} of the {len(qs)} queries, one per worker thread on {workers} cores "
                       f"({dtp:.1f} s wall)", single_thread=single, **host)


def same_answers(flat: dict, results) -> bool:
    """The flat batch result holds exactly the per-query results (roots,
    scores, keyword distances, answer edges)."""
    rp, dp, ep = flat["root_ptr"], flat["dist_ptr"], flat["edge_ptr"]
    for q, r in enumerate(results):
        a, b = int(rp[q]), int(rp[q + 1])
        if not (np.array_equal(flat["roots"][a:b], r.roots) and np.array_equal(flat["scores"][a:b], r.scores)):
            return False
        if not np.array_equal(flat["kw_dist"][int(dp[q]):int(dp[q + 1])], r.kw_dist.reshape(-1)):
            return False
        e0, e1 = int(ep[a]), int(ep[b])
        if not (np.array_equal(flat["edge_src"][e0:e1], r.edge_src) and
                np.array_equal(flat["edge_dst"][e0:e1], r.edge_dst) and
                np.array_equal(flat["edge_ptr"][a:b + 1] - e0, r.edge_ptr)):
            return False
    return True


def serve_bench(G, K, g, qs, args):
    """Serving: saturation throughput, then Poisson arrivals at fractions of it."""
    import threading
    from synth import workloads as W
    S = K.Server(G, max_dmax=4, tile_words=args.tile_words or 0, max_words=args.serve_words)
    # saturation: everything submitted at once
    n_sat = min(len(qs), args.serve_sat)
    for q in qs[:64]:
        S.submit(q.kw, q.d_max, q.k)
    while S.stats()["completed"] < 64:
        time.sleep(0.01)
    t0 = time.perf_counter()
    ts = [S.submit(q.kw, q.d_max, q.k) for q in qs[:n_sat]]
    te = 0
    for t in ts:
        te += S.wait(t).te
    sat_s = time.perf_counter() - t0
    sat_qps = n_sat / sat_s
    log("saturation: %d queries in %.3f s = %.1f queries/s" % (n_sat, sat_s, sat_qps))
    runs = []
    for frac in (0.5, 0.8):
        lam = frac * sat_qps
        count = max(1, min(len(qs), int(lam * args.serve_seconds)))
        arr = W.serve_arrivals(count, lam)
        S.close()
        S = K.Server(G, max_dmax=4, tile_words=args.tile_words or 0, max_words=args.serve_words)
        tickets = [None] * count
        lat = [0.0] * count
        sub_t = [0.0] * count

        def waiter():
            for i in range(count):
                while tickets[i] is None:
                    time.sleep(0.0002)
                S.wait(tickets[i])
                lat[i] = (time.perf_counter() - sub_t[i]) * 1e3

        th = threading.Thread(target=waiter)
        th.start()
        base = time.perf_counter()
        for i in range(count):
            dt = arr[i] - (time.perf_counter() - base)
            if dt > 0:
                time.sleep(dt)
            q = qs[i % len(qs)]
            sub_t[i] = time.perf_counter()
            tickets[i] = S.submit(q.kw, q.d_max, q.k)
        th.join()
        wall = time.perf_counter() - base
        st = S.stats()
        runs.append(dict(load=frac, offered_qps=round(lam, 2), queries=count, qps=round(count / wall, 2),
                         p50_ms=round(float(np.percentile(lat, 50)), 3), p99_ms=round(float(np.percentile(lat, 99)), 3),
                         server_p50_ms=round(st["p50_us"] / 1e3, 3), server_p99_ms=round(st["p99_us"] / 1e3, 3),
                         mean_active_words=round(st["mean_active_words"], 2), steps=st["steps"]))
        log("load %.1f: %s" % (frac, runs[-1]))
    S.close()
    return dict(saturation_qps=round(sat_qps, 2), saturation_queries=n_sat, saturation_gteps=round(te / sat_s / 1e9, 3),
                poisson=runs)


PEEL_METRIC = ("densest-subgraph parallel peeling (eps=0.1): input edges per second of a full run "
               "(input size over run time, not incidences read); rounds; time")


def peel_bytes(metric: str, n: int, sizes, summary) -> dict:
    """Algorithmic bytes of one run per kernel class, counted per peeling
    round. decide reads an alive vertex's list entry (not in the first
    step, whose list is the identity), weight and row offsets and writes it
    to one list (32 B, 28 B in the first step), plus the round of a removed
    vertex (4 B); update writes every survivor's new weight from its list
    entry and row offsets (28 B, FD 36 B with the vertex weight); the
    incidences it reads depend on the path (a binary search per survivor,
    or a pass over the survivors' rows) and are not counted; reduce reads
    list entry, weight and vertex weight (FD) of every survivor (12 or 20
    B). A trimming step of local trimming is not in the rounds record."""
    alive_before = int(sum(sizes[:-1]))
    survivors = int(sum(sizes[1:]))
    return dict(decide=32.0 * alive_before - 4.0 * int(sizes[0]) + 4.0 * n,
                update=(36.0 if metric == "FD" else 28.0) * survivors,
                reduce=(20.0 if metric == "FD" else 12.0) * survivors)


def copy_probe(mb: int):
    """Three plain device copies of `mb` MiB: the reference dispatch that
    scales the FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    x = torch.empty(mb << 20, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()


def peel_bench(args):
    """Parallel peeling on a peeling input: every metric and mode timed over
    full runs; value and roofline come from the first metric and mode."""
    import torch
    import paper_2504_09311_amd as K
    from synth import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    inp = W.peel_input(args.workload, scale=args.scale)
    n, src, dst = inp["n"], inp["src"], inp["dst"]
    m = int(src.shape[0])
    log("peeling input", args.workload, n, "vertices", m, "edges")
    per = {}
    roof = None
    metrics = [x for x in args.peel_metrics.split(",") if x]
    assert metrics and set(metrics) <= {"DG", "DW", "FD"}, args.peel_metrics
    modes = [x for x in args.peel_modes.split(",") if x]
    assert modes and set(modes) <= {"plain", "gpo", "lpo"}, args.peel_modes
    for metric in metrics:
        t0 = time.perf_counter()
        G = K.PeelGraph(n, src, dst, metric, edge_w=inp["edge_w"], vertex_w=inp["vertex_w"])
        load_s = time.perf_counter() - t0
        per_mode = {}
        for mode in modes:
            lead = metric == metrics[0] and mode == modes[0]
            # the peel rounds stay in HBM in the timed runs (inputs and outputs
            # resident); one more run returns them to host memory
            for _ in range(max(1, args.warmup)):
                G.peel(2, 1, 10, rounds=False, mode=mode)
            # per-class times from one untimed run with events on every class
            _, sizes_p, _, smp = G.peel(2, 1, 10, profile=True, rounds=False, mode=mode)
            bytes_ = peel_bytes(metric, n, sizes_p, smp)
            kern = {k: dict(launches=int(smp[k + "_launches"]), total_ms=round(smp[k + "_ms"], 4),
                            avg_us=round(smp[k + "_ms"] * 1e3 / max(1, smp[k + "_launches"]), 3)) for k in bytes_}
            # the roofline kernel: k_decide, which runs once per step over
            # the whole alive set and is, with the pull reset's binary
            # searches, the largest single kernel of a run (update is a class
            # of four launches, of which the paths not taken return at once,
            # so its event time holds their launch gaps)
            dom = "decide"
            # timed runs; for the lead configuration the dominant class is
            # bracketed by events (read after each run) for the roofline
            dom_ms, dom_launches = 0.0, 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                _, sizes, fs, sm = G.peel(2, 1, 10, rounds=False, mode=mode, profile=[dom] if lead else False)
                if lead:
                    dom_ms += sm[dom + "_ms"]
                    dom_launches += int(sm[dom + "_launches"])
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / args.steps
            t0 = time.perf_counter()
            G.peel(2, 1, 10, mode=mode)
            wall_host = time.perf_counter() - t0
            per_mode[mode] = dict(seconds=round(wall, 5), edges_per_s=round(m / wall, 1),
                                  seconds_host_output=round(wall_host, 5), rounds=int(sm["rounds"]),
                                  trims=int(sm["trims"]), best=int(sm["best"]), best_size=int(sm["best_size"]),
                                  best_f=int(sm["best_f"]), kernels=kern)
            if lead and dom_launches:
                per_launch = bytes_[dom] / max(1, kern[dom]["launches"])
                avg_s = dom_ms / 1e3 / dom_launches
                roof = dict(kernel=dom, bound="hbm", achieved=round(per_launch / avg_s / 1e9, 2), peak=HBM_PEAK_GBS,
                            unit="GB/s", frac=round(per_launch / avg_s / 1e9 / HBM_PEAK_GBS, 4),
                            traffic=measured_traffic("peel_" + dom, args.workload),
                            bytes_per_launch=int(per_launch), avg_launch_us=round(avg_s * 1e6, 3),
                            launches=dom_launches)
            log(metric, mode, per_mode[mode])
        G.close()
        per[metric] = dict(load_s=round(load_s, 3), **per_mode)
    if args.copy_probe_mb:
        copy_probe(args.copy_probe_mb)
    cpu = None
    if args.cpu_budget > 0 and metrics[0] == "DG":
        import oracle
        # the oracle recomputes every sum in every round: the whole input up
        # to 2^29 edges (R-MAT 2^24, 263 M edges: ~20 s on one core), else the
        # same recipe at 2^20 vertices
        sample = inp if m <= (1 << 29) else W.peel_input("peel_rmat20")
        c, a = oracle.metric_weights("DG", sample["src"], sample["dst"], sample["n"])
        t0 = time.perf_counter()
        oracle.peel(sample["n"], sample["src"], sample["dst"], c, a, 2, 1, 10, cap=4096)
        dt = time.perf_counter() - t0
        cpu = dict(value=round(sample["src"].shape[0] / dt, 1), unit="edges/s", cores=1, kind="oracle",
                   sample=f"DG peeling of {sample['name']} ({sample['n']} vertices, {sample['src'].shape[0]} "
                          f"edges), one full run in {dt:.1f} s")
    lead = metrics[0]
    out = {
        "metric": PEEL_METRIC, "value": per[lead][modes[0]]["edges_per_s"], "unit": "edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(per[lead][modes[0]]["seconds"] * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": dict(workload=args.workload, n=n, m=m, eps="1/10", k=2,
                       metric=lead + (" (%s alongside)" % ", ".join(metrics[1:]) if metrics[1:] else ""),
                       mode=modes[0] + (" (%s alongside)" % ", ".join(modes[1:]) if modes[1:] else "")),
        "per_metric": per, "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat24_hier")
    ap.add_argument("--scale", type=int, default=None)
    ap.add_argument("--queries", type=int, default=None)
    ap.add_argument("--tile-words", type=int, default=0)
    ap.add_argument("--direction", type=int, default=0)
    ap.add_argument("--alpha", type=float, default=0.0)
    ap.add_argument("--graph", type=int, default=0, help="replay a captured hipGraph per batch shape")
    ap.add_argument("--graph-check", type=int, default=20,
                    help="steps timed without events with direct launches and with graph replay (0 = skip)")
    ap.add_argument("--fused-pull", type=int, default=0,
                    help="pulled levels finalize inside the pull: 0 the library's choice, 1 always, -1 never")
    ap.add_argument("--early-stop", type=int, default=0,
                    help="top-k early termination: 1 on, 0 or -1 off (the library's default)")
    ap.add_argument("--seed-table", type=int, default=0,
                    help="vertex seeding from a per-batch type-row table: 0 the library's choice, 1 always, -1 never")
    ap.add_argument("--pipeline", type=int, default=1,
                    help="1: submit batch i+1 before collecting batch i (host work overlaps the device)")
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel events")
    ap.add_argument("--plain", type=int, default=-1,
                    help="queries timed through the plain path (-1: all of the batch, 0: skip)")
    ap.add_argument("--autotune", type=int, default=0,
                    help="1: run the library's autotuner on the batch first and time with its choice")
    ap.add_argument("--cpu-budget", type=float, default=20.0,
                    help="seconds of single-thread oracle time (0 = skip the CPU baseline)")
    ap.add_argument("--cpu-workers", type=int, default=16, help="oracle threads of the all-cores leg")
    ap.add_argument("--copy-probe-mb", type=int, default=0, help="also run a plain copy of this size")
    ap.add_argument("--peel-metrics", default="DG,DW,FD",
                    help="peeling inputs: metrics to run (the first gives value and roofline)")
    ap.add_argument("--peel-modes", default="plain,gpo,lpo",
                    help="peeling inputs: Algorithm 2 (plain), with the global threshold (gpo) and with local "
                         "trimming (lpo); the first gives value and roofline")
    ap.add_argument("--serve", action="store_true", help="measure the serving loop instead of batches")
    ap.add_argument("--serve-sat", type=int, default=1024, help="queries for the saturation run")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="length of each Poisson run")
    ap.add_argument("--serve-words", type=int, default=0, help="server word slots (0 = memory budget)")
    args = ap.parse_args()

    if args.workload.startswith("peel_"):
        if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
            print("bench.py measures one GPU only", file=sys.stderr)
            sys.exit(2)
        peel_bench(args)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(queries would shard across GPUs with a replicated graph; not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2504_09311_amd as K

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    log("generating workload", args.workload)
    g, qs, desc = make_workload(args.workload, args.scale, args.queries)
    log("graph", g.n, "vertices", g.m, "edges;", len(qs), "queries")
    t0 = time.perf_counter()
    G = K.Graph.from_synth(g)
    load_s = time.perf_counter() - t0
    G.set_options(direction=args.direction, alpha=args.alpha, tile_words=args.tile_words, use_graph=args.graph,
                  count_te=1, fused_pull=args.fused_pull, early_stop=args.early_stop, seed_table=args.seed_table)
    log("graph loaded in %.2f s" % load_s)
    tuned = None
    if args.autotune:
        t0 = time.perf_counter()
        best, rep = G.autotune(qs, reps=3)
        tuned = dict(options=best, report=rep, seconds=round(time.perf_counter() - t0, 2))
        log("autotuned:", tuned)

    def set_count_te(on: int, use_graph=None):
        o = G.get_options()
        if args.autotune:
            G.set_options(direction=o.direction, alpha=o.alpha, tile_words=o.tile_words,
                          use_graph=o.use_graph if use_graph is None else use_graph, share_lanes=o.share_lanes,
                          count_te=on, seed_mode=o.seed_mode, fused_pull=o.fused_pull, early_stop=o.early_stop,
                          seed_table=o.seed_table)
        else:
            G.set_options(direction=args.direction, alpha=args.alpha, tile_words=args.tile_words,
                          use_graph=args.graph if use_graph is None else use_graph, count_te=on,
                          fused_pull=args.fused_pull, early_stop=args.early_stop, seed_table=args.seed_table)

    set_count_te(1)

    if args.serve or args.workload == "rmat26_serve":
        out = serve_bench(G, K, g, qs, args)
        line = {
            "metric": METRIC, "value": out["poisson"][-1]["qps"], "unit": "queries/s", "n_gpus": 1,
            "steps": out["poisson"][-1]["steps"], "warmup": 64, "ms_per_step": None, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": dict(workload=args.workload, path="served", n=g.n, m=g.m, **desc),
            "serving": out, "load_s": round(load_s, 3),
        }
        print(json.dumps(line), flush=True)
        G.close()
        return

    # ---- batched path: warmup, then K timed steps. The scanned-edge count te
    # (the GTEPS numerator) is a statistic, not part of the answers: it is
    # taken from a counted warm-up step and the timed steps do not count it.
    te_step = 0
    batch_answers = None
    for i in range(max(1, args.warmup)):
        r = G.search_batch_flat(qs)
        if i == 0:
            te_step = int(r["te"].sum())
            batch_answers = r
    set_count_te(0)
    torch.cuda.synchronize()

    def run_steps(nsteps):
        step_ms, batch_ms = [], []
        t_start = time.perf_counter()
        if args.pipeline:
            # batch i + 1 is planned and enqueued while batch i runs on the device
            t, t_sub = G.search_batch_submit(qs), time.perf_counter()
            last = t_start
            for i in range(nsteps):
                nxt, nxt_sub = (G.search_batch_submit(qs), time.perf_counter()) if i + 1 < nsteps else (None, 0.0)
                G.search_batch_collect(t)
                now = time.perf_counter()
                step_ms.append((now - last) * 1e3)
                batch_ms.append((now - t_sub) * 1e3)
                last = now
                t, t_sub = nxt, nxt_sub
        else:
            for i in range(nsteps):
                a = time.perf_counter()
                G.search_batch_flat(qs)
                step_ms.append((time.perf_counter() - a) * 1e3)
                batch_ms.append(step_ms[-1])
        return time.perf_counter() - t_start, step_ms, batch_ms

    # ---- per-class kernel times from an untimed profiled run (events around
    # every launch); the timed steps then bracket only the class whose
    # roofline is reported, so the events cost the timed run almost nothing
    kernels, dom, calib_steps = {}, None, 0
    if not args.no_profile:
        calib_steps = min(args.steps, 10)
        G.profile_classes(None)
        G.profile_enable(True)
        G.profile_reset()
        run_steps(calib_steps)
        G.profile_enable(False)
        prof_all = G.profile_read()
        kernels = {k: dict(launches=v[0], total_ms=round(v[1], 4),
                           avg_us=round(v[1] * 1e3 / v[0], 3) if v[0] else 0.0)
                   for k, v in prof_all.items() if v[0]}
        st_all = G.last_batch_stats().as_dict()
        fused = bool(G.last_batch_stats().as_dict()["fused_pull"])
        modeled_all = {k: byte_model(st_all, g.n, k, kernels.get(k, {}).get("launches", 0) / calib_steps, fused)
                       for k in ("pull", "push", "finalize", "score")}
        cand = [k for k in modeled_all if k in kernels and modeled_all[k] > 0]
        if cand:
            dom = max(cand, key=lambda k: kernels[k]["total_ms"])
            G.profile_classes([dom])
            G.profile_enable(True)
            G.profile_reset()
    te_total = te_step * args.steps
    torch.cuda.synchronize()
    wall, step_ms, batch_ms = run_steps(args.steps)
    torch.cuda.synchronize()
    G.profile_enable(False)
    G.profile_classes(None)
    prof = G.profile_read()
    st = G.last_batch_stats().as_dict()
    log("timed %d steps in %.3f s" % (args.steps, wall))

    qps = len(qs) * args.steps / wall
    gteps = te_total / wall / 1e9
    ms_per_step = wall * 1e3 / args.steps

    # ---- roofline of the dominant kernel: HIP events on the library's
    # stream around its launches in the timed steps
    roofline = None
    if dom and prof.get(dom, (0, 0.0))[0]:
        launches, total_ms = prof[dom]
        modeled_dom = byte_model(st, g.n, dom, launches / args.steps, bool(st["fused_pull"]))
        if modeled_dom > 0:
            per_launch_bytes = modeled_dom * args.steps / launches
            avg_s = total_ms / 1e3 / launches
            achieved = per_launch_bytes / avg_s / 1e9
            kname = None
            if dom == "pull":
                kname = ("k_pull_fin<%d>" if st["fused_pull"] else "k_pull<%d>") % st["tile_words"]
            traffic = measured_traffic(dom, args.workload, kname)
            roofline = dict(kernel=dom, bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                            frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                            bytes_per_launch=int(per_launch_bytes), avg_launch_us=round(avg_s * 1e6, 3),
                            launches=launches)
            if traffic:
                roofline["traffic_gbs"] = round(traffic / avg_s / 1e9, 2)
                roofline["traffic_frac"] = round(traffic / avg_s / 1e9 / HBM_PEAK_GBS, 4)
                roofline["waste_ratio"] = round(traffic / per_launch_bytes, 3)

    # ---- launch modes without events: direct launches against one captured
    # hipGraph per pass shape replayed for every step (the timed steps above
    # bracket the roofline kernel with events, which needs direct launches)
    launch_modes = None
    if args.graph_check > 0:
        launch_modes = {}
        for mode in (0, 1):
            set_count_te(0, use_graph=mode)
            run_steps(2)
            torch.cuda.synchronize()
            w_mode, _, _ = run_steps(args.graph_check)
            torch.cuda.synchronize()
            launch_modes["graph_qps" if mode else "direct_qps"] = round(len(qs) * args.graph_check / w_mode, 2)
        info = G.info()
        launch_modes.update(steps=args.graph_check, graph_captures=int(info.graph_captures),
                            graph_replays=int(info.graph_replays))
        set_count_te(0)

    # ---- plain path: one query per call, same queries
    plain = None
    if args.plain != 0:
        pq = qs if args.plain < 0 else qs[: args.plain]
        for q in pq[:3]:
            G.keyword_search(q.kw, q.d_max, q.k)
        lat, answers = [], []
        t0 = time.perf_counter()
        for q in pq:
            a = time.perf_counter()
            answers.append(G.keyword_search(q.kw, q.d_max, q.k))
            lat.append((time.perf_counter() - a) * 1e3)
        pw = time.perf_counter() - t0
        # equal results: the plain answers of these queries against the
        # batched answers of the warm-up step (same queries, same order)
        plain = dict(queries=len(pq), qps=round(len(pq) / pw, 2), p50_ms=round(float(np.percentile(lat, 50)), 4),
                     p99_ms=round(float(np.percentile(lat, 99)), 4),
                     equal_to_batched=bool(same_answers(batch_answers, answers)))

    if args.copy_probe_mb:
        copy_probe(args.copy_probe_mb)

    cpu = None
    if args.cpu_budget > 0:
        log("timing the CPU oracle (one pinned thread, then one query per core)")
        cpu = cpu_baseline(g, qs, args.cpu_budget, args.cpu_workers)

    out = {
        "metric": METRIC,
        "value": round(qps, 2),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": dict(workload=args.workload, queries_per_step=len(qs), path="batched", n=g.n, m=g.m, **desc),
        "gteps": round(gteps, 3),
        "step_latency_ms": dict(p50=round(float(np.percentile(step_ms, 50)), 4),
                                p99=round(float(np.percentile(step_ms, 99)), 4)),
        "batch_latency_ms": dict(p50=round(float(np.percentile(batch_ms, 50)), 4),
                                 p99=round(float(np.percentile(batch_ms, 99)), 4)),
        "pipelined": bool(args.pipeline),
        "autotuned": tuned,
        "launch_modes": launch_modes,
        "plain": plain,
        "speedup_vs_plain": round(qps / plain["qps"], 2) if plain else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "kernels_from": (f"HIP events around every launch in an untimed profiled run of {calib_steps} steps; "
                         f"the timed steps bracket only the roofline kernel ({dom})") if kernels else None,
        "batch": st,
        "load_s": round(load_s, 3),
    }
    print(json.dumps(out), flush=True)
    G.close()


if __name__ == "__main__":
    main()
