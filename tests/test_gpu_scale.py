"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times.

* 2^24-vertex R-MAT with the type tree (256M sampled edges), 512 queries of
  2-6 keywords in one batch: 65 queries against the oracle (13 per keyword
  count 2..6, covering every keyword depth 2..6 of the type tree), the
  answer paths of all 512 queries checked without the oracle, and the BFS
  certificate on exported per-keyword distances.
* 2^20-vertex R-MAT, the benchmark's 100 four-keyword queries through the
  tuned batched path: every query against the oracle.
* 2^26-vertex R-MAT (1B sampled edges) through the server: sampled queries
  against the oracle and the certificate.
"""
import sys
import time

import numpy as np
import pytest

import brute
import oracle
from parity import assert_all_same, assert_same, oracle_results
from synth import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def K():
    import paper_2504_09311_amd as K
    K.load_library()
    return K


def edge_set_check(g, res):
    """Every answer edge is a graph edge (rows are sorted, so binary search)."""
    rp, col = g.row_ptr, g.col
    for i in range(len(res.roots)):
        for x, y in res.edges_of(i):
            a, b = int(rp[x]), int(rp[x + 1])
            j = a + int(np.searchsorted(col[a:b], y))
            assert j < b and col[j] == y, (x, y)


def type_depth(parent, t):
    d = 0
    while parent[t] >= 0:
        t = int(parent[t])
        d += 1
    return d


def matched_types(g, v, memo):
    """The keywords vertex v matches: its labels and their ancestor types."""
    got = memo.get(v)
    if got is None:
        got = set()
        for lab in g.lab[g.lab_ptr[v]:g.lab_ptr[v + 1]].tolist():
            while lab >= 0 and lab not in got:
                got.add(lab)
                lab = int(g.type_parent[lab]) if g.type_parent is not None else -1
        memo[v] = got
    return got


def answer_paths_check(g, res, d_max, ctx, memo=None):
    """Without the oracle: every answer edge is a graph edge; per (root,
    keyword) a distance of 0 means the root carries the keyword; otherwise
    the root's answer edges hold a path of exactly that many edges to a
    vertex carrying it and none shorter (a shorter one would be a shorter
    graph path, so the reported distance would be wrong); no more edges than
    the distances add up to; scores are the distance sums, in (score, id)
    order, all within d_max."""
    memo = {} if memo is None else memo
    edge_set_check(g, res)
    assert np.array_equal(res.scores, res.kw_dist.astype(np.int64).sum(axis=1)), ctx
    keys = list(zip(res.scores.tolist(), res.roots.tolist()))
    assert keys == sorted(keys) and len(set(res.roots.tolist())) == len(keys), ctx
    for i, r in enumerate(res.roots.tolist()):
        ed = res.edges_of(i)
        dist = res.kw_dist[i].tolist()
        assert len(ed) <= sum(dist) and max(dist, default=0) <= d_max, (ctx, i)
        adj = {}
        for x, y in ed:
            adj.setdefault(x, []).append(y)
        # BFS inside the answer edges from the root
        level, seen, frontier = {r: 0}, {r}, [r]
        while frontier:
            nxt = []
            for x in frontier:
                for y in adj.get(x, ()):
                    if y not in seen:
                        seen.add(y)
                        level[y] = level[x] + 1
                        nxt.append(y)
            frontier = nxt
        for t, d in zip(res.kw, dist):
            best = min((lv for v, lv in level.items() if t in matched_types(g, v, memo)), default=None)
            assert best == d, (ctx, "root", r, "keyword", t, "dist", d, "answer-path length", best)


def stratified_sample(qs, parent, per_count=13):
    """Query indices: per keyword count 2..6, per_count queries spread over
    the batch, first making sure every keyword depth 2..6 appears."""
    picks = []
    for nk in range(2, 7):
        pool = [i for i, q in enumerate(qs) if len(set(q.kw)) == nk]
        chosen = []
        for depth in range(2, 7):
            for i in pool:
                if i not in chosen and any(type_depth(parent, t) == depth for t in qs[i].kw):
                    chosen.append(i)
                    break
        step = max(1, len(pool) // per_count)
        for i in pool[::step]:
            if len(chosen) >= per_count:
                break
            if i not in chosen:
                chosen.append(i)
        picks += sorted(chosen[:per_count])
    return picks


def test_rmat20_bench_queries_tuned(K):
    g, qs = workloads.rmat20_q4()
    o = oracle.Oracle(g)
    want = oracle_results(o, qs)
    G = K.Graph.from_synth(g)
    say("rmat20 bench queries, default options")
    assert_all_same(G.search_batch(qs), want, "rmat20 q4 default")
    best, rep = G.autotune(qs, reps=1, budget_ms=3000)
    say("tuned", best, rep)
    assert_all_same(G.search_batch(qs), want, "rmat20 q4 tuned")
    G.close()


def test_rmat24_hier_full_scale(K):
    t0 = time.time()
    g, qs = workloads.rmat24_hier(24, 512)
    say("rmat24 hier generated", g.n, g.m, "in %.1f s" % (time.time() - t0))
    G = K.Graph.from_synth(g)
    say("loaded on the device in %.1f s" % (time.time() - t0))
    res = G.search_batch(qs)
    say("batch of 512 done in %.1f s" % (time.time() - t0))
    memo = {}
    for i, (q, r) in enumerate(zip(qs, res)):
        answer_paths_check(g, r, q.d_max, f"rmat24 query {i}", memo)
    say("answer paths of all 512 queries checked in %.1f s" % (time.time() - t0))
    o = oracle.Oracle(g)
    sample = stratified_sample(qs, g.type_parent)
    counts = sorted({len(set(qs[i].kw)) for i in sample})
    depths = sorted({type_depth(g.type_parent, t) for i in sample for t in qs[i].kw})
    say("oracle sample: %d queries, keyword counts %s, keyword depths %s" % (len(sample), counts, depths))
    assert len(sample) >= 64 and counts == [2, 3, 4, 5, 6] and depths == [2, 3, 4, 5, 6]
    want = oracle_results(o, [qs[i] for i in sample])
    say("oracle sample done in %.1f s" % (time.time() - t0))
    for i, w in zip(sample, want):
        assert_same(res[i], w, f"rmat24 query {i}")
    for t in qs[0].kw[:2]:
        d = G.debug_distances(t, 3)
        assert brute.certificate(g.row_ptr, g.col, o.keyword_set(t), d, 3) == []
    say("certificates done in %.1f s" % (time.time() - t0))
    G.close()


def test_rmat26_served_full_scale(K):
    t0 = time.time()
    g, qs = workloads.rmat26_serve(26, 256)
    say("rmat26 generated", g.n, g.m, "in %.1f s" % (time.time() - t0))
    G = K.Graph.from_synth(g)
    say("loaded in %.1f s" % (time.time() - t0))
    S = K.Server(G, max_dmax=4, max_words=16)
    ts = [S.submit(q.kw, q.d_max, q.k) for q in qs]
    got = [S.wait(t, 600.0) for t in ts]
    say("served 256 in %.1f s" % (time.time() - t0), S.stats())
    S.close()
    o = oracle.Oracle(g)
    sample = [0, 100, 255]
    want = oracle_results(o, [qs[i] for i in sample], workers=3)
    say("oracle sample in %.1f s" % (time.time() - t0))
    for i, w in zip(sample, want):
        assert_same(got[i], w, f"rmat26 served query {i}")
    t = qs[0].kw[0]
    d = G.debug_distances(t, 4)
    assert brute.certificate(g.row_ptr, g.col, o.keyword_set(t), d, 4) == []
    say("done in %.1f s" % (time.time() - t0))
    G.close()
