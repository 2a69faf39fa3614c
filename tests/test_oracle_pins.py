"""Pins for the CPU oracle: checks against things other than itself.

* hand-derived worked examples (tests/golden/worked_examples.json);
* an independent brute force (all-pairs forward BFS, top-down type walk)
  on hundreds of random tiny graphs with loops, multi-edges, duplicate
  keywords, d_max 0..6 and k from 0 past n;
* SciPy's unweighted shortest paths through a super-source;
* the BFS certificate (a linear-time characterisation of truncated BFS
  distances) on larger R-MAT graphs, plus a check that the certificate
  rejects perturbed distances;
* special cases with closed forms (d_max = 0, single keyword, path,
  complete digraph, no edges);
* validity of answer edges independent of the tie-break.
"""
import json
import os

import numpy as np
import pytest

import brute
import oracle
from synth import tiny, workloads, gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def _as_dict(res):
    return dict(kw=res.kw, roots=res.roots.tolist(), scores=res.scores.tolist(),
                kw_dist=res.kw_dist.tolist(),
                edges=[[list(e) for e in res.edges_of(i)] for i in range(len(res.roots))],
                te=res.te)


def test_golden_worked_examples():
    spec = json.load(open(GOLDEN))
    for case in spec["cases"]:
        g = tiny.from_edges(case["n"], case["edges"], case["labels"], case["n_labels"],
                            case["type_parent"], case["name"])
        o = oracle.Oracle(g)
        for q in case["queries"]:
            got = _as_dict(o.search(q["kw"], q["d_max"], q["k"]))
            assert got == q["expect"], (case["name"], q["kw"])


@pytest.mark.parametrize("block", range(6))
def test_brute_force_tiny(block):
    for seed in range(block * 60, block * 60 + 60):
        g = tiny.random_graph(seed)
        o = oracle.Oracle(g)
        D = brute.all_pairs(g)
        for q in tiny.random_queries(g, seed):
            want = brute.search(g, q.kw, q.d_max, q.k, D)
            got = _as_dict(o.search(q.kw, q.d_max, q.k))
            want["edges"] = [[list(e) for e in es] for es in want["edges"]]
            assert got == want, (seed, q)


def test_scipy_distances():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    for g in (workloads.chunglu10k(), workloads.rmat_flat(13)):
        o = oracle.Oracle(g)
        n = g.n
        src = np.repeat(np.arange(n), np.diff(g.row_ptr))
        # transpose plus a super-source s = n with an edge to every keyword vertex
        qs = gen.queries(6, g.n_labels, 1.0, 1, 1, [1, 2, 3, 4], 1, 0x5EED0101, 99)
        for q in qs:
            t = q.kw[0]
            seeds = np.flatnonzero(o.keyword_set(t))
            rows = np.concatenate([g.col, np.full(seeds.shape[0], n)])
            cols = np.concatenate([src, seeds])
            A = csr_matrix((np.ones(rows.shape[0]), (rows, cols)), shape=(n + 1, n + 1))
            d = shortest_path(A, unweighted=True, indices=n, directed=True)
            want = np.where(d - 1 <= q.d_max, d - 1, 255)
            want = np.where(np.isinf(d), 255, want).astype(np.uint8)[:n]
            got, _ = o.distances(t, q.d_max)
            assert np.array_equal(got, want), (g.name, t, q.d_max)


def test_certificate_rmat_and_rejects_perturbation():
    g = workloads.rmat_flat(15)
    o = oracle.Oracle(g)
    rng = np.random.default_rng(7)
    for t in rng.integers(0, g.n_labels, 5).tolist() + [int(g.lab[0])]:
        for d_max in (0, 1, 3, 5):
            dist, _ = o.distances(t, d_max)
            S = o.keyword_set(t)
            assert brute.certificate(g.row_ptr, g.col, S, dist, d_max) == []
    # the checker itself must notice small corruptions
    t = int(g.lab[0])
    dist, _ = o.distances(t, 3)
    S = o.keyword_set(t)
    finite = np.flatnonzero((dist > 0) & (dist < 255))
    for v in finite[:20]:
        for delta in (-1, 1):
            bad = dist.copy()
            bad[v] = int(bad[v]) + delta
            assert brute.certificate(g.row_ptr, g.col, S, bad, 3) != []
    inf = np.flatnonzero(dist == 255)
    bad = dist.copy()
    bad[inf[0]] = 3
    assert brute.certificate(g.row_ptr, g.col, S, bad, 3) != []


def test_dmax_zero_is_intersection():
    g = workloads.chunglu10k()
    o = oracle.Oracle(g)
    lab_sets = [set(g.lab[g.lab_ptr[v]:g.lab_ptr[v + 1]].tolist()) for v in range(g.n)]
    for q in workloads.chunglu10k_queries(20):
        res = o.search(q.kw, 0, 10_000)
        want = sorted(v for v in range(g.n) if set(q.kw) <= lab_sets[v])
        assert res.roots.tolist() == want
        assert not res.scores.any() and res.edge_ptr[-1] == 0 and res.te == 0


def test_single_keyword_is_bfs_ball():
    g = workloads.rmat_flat(12)
    o = oracle.Oracle(g)
    t = int(np.bincount(g.lab).argmax())
    dist, te = o.distances(t, 2)
    res = o.search([t], 2, g.n + 5)
    ball = np.flatnonzero(dist <= 2)
    order = sorted(ball.tolist(), key=lambda r: (int(dist[r]), r))
    assert res.roots.tolist() == order
    assert res.scores.tolist() == [int(dist[r]) for r in order]
    assert res.te == te


def test_path_graph_closed_form():
    for n in (1, 2, 7, 40):
        g = tiny.path_graph(n)
        o = oracle.Oracle(g)
        for d_max in (0, 1, 3, 50):
            dist, te = o.distances(0, d_max)
            want = [n - 1 - r if n - 1 - r <= d_max else 255 for r in range(n)]
            assert dist.tolist() == want
            assert te == min(d_max, n - 1)   # every expanded vertex but 0 has in-degree 1
            res = o.search([0], d_max, n)
            assert res.roots.tolist() == list(range(n - 1, n - 2 - min(d_max, n - 1), -1))
            for i, r in enumerate(res.roots.tolist()):
                assert res.edges_of(i) == [(x, x + 1) for x in range(r, n - 1)]


def test_complete_digraph():
    g = tiny.complete_digraph(9, {2, 5})
    o = oracle.Oracle(g)
    dist, te = o.distances(0, 3)
    assert dist.tolist() == [0 if v in (2, 5) else 1 for v in range(9)]
    res = o.search([0], 3, 20)
    assert res.roots.tolist() == [2, 5, 0, 1, 3, 4, 6, 7, 8]
    assert res.edges_of(2) == [(0, 2)]      # min-id successor at distance 0


def test_no_edges():
    labels = [[0, 1], [1], [], [0, 1, 2], [0]]
    g = tiny.no_edges(5, labels, 3)
    o = oracle.Oracle(g)
    for d_max in (0, 4):
        res = o.search([1, 0], d_max, 10)
        assert res.roots.tolist() == [0, 3]
        assert res.scores.tolist() == [0, 0] and res.te == 0


def test_answer_edges_valid_on_rmat():
    g = workloads.rmat_flat(13)
    o = oracle.Oracle(g)
    edges = set(zip(np.repeat(np.arange(g.n), np.diff(g.row_ptr)).tolist(), g.col.tolist()))
    for q in workloads.rmat_flat_queries(12, 2, 5, [2, 3, 4], 20, cfg=2, qcfg=3):
        res = o.search(q.kw, q.d_max, q.k)
        dists = {t: o.distances(t, q.d_max)[0] for t in res.kw}
        sets = {t: o.keyword_set(t) for t in res.kw}
        for i, r in enumerate(res.roots.tolist()):
            es = res.edges_of(i)
            assert all(e in edges for e in es)
            adj = {}
            for x, y in es:
                adj.setdefault(x, []).append(y)
            for j, t in enumerate(res.kw):
                d = int(res.kw_dist[i, j])
                assert d == dists[t][r]
                # a path of exactly d answer edges from r into S_t
                level = {r}
                for _ in range(d):
                    level = {y for x in level for y in adj.get(x, []) if dists[t][y] == dists[t][x] - 1}
                assert any(sets[t][v] for v in level)


def test_rejects_bad_arguments():
    g = workloads.chunglu10k()
    o = oracle.Oracle(g)
    with pytest.raises(ValueError):
        o.search([10_000], 3, 10)
    with pytest.raises(ValueError):
        o.search([1], 255, 10)
    with pytest.raises(ValueError):
        o.search([1], -1, 10)
