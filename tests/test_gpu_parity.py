"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bit-exact on every field (roots, scores, per-keyword distances, answer
edges, scanned-edge counts). Covers the plain one-query path and the
batched path, every tile width, forced push / forced pull / automatic
direction, lane sharing on and off, hand-derived worked examples,
hundreds of random tiny graphs with the awkward cases, the small
Chung-Lu workload, the 2^20-vertex R-MAT workloads (plain query set and
the 256-query batch), the type-tree workload at reduced scale, and the
per-keyword distance export checked against the BFS certificate.
"""
import json
import os
import sys

import numpy as np
import pytest

import brute
import oracle
from parity import assert_all_same, assert_same, oracle_results
from synth import tiny, workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def K():
    import paper_2504_09311_amd as K
    K.load_library()
    return K


def test_golden_worked_examples(K):
    spec = json.load(open(GOLDEN))
    for case in spec["cases"]:
        g = tiny.from_edges(case["n"], case["edges"], case["labels"], case["n_labels"],
                            case["type_parent"], case["name"])
        say("golden", case["name"])
        G = K.Graph.from_synth(g)
        for q in case["queries"]:
            r = G.keyword_search(q["kw"], q["d_max"], q["k"])
            e = q["expect"]
            assert r.kw == e["kw"] and r.roots.tolist() == e["roots"]
            assert r.scores.tolist() == e["scores"] and r.kw_dist.tolist() == e["kw_dist"]
            assert [[list(x) for x in r.edges_of(i)] for i in range(len(r.roots))] == e["edges"]
            assert r.te == e["te"]
        G.close()


@pytest.mark.parametrize("block", range(4))
def test_tiny_random(K, block):
    for seed in range(block * 50, block * 50 + 50):
        g = tiny.random_graph(seed)
        qs = tiny.random_queries(g, seed, 6)
        o = oracle.Oracle(g)
        want = [o.search(q.kw, q.d_max, q.k) for q in qs]
        say("tiny", seed, g.n, g.m, [(q.kw, q.d_max, q.k) for q in qs])
        G = K.Graph.from_synth(g)
        for i, q in enumerate(qs):
            assert_same(G.keyword_search(q.kw, q.d_max, q.k), want[i], f"tiny {seed} plain {i}")
        for direction in (0, 1, 2):
            fused = 1 if (seed + direction) % 2 else -1
            table = 1 if (seed // 2 + direction) % 2 else -1
            G.set_options(direction=direction, tile_words=[1, 2, 4, 8, 16][seed % 5],
                          share_lanes=1 if seed % 2 else -1, seed_mode=(seed + direction) % 3, fused_pull=fused,
                          seed_table=table)
            assert_all_same(G.search_batch(qs), want, f"tiny {seed} batch dir {direction} fused {fused} table {table}")
        assert_all_same(G.search_batch_each(qs), want, f"tiny {seed} batch (per-query results)")
        G.close()


def test_tiny_batch_of_many_words(K):
    # one small graph, 300 queries: several words, tiles and shared lanes
    g = tiny.random_graph(7, n_max=48)
    while g.m == 0:
        g = tiny.random_graph(g.n + 1000, n_max=48)
    qs = []
    for s in range(75):
        qs += tiny.random_queries(g, 1000 + s, 4)
    o = oracle.Oracle(g)
    want = [o.search(q.kw, q.d_max, q.k) for q in qs]
    G = K.Graph.from_synth(g)
    for tw in (1, 4, 16):
        for share in (1, -1):
            for sm, table in ((1, 0), (2, -1), (2, 1)):
                say("many words", tw, share, sm, table)
                G.set_options(tile_words=tw, share_lanes=share, seed_mode=sm, fused_pull=share, seed_table=table)
                assert_all_same(G.search_batch(qs), want, f"many tw {tw} share {share} seed {sm} table {table}")
                assert G.last_batch_stats().seed_table == (1 if table == 1 else 0)
    G.close()


def test_special_graphs(K):
    for g, kw in [(tiny.path_graph(40), [0]), (tiny.complete_digraph(9, {2, 5}), [0]),
                  (tiny.no_edges(5, [[0, 1], [1], [], [0, 1, 2], [0]], 3), [1, 0])]:
        o = oracle.Oracle(g)
        G = K.Graph.from_synth(g)
        for d_max in (0, 1, 3, 15):
            for k in (0, 1, 5, 100):
                say("special", g.name, d_max, k)
                assert_same(G.keyword_search(kw, d_max, k), o.search(kw, d_max, k), g.name)
        G.close()


@pytest.fixture(scope="module")
def chunglu(K):
    g = workloads.chunglu10k()
    return g, oracle.Oracle(g), K.Graph.from_synth(g)


def test_chunglu10k_plain_and_batch(K, chunglu):
    g, o, G = chunglu
    qs = workloads.chunglu10k_queries(101)
    want = oracle_results(o, qs)
    say("chunglu10k plain")
    for i, q in enumerate(qs):
        assert_same(G.keyword_search(q.kw, q.d_max, q.k), want[i], f"chunglu plain {i}")
    for direction in (0, 1, 2):
        say("chunglu10k batch", direction)
        G.set_options(direction=direction)
        assert_all_same(G.search_batch(qs), want, f"chunglu batch {direction}")
    G.set_options()


def test_chunglu10k_mixed_shapes(K, chunglu):
    g, o, G = chunglu
    from synth import gen
    qs = gen.queries(200, 500, 1.1, 1, 12, [0, 1, 2, 3, 4, 6], 25, 0x5EED0101, 42)
    want = oracle_results(o, qs)
    for tw in (1, 2, 8, 16):
        say("chunglu mixed", tw)
        G.set_options(tile_words=tw)
        assert_all_same(G.search_batch(qs), want, f"chunglu mixed tw {tw}")
    G.set_options()


def test_chunglu10k_large_batch(K, chunglu):
    # 2400 queries: the score step's query table no longer fits in LDS, so
    # the global-memory variant runs
    g, o, G = chunglu
    from synth import gen
    qs = gen.queries(2400, 500, 1.1, 1, 6, [1, 2, 3], 10, 0x5EED0101, 77)
    want = oracle_results(o, qs)
    say("chunglu large batch")
    assert_all_same(G.search_batch(qs), want, "chunglu 2400 queries")


def test_distances_export_certificate(K, chunglu):
    g, o, G = chunglu
    for t in (0, 1, 17, 250, 499):
        for d_max in (0, 2, 5):
            say("export", t, d_max)
            G.set_options(seed_mode=1 + (t + d_max) % 2)
            d = G.debug_distances(t, d_max)
            want, _ = o.distances(t, d_max)
            assert np.array_equal(d, want)
            assert brute.certificate(g.row_ptr, g.col, o.keyword_set(t), d, d_max) == []
    G.set_options()


@pytest.fixture(scope="module")
def rmat14(K):
    g = workloads.rmat_flat(14)
    return g, oracle.Oracle(g), K.Graph.from_synth(g)


def test_rmat14_options_grid(K, rmat14):
    g, o, G = rmat14
    qs = workloads.rmat_flat_queries(96, 2, 8, [2, 3, 4], 20, cfg=2, qcfg=3)
    want = oracle_results(o, qs)
    for tw in (1, 2, 4, 8, 16):
        for direction in (0, 1, 2):
            say("rmat14", tw, direction)
            G.set_options(direction=direction, tile_words=tw)
            assert_all_same(G.search_batch(qs), want, f"rmat14 tw {tw} dir {direction}")
        # pulled levels with the separate finalize pass
        G.set_options(direction=2, tile_words=tw, fused_pull=-1)
        assert_all_same(G.search_batch(qs), want, f"rmat14 tw {tw} pull, unfused")
    G.set_options(share_lanes=-1)
    assert_all_same(G.search_batch(qs), want, "rmat14 no sharing")
    for sm, table in ((1, 0), (2, -1), (2, 1)):
        G.set_options(seed_mode=sm, tile_words=4, seed_table=table)
        assert_all_same(G.search_batch(qs), want, f"rmat14 seed mode {sm} table {table}")
    G.set_options()
    for i in range(0, 96, 7):
        assert_same(G.keyword_search(qs[i].kw, qs[i].d_max, qs[i].k), want[i], f"rmat14 plain {i}")


def test_rmat14_hierarchy(K):
    g, leaves = workloads.rmat_hier(14, cfg=4)
    qs = workloads.rmat_hier_queries(g.type_parent, leaves, 64, cfg=4)
    o = oracle.Oracle(g)
    want = oracle_results(o, qs)
    G = K.Graph.from_synth(g)
    for direction in (0, 1, 2):
        for sm in (0, 1, 2):
            # the type-row table on for vertex seeding (every type's row walks its ancestors)
            table = 1 if (sm + direction) % 2 else -1
            say("rmat14 hier", direction, sm, table)
            G.set_options(direction=direction, seed_mode=sm, fused_pull=-1 if sm == 1 else 1, seed_table=table)
            assert_all_same(G.search_batch(qs), want, f"hier dir {direction} seed {sm} table {table}")
            if sm == 2:
                assert G.last_batch_stats().seed_table == (1 if table == 1 else 0)
    G.set_options()
    for i in range(0, 64, 9):
        assert_same(G.keyword_search(qs[i].kw, qs[i].d_max, qs[i].k), want[i], f"hier plain {i}")
    G.close()


def test_early_stop_is_exact(K, chunglu, rmat14):
    """Top-k early termination forced on: every root, score, keyword
    distance and answer edge equals the oracle's, for the plain path and for
    batches (fused and unfused pulls, graph replay); te is left out, since a
    query that stops early scans fewer edges. Queries do stop early."""
    stopped = 0
    cases = [("chunglu", chunglu[0], chunglu[1], chunglu[2], workloads.chunglu10k_queries(101)),
             ("rmat14", rmat14[0], rmat14[1], rmat14[2],
              workloads.rmat_flat_queries(96, 2, 8, [2, 3, 4], 20, cfg=2, qcfg=3))]
    gh, leaves = workloads.rmat_hier(14, cfg=4)
    cases.append(("rmat14 hier", gh, oracle.Oracle(gh), None, workloads.rmat_hier_queries(gh.type_parent, leaves,
                                                                                             64, cfg=4)))
    for name, g, o, G, qs in cases:
        own = G is None
        if own:
            G = K.Graph.from_synth(g)
        want = oracle_results(o, qs)
        for fused in (1, -1):
            for graph in (0, 1):
                say("early stop", name, fused, graph)
                G.set_options(early_stop=1, fused_pull=fused, use_graph=graph, count_te=0)
                assert_all_same(G.search_batch(qs), want, f"{name} early batch fused {fused} graph {graph}", te=False)
                stopped += G.last_batch_stats().early_stopped
        for i in range(0, len(qs), 5):
            G.set_options(early_stop=1, count_te=0)
            assert_same(G.keyword_search(qs[i].kw, qs[i].d_max, qs[i].k), want[i], f"{name} early plain {i}", te=False)
            stopped += G.last_batch_stats().early_stopped
        G.set_options()
        if own:
            G.close()
    say("queries stopped early:", stopped)
    assert stopped > 0


def test_early_stop_tiny(K):
    for seed in range(0, 200, 3):
        g = tiny.random_graph(seed)
        qs = tiny.random_queries(g, seed, 6)
        o = oracle.Oracle(g)
        want = [o.search(q.kw, q.d_max, q.k) for q in qs]
        G = K.Graph.from_synth(g)
        G.set_options(early_stop=1, count_te=0, tile_words=[1, 2, 4, 8, 16][seed % 5], fused_pull=1 - 2 * (seed % 2))
        assert_all_same(G.search_batch(qs), want, f"tiny {seed} early batch", te=False)
        for i, q in enumerate(qs):
            assert_same(G.keyword_search(q.kw, q.d_max, q.k), want[i], f"tiny {seed} early plain {i}", te=False)
        G.close()


@pytest.fixture(scope="module")
def rmat20(K):
    g, qs = workloads.rmat20_q4()
    say("rmat20 load", g.n, g.m)
    return g, qs, oracle.Oracle(g), K.Graph.from_synth(g)


def test_rmat20_q4_plain(K, rmat20):
    g, qs, o, G = rmat20
    sample = qs[:12]
    want = oracle_results(o, sample)
    for i, q in enumerate(sample):
        say("rmat20 plain", i)
        assert_same(G.keyword_search(q.kw, q.d_max, q.k), want[i], f"rmat20 plain {i}")
    say("rmat20 q4 batch")
    assert_all_same(G.search_batch(sample), want, "rmat20 q4 batch")


def test_rmat20_batch256(K, rmat20):
    g, _, o, G = rmat20
    qs = workloads.rmat_flat_queries(256, 2, 8, [2, 3, 4], 20, cfg=2, qcfg=3)
    want = oracle_results(o, qs)
    for direction, fused in ((0, 1), (2, 1), (2, -1)):
        say("rmat20 batch256", direction, fused)
        G.set_options(direction=direction, fused_pull=fused)
        assert_all_same(G.search_batch(qs), want, f"rmat20 batch256 dir {direction} fused {fused}")
    G.set_options()


def test_rmat20_export_certificate(K, rmat20):
    g, qs, o, G = rmat20
    for t in qs[0].kw[:2]:
        say("rmat20 export", t)
        d = G.debug_distances(t, 3)
        assert brute.certificate(g.row_ptr, g.col, o.keyword_set(t), d, 3) == []


def test_errors(K, chunglu):
    g, o, G = chunglu
    for bad in ([10_000], [-1]):
        with pytest.raises(K.KwsError) as e:
            G.keyword_search(bad, 3, 10)
        assert e.value.status == K.EINVAL
    with pytest.raises(K.KwsError):
        G.keyword_search([1], 16, 10)
    with pytest.raises(K.KwsError):
        G.keyword_search(list(range(65)), 2, 10)
    with pytest.raises(K.KwsError):
        G.keyword_search([1], 2, K.MAX_K + 1)
    # 64 distinct keywords is the limit and works
    r = G.keyword_search(list(range(64)), 1, 5)
    w = o.search(list(range(64)), 1, 5)
    assert_same(r, w, "64 keywords")


def test_unsorted_rows_and_multi_edges(K):
    # rows given in arbitrary order (with repeated edges) must give the same answers
    g = workloads.chunglu10k()
    rng = np.random.default_rng(5)
    col = g.col.copy()
    for u in range(g.n):
        a, b = g.row_ptr[u], g.row_ptr[u + 1]
        col[a:b] = rng.permutation(col[a:b])
    from synth.gen import Graph as SG
    # repeat the first out-edge of every 7th vertex
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    extra = np.flatnonzero(np.diff(g.row_ptr) > 0)[::7]
    rows = [list(col[g.row_ptr[u]:g.row_ptr[u + 1]]) for u in range(g.n)]
    for u in extra:
        rows[u].append(rows[u][0])
    rp = np.zeros(g.n + 1, np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col2 = np.array([x for r in rows for x in r], np.int32)
    g2 = SG(rp, col2, g.n_labels, g.lab_ptr, g.lab, None, "chunglu_unsorted")
    qs = workloads.chunglu10k_queries(40)
    want = oracle_results(oracle.Oracle(g2), qs)
    G = K.Graph.from_synth(g2)
    say("unsorted rows")
    assert_all_same(G.search_batch(qs), want, "unsorted batch")
    for i in range(0, 40, 5):
        assert_same(G.keyword_search(qs[i].kw, qs[i].d_max, qs[i].k), want[i], f"unsorted plain {i}")
    G.close()
