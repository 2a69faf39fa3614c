"""GPU tests of the serving loop and of the captured-graph batch path.

* every served result equals the oracle's, whether the query ran alone or
  arrived while others were on the device (continuous batching);
* queries with different radii and keyword counts share slots and steps;
* cancel, queue-full (EBUSY) and shutdown with work in flight;
* the hipGraph replay of a batch gives the same answers as direct launches;
* pipelined batches (submit, then collect) give the same answers as
  synchronous ones, in any collection order and with synchronous calls
  interleaved.
"""
import sys
import time

import numpy as np
import pytest

import oracle
from parity import assert_all_same, assert_same, oracle_results
from synth import gen, tiny, workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def K():
    import paper_2504_09311_amd as K
    K.load_library()
    return K


@pytest.fixture(scope="module")
def rmat14(K):
    g = workloads.rmat_flat(14)
    return g, oracle.Oracle(g), K.Graph.from_synth(g)


def test_served_alone_equals_mix_equals_oracle(K, rmat14):
    g, o, G = rmat14
    qs = workloads.rmat_flat_queries(120, 2, 8, [2, 3, 4], 20, cfg=2, qcfg=3)
    want = oracle_results(o, qs)
    S = K.Server(G, max_words=6, max_dmax=4, tile_words=2)
    say("served alone")
    alone = []
    for q in qs[:20]:
        t = S.submit(q.kw, q.d_max, q.k)
        alone.append(S.wait(t, 30.0))
    assert_all_same(alone, want[:20], "alone")
    say("served mix")
    tickets = []
    for i, q in enumerate(qs):
        tickets.append(S.submit(q.kw, q.d_max, q.k))
        if i % 7 == 0:
            time.sleep(0.0005)      # arrivals spread while earlier queries run
    mix = [S.wait(t, 60.0) for t in tickets]
    assert all(r is not None for r in mix)
    assert_all_same(mix, want, "mix")
    st = S.stats()
    assert st["completed"] == 140 and st["steps"] > 0 and st["p99_us"] >= st["p50_us"] > 0
    assert st["mean_active_words"] > 1.0          # slots really overlapped on the device
    S.close()


def test_served_tiny_graphs(K):
    for seed in range(0, 40):
        g = tiny.random_graph(seed)
        qs = [q for q in tiny.random_queries(g, seed, 8)]
        o = oracle.Oracle(g)
        want = [o.search(q.kw, q.d_max, q.k) for q in qs]
        G = K.Graph.from_synth(g)
        # a server takes the graph's seeding options when it is created
        table = 1 if seed % 2 else -1
        G.set_options(seed_mode=2 if seed % 3 else 0, seed_table=table)
        S = K.Server(G, max_words=3, tile_words=1)
        ts = [S.submit(q.kw, q.d_max, q.k) for q in qs]
        got = [S.wait(t, 30.0) for t in ts]
        assert_all_same(got, want, f"served tiny {seed} table {table}")
        S.close()
        G.close()


def test_served_type_hierarchy(K):
    # vertex seeding through the type-row table and by walking each label
    g, leaves = workloads.rmat_hier(12, cfg=4)
    qs = workloads.rmat_hier_queries(g.type_parent, leaves, 48, cfg=4)
    want = oracle_results(oracle.Oracle(g), qs)
    G = K.Graph.from_synth(g)
    for table in (1, -1):
        say("served hierarchy, table", table)
        G.set_options(seed_mode=2, seed_table=table)
        S = K.Server(G, max_words=4, max_dmax=4, tile_words=2)
        ts = [S.submit(q.kw, q.d_max, q.k) for q in qs]
        got = [S.wait(t, 60.0) for t in ts]
        assert_all_same(got, want, f"served hierarchy table {table}")
        S.close()
    G.close()


def test_server_cancel_busy_and_shutdown(K, rmat14):
    g, o, G = rmat14
    qs = workloads.rmat_flat_queries(40, 2, 6, [3], 10, cfg=2, qcfg=7)
    S = K.Server(G, max_words=1, queue_capacity=8, max_dmax=3)
    tickets, busy = [], 0
    for q in qs:
        try:
            tickets.append(S.submit(q.kw, q.d_max, q.k))
        except K.KwsError as e:
            assert e.status == K.EBUSY
            busy += 1
    assert busy > 0
    S.cancel(tickets[-1])
    with pytest.raises(K.KwsError) as e:
        S.wait(tickets[-1], 30.0)
    assert e.value.status == K.ECANCELLED
    first = S.wait(tickets[0], 30.0)
    assert_same(first, o.search(qs[0].kw, qs[0].d_max, qs[0].k), "first served")
    with pytest.raises(K.KwsError) as e:
        S.poll(123456789)
    assert e.value.status == K.EINVAL
    with pytest.raises(K.KwsError):
        S.submit([1], 4, 5)                       # above the server's max_dmax
    S.close()                                    # queued work cancelled, running slot drained
    # the graph is still usable afterwards
    r = G.keyword_search(qs[1].kw, qs[1].d_max, qs[1].k)
    assert_same(r, o.search(qs[1].kw, qs[1].d_max, qs[1].k), "after shutdown")


def test_graph_replay_matches(K, rmat14):
    g, o, G = rmat14
    qs = workloads.rmat_flat_queries(64, 2, 8, [2, 3, 4], 20, cfg=2, qcfg=5)
    want = oracle_results(o, qs)
    G.set_options(use_graph=1)
    for rep in range(3):
        say("graph replay", rep)
        assert_all_same(G.search_batch(qs), want, f"graph replay {rep}")
        # the program's own eager work between replays
        r = G.keyword_search(qs[rep].kw, qs[rep].d_max, qs[rep].k)
        assert_same(r, want[rep], "eager between replays")
    G.set_options()


def test_graph_replays_across_batches(K, rmat14):
    """Different batches of one shape (48 queries of 4 keywords, d_max 3,
    k 20) run through one captured graph: the capture counter moves once,
    the replay counter once per later batch, and every answer equals the
    oracle's. The pipelined path (two plan buffers) captures once per buffer."""
    g, o, _ = rmat14
    from synth import gen
    G = K.Graph.from_synth(g)
    # no lane sharing: 16 four-keyword queries fill a word, so every batch has 3 words
    G.set_options(use_graph=1, seed_mode=2, share_lanes=-1)
    batches = [gen.queries(48, g.n_labels, 1.0, 4, 4, [3], 20, 0x5EED0102, 900 + i) for i in range(6)]
    wants = [oracle_results(o, qs) for qs in batches]
    assert len({tuple(tuple(q.kw) for q in qs) for qs in batches}) == 6      # six different batches
    i0 = G.info()
    for i, (qs, want) in enumerate(zip(batches, wants)):
        say("replay batch", i)
        assert_all_same(G.search_batch(qs), want, f"graph batch {i}")
    i1 = G.info()
    assert (i1.graph_captures - i0.graph_captures, i1.graph_replays - i0.graph_replays) == (1, 5)
    # pipelined: submit the next batch before collecting the previous one
    t = G.search_batch_submit(batches[0])
    for i in range(1, 7):
        nxt = G.search_batch_submit(batches[i % 6]) if i < 6 else None
        got = K.Graph.results_of(G.search_batch_collect(t), len(batches[i - 1]))
        assert_all_same(got, wants[i - 1], f"pipelined graph batch {i - 1}")
        t = nxt
    i2 = G.info()
    assert (i2.graph_captures - i1.graph_captures, i2.graph_replays - i1.graph_replays) == (2, 4)
    G.close()


def test_caller_stream(K, rmat14):
    """Work on a stream the caller created through the library's own HIP runtime."""
    import ctypes
    g, o, G = rmat14
    hip = ctypes.CDLL("libamdhip64.so.7")          # the instance libkws.so is linked against
    st = ctypes.c_void_p()
    assert hip.hipStreamCreate(ctypes.byref(st)) == 0
    try:
        qs = workloads.rmat_flat_queries(32, 2, 6, [2, 3], 10, cfg=2, qcfg=8)
        want = oracle_results(o, qs)
        G.set_stream(st.value)
        assert G.get_stream() == st.value
        say("caller stream")
        assert_all_same(G.search_batch(qs), want, "caller stream")
        assert_same(G.keyword_search(qs[0].kw, qs[0].d_max, qs[0].k), want[0], "caller stream, one query")
        G.set_stream(None)
        assert G.get_stream() not in (0, st.value)
        assert_all_same(G.search_batch(qs), want, "own stream again")
    finally:
        G.set_stream(None)
        hip.hipStreamDestroy(st)


def test_profile_class_mask(K, rmat14):
    g, o, G = rmat14
    qs = workloads.rmat_flat_queries(32, 2, 6, [2, 3], 10, cfg=2, qcfg=9)
    want = oracle_results(o, qs)
    G.profile_classes(["pull", "score"])
    G.profile_enable(True)
    G.profile_reset()
    assert_all_same(G.search_batch(qs), want, "profiled, two classes")
    G.profile_enable(False)
    prof = G.profile_read()
    assert prof["score"][0] >= 1 and prof["seed"][0] == 0 and prof["finalize"][0] == 0 and prof["answer"][0] == 0
    assert prof["host_plan"][0] >= 1                      # host phases use no events
    G.profile_classes(None)
    G.profile_enable(True)
    G.profile_reset()
    assert_all_same(G.search_batch(qs), want, "profiled, every class")
    G.profile_enable(False)
    prof = G.profile_read()
    assert prof["seed"][0] >= 1 and prof["score"][0] >= 1 and prof["answer"][0] >= 1


def test_pipelined_batches(K, rmat14):
    g, o, G = rmat14
    qa = workloads.rmat_flat_queries(64, 2, 8, [2, 3, 4], 20, cfg=2, qcfg=6)
    qb = workloads.rmat_flat_queries(48, 2, 6, [1, 2, 3], 10, cfg=2, qcfg=7)
    wa, wb = oracle_results(o, qa), oracle_results(o, qb)
    for use_graph in (0, 1):
        G.set_options(use_graph=use_graph)
        say("pipelined, graph", use_graph)
        ta = G.search_batch_submit(qa)
        tb = G.search_batch_submit(qb)
        with pytest.raises(K.KwsError) as e:          # two in flight at most
            G.search_batch_submit(qa)
        assert e.value.status == K.EBUSY
        # a synchronous call while both are pending
        assert_same(G.keyword_search(qa[0].kw, qa[0].d_max, qa[0].k), wa[0], "sync between")
        fb = G.search_batch_collect(tb)            # out of order
        fa = G.search_batch_collect(ta)
        assert_all_same(G.results_of(fa, len(qa)), wa, f"pipelined a, graph {use_graph}")
        assert_all_same(G.results_of(fb, len(qb)), wb, f"pipelined b, graph {use_graph}")
        with pytest.raises(K.KwsError):
            G.search_batch_collect(ta)             # each ticket once
        # a steady pipeline: submit batch i + 1 before collecting batch i
        order = [(qa, wa), (qb, wb), (qb, wb), (qa, wa), (qa, wa)]
        t = G.search_batch_submit(order[0][0])
        for i in range(len(order)):
            nxt = G.search_batch_submit(order[i + 1][0]) if i + 1 < len(order) else None
            qs, want = order[i]
            assert_all_same(G.results_of(G.search_batch_collect(t), len(qs)), want, f"steady {i}")
            t = nxt
    G.set_options()


def test_autotune_picks_identical_answers_and_caches(K, rmat14, tmp_path):
    g, o, G = rmat14
    qs = workloads.rmat_flat_queries(48, 2, 8, [2, 3, 4], 20, cfg=2, qcfg=9)
    want = oracle_results(o, qs)
    cache = str(tmp_path / "tune.txt")
    best, rep = G.autotune(qs, reps=2, cache_path=cache)
    assert rep["configs_tried"] > 10 and rep["best_ms"] <= rep["default_ms"] and not rep["from_cache"]
    assert_all_same(G.search_batch(qs), want, "tuned")
    best2, rep2 = G.autotune(qs, reps=2, cache_path=cache)
    assert rep2["from_cache"] and best2["tile_words"] == best["tile_words"]
    G.set_options()
