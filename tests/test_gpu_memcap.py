"""The device-memory cap (kws_set_mem_limit) and its ENOMEM paths.

* loading a graph over the cap is refused with ENOMEM and holds nothing;
* a search whose state does not fit the budget fails with ENOMEM, and the
  same handle works once the cap is lifted;
* a server whose budget holds no word slot is refused; one whose budget
  holds two slots serves many more queries than fit at once (they queue and
  are admitted as slots free up), every answer equal to the oracle's, and
  the library never holds more than the cap.
"""
import sys

import numpy as np
import pytest

import oracle
from parity import assert_all_same, oracle_results
from synth import gen, workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def K():
    import paper_2504_09311_amd as K
    K.load_library()
    yield K
    K.set_mem_limit(-1)


def graph_bytes(K, g):
    base = K.mem_in_use()
    G = K.Graph.from_synth(g)
    used = K.mem_in_use() - base
    G.close()
    assert K.mem_in_use() == base
    return used


def test_load_refused_over_cap(K):
    g = workloads.chunglu10k()
    need = graph_bytes(K, g)
    base = K.mem_in_use()
    try:
        K.set_mem_limit(base + need // 2)
        with pytest.raises(K.KwsError) as ei:
            K.Graph.from_synth(g)
        assert ei.value.status == K.ENOMEM
        assert K.mem_in_use() == base, "a refused load must hold nothing"
    finally:
        K.set_mem_limit(-1)
    G = K.Graph.from_synth(g)
    G.close()


def test_search_over_budget_then_recovers(K):
    g = workloads.chunglu10k()
    qs = workloads.chunglu10k_queries(4)
    need = graph_bytes(K, g)
    base = K.mem_in_use()
    # loading also needs transient scratch (in-degree counts, label keys and
    # counts: about 125 KB here); 256 KB covers it but not one word of search
    # state (vis, two frontiers, nxt and two planes: 6 * 8 * n = 480 KB)
    margin = 256 << 10
    assert margin < 6 * 8 * g.n
    try:
        K.set_mem_limit(base + need + margin)
        G = K.Graph.from_synth(g)
        with pytest.raises(K.KwsError) as ei:
            G.keyword_search(qs[0].kw, qs[0].d_max, qs[0].k)
        assert ei.value.status == K.ENOMEM
        with pytest.raises(K.KwsError) as ei:
            G.search_batch(qs)
        assert ei.value.status == K.ENOMEM
        assert K.mem_in_use() <= base + need + margin
    finally:
        K.set_mem_limit(-1)
    o = oracle.Oracle(g)
    assert_all_same(G.search_batch(qs), oracle_results(o, qs), "after the cap was lifted")
    G.close()


def test_server_admission_under_cap(K):
    g = workloads.chunglu10k()
    n = g.n
    per_word = n * 8 * (4 + 3)            # vis, two frontiers, nxt and 3 distance planes (d_max <= 4)
    # frontier list, offsets, flags, per-step tables and results; also more
    # than the transient scratch of loading (about 125 KB here)
    slack = 10 * n + (256 << 10)
    assert slack < per_word and per_word // 2 > (128 << 10)
    need = graph_bytes(K, g)
    base = K.mem_in_use()
    qs = gen.queries(40, g.n_labels, 1.1, 8, 8, [2, 3, 4], 10, 0x5EED0101, 0x5EED0777)
    o = oracle.Oracle(g)
    want = oracle_results(o, qs)
    try:
        K.set_mem_limit(base + need + per_word // 2)
        G = K.Graph.from_synth(g)
        with pytest.raises(K.KwsError) as ei:
            K.Server(G, max_dmax=4)
        assert ei.value.status == K.ENOMEM
        G.close()
        cap = base + need + 2 * per_word + slack
        K.set_mem_limit(cap)
        G = K.Graph.from_synth(g)
        S = K.Server(G, max_dmax=4)
        st = S.stats()
        say("server under the cap:", st["max_words"], "word slots")
        assert st["max_words"] == 2
        ts = [S.submit(q.kw, q.d_max, q.k) for q in qs]   # 40 queries x 8 lanes = 5 words' worth
        got = [S.wait(t, 60.0) for t in ts]
        st = S.stats()
        assert K.mem_in_use() <= cap
        S.close()
        G.close()
    finally:
        K.set_mem_limit(-1)
    assert st["completed"] == len(qs) and st["steps"] > max(q.d_max for q in qs) + 1
    assert_all_same(got, want, "served under the cap")
