"""GPU parity of parallel peeling (densest-subgraph discovery) through the
C ABI of include/dsd.h.

Every field the oracle produces is compared exactly: the round in which
each vertex is peeled, |S_i| and f(S_i) for every round, and the index of
the densest S_i; for DG, DW and FD and several eps. At the full benchmark
size (R-MAT 2^24, where the oracle's per-round recomputation takes too
long) the run is certified instead: for sampled rounds every vertex's
decision is recomputed on the host from the returned peel rounds, and the
sizes and f values are recomputed from their definitions.
"""
import math
import sys
from fractions import Fraction

import numpy as np
import pytest

import oracle
from synth import workloads
from test_peel_pins import random_graph

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def K():
    import paper_2504_09311_amd as K
    K.load_library()
    return K


def check_same(K, n, src, dst, ew, vw, metric, num, den, what):
    c, a = oracle.metric_weights(metric, src, dst, n, ew, vw)
    want = oracle.peel(n, src, dst, c, a, 2, num, den)
    G = K.PeelGraph(n, src, dst, metric, edge_w=ew, vertex_w=vw)
    pr, sizes, fs, sm = G.peel(2, num, den)
    G.close()
    assert np.array_equal(pr, want.peel_round), what
    assert np.array_equal(sizes, want.sizes) and np.array_equal(fs, want.f), what
    assert sm["rounds"] == want.rounds and sm["best"] == want.best, what
    if n:
        assert sm["best_size"] == want.sizes[want.best] and sm["best_f"] == want.f[want.best], what


@pytest.mark.parametrize("block", range(3))
def test_tiny_random(K, block):
    for seed in range(block * 60, block * 60 + 60):
        n, src, dst, ew, vw = random_graph(seed, n_max=24, p_max=0.4)
        for metric in oracle.METRICS:
            num, den = [(0, 1), (1, 10), (1, 2), (3, 1)][seed % 4]
            check_same(K, n, src, dst, ew, vw, metric, num, den, f"tiny {seed} {metric} {num}/{den}")


def test_empty_and_edgeless(K):
    e = np.zeros(0, np.int32)
    check_same(K, 0, e, e, np.zeros(0, np.int64), np.zeros(0, np.int64), "DG", 1, 10, "empty")
    vw = np.array([5, 0, 7, 7], np.int64)
    for metric in oracle.METRICS:
        check_same(K, 4, e, e, np.zeros(0, np.int64), vw, metric, 1, 10, f"edgeless {metric}")


def test_fd_golden_hand_derived(K):
    """The device's own FD weights (computed from degrees at load) give the
    hand-derived rounds, sizes and f values of tests/golden/fd_weights.json."""
    from test_peel_pins import load_fd_golden
    gd = load_fd_golden()
    n = gd["n"]
    src = np.array([e[0] for e in gd["edges"]], np.int32)
    dst = np.array([e[1] for e in gd["edges"]], np.int32)
    vw = np.array(gd["vertex_w"], np.int64)
    for case in gd["cases"]:
        G = K.PeelGraph(n, src, dst, "FD", edge_w=None, vertex_w=vw)
        pr, sizes, fs, sm = G.peel(case["k"], case["eps_num"], case["eps_den"])
        G.close()
        assert pr.tolist() == case["peel_round"], case
        assert sizes.tolist() == case["sizes"] and fs.tolist() == case["f"], case
        assert sm["rounds"] == case["rounds"] and sm["best"] == case["best"], case


def test_threshold_below_two_is_rejected(K):
    n = 6
    src = np.arange(n, dtype=np.int32)
    dst = ((np.arange(n) + 1) % n).astype(np.int32)
    G = K.PeelGraph(n, src, dst, "DG")
    for k, num, den in [(1, 0, 1), (1, 9, 10)]:
        with pytest.raises(K.KwsError) as ei:
            G.peel(k, num, den)
        assert ei.value.status == K.EINVAL
    pr, sizes, fs, sm = G.peel(1, 1, 1)
    G.close()
    assert sm["rounds"] == 1 and (pr == 1).all() and sizes.tolist() == [6, 0]


@pytest.mark.parametrize("name,scale", [("peel_chunglu10k", None), ("peel_rmat20", 14), ("peel_rmat20", 16)])
def test_synthetic_graphs(K, name, scale):
    inp = workloads.peel_input(name, scale=scale)
    for metric in oracle.METRICS:
        for num, den in [(1, 10), (1, 2)]:
            say(name, scale, metric, num, den)
            check_same(K, inp["n"], inp["src"], inp["dst"], inp["edge_w"], inp["vertex_w"], metric, num, den,
                       f"{name} {scale} {metric} {num}/{den}")


def certify(n, src, dst, c, a, k, num, den, pr, sizes, fs, best, rounds_to_check):
    """Recompute decisions and records of the given rounds from peel rounds."""
    R = len(sizes) - 1
    assert sizes[R] == 0 and (pr >= 1).all() and (pr <= R).all()
    for i in range(1, R + 1):
        assert sizes[i] * (den + num) < sizes[i - 1] * den          # shrink bound of every round
    cnt = np.bincount(pr, minlength=R + 2)
    for i in range(R + 1):                                           # |S_i| from the peel rounds
        assert sizes[i] == n - int(cnt[1:i + 1].sum())
    src64, dst64 = src.astype(np.int64), dst.astype(np.int64)
    for i in rounds_to_check:
        alive_prev = pr >= i                                         # S_{i-1}
        both = alive_prev[src64] & alive_prev[dst64]
        f_prev = int(a[alive_prev].sum()) + int(c[both].sum())
        assert f_prev == fs[i - 1]
        # per-vertex sums of at most 2^53 each, so float64 bin counts are exact
        w = a.astype(np.int64) + \
            np.bincount(src64[both], weights=c[both], minlength=n).astype(np.int64) + \
            np.bincount(dst64[both], weights=c[both], minlength=n).astype(np.int64)
        s = int(alive_prev.sum())
        thr = (k * (den + num) * f_prev) // (s * den)      # w * s * den <= rhs  <=>  w <= thr
        assert np.array_equal(w[alive_prev] <= thr, pr[alive_prev] == i), i
    g = [Fraction(int(fs[i]), int(sizes[i])) for i in range(R)]
    assert best == g.index(max(g))                                   # first densest


def test_rmat24_full_scale_certified(K):
    inp = workloads.peel_input("peel_rmat24")
    n, src, dst = inp["n"], inp["src"], inp["dst"]
    say("peel rmat24", n, src.shape[0])
    for metric in ("DG", "FD"):
        if metric != "FD":
            c, a = oracle.metric_weights(metric, src, dst, n, inp["edge_w"], inp["vertex_w"])
        G = K.PeelGraph(n, src, dst, metric, edge_w=inp["edge_w"], vertex_w=inp["vertex_w"])
        pr, sizes, fs, sm = G.peel(2, 1, 10)
        G.close()
        say(metric, "rounds", sm["rounds"], "best", sm["best"], sm["best_size"])
        if metric == "FD":
            # FD weights depend only on source degrees: one table lookup per edge
            deg = np.bincount(src, minlength=n) + np.bincount(dst, minlength=n)
            lib = oracle.load()
            table = np.array([lib.orc_fd_weight(int(d)) for d in range(int(deg.max()) + 1)], np.int64)
            c, a = table[deg[src]], np.ascontiguousarray(inp["vertex_w"], np.int64)
        R = sm["rounds"]
        assert R - 1 < math.log(n) / math.log(1.1)
        say("certifying rounds", sorted({1, 2, R // 2, R}))
        certify(n, src, dst, c, a, 2, 1, 10, pr, sizes, fs, sm["best"], sorted({1, 2, R // 2, R}))



def test_rounds_left_on_device(K):
    inp = workloads.peel_input("peel_rmat20", scale=14)
    n = inp["n"]
    for metric in oracle.METRICS:
        G = K.PeelGraph(n, inp["src"], inp["dst"], metric, edge_w=inp["edge_w"], vertex_w=inp["vertex_w"])
        with pytest.raises(K.KwsError):
            G.rounds()                                   # no run yet
        pr, sizes, fs, sm = G.peel(2, 1, 10)
        none, sizes_d, fs_d, sm_d = G.peel(2, 1, 10, rounds=False)
        assert none is None and np.array_equal(G.rounds(), pr), metric
        assert np.array_equal(sizes_d, sizes) and np.array_equal(fs_d, fs) and sm_d["best"] == sm["best"], metric
        assert G.device_rounds() != 0
        G.close()


# ---- the long-tail optimisations (global threshold, local trimming)

def check_same_opt(K, n, src, dst, ew, vw, metric, num, den, mode, what, c=None, a=None):
    if c is None:
        c, a = oracle.metric_weights(metric, src, dst, n, ew, vw)
    want = oracle.peel_opt(n, src, dst, c, a, 2, num, den, mode=mode)
    G = K.PeelGraph(n, src, dst, metric, edge_w=ew, vertex_w=vw)
    pr, sizes, fs, sm = G.peel(2, num, den, mode=mode)
    G.close()
    assert np.array_equal(pr, want.peel_round), what
    assert np.array_equal(sizes, want.sizes) and np.array_equal(fs, want.f), what
    assert sm["rounds"] == want.rounds and sm["best"] == want.best and sm["trims"] == want.trims, what
    assert sm["steps"] == want.rounds + want.trims, what


@pytest.mark.parametrize("mode", ["gpo", "lpo"])
def test_optimised_tiny_random(K, mode):
    for seed in range(200, 320):
        n, src, dst, ew, vw = random_graph(seed, n_max=24, p_max=0.4)
        for metric in oracle.METRICS:
            num, den = [(0, 1), (1, 10), (1, 2), (3, 1)][seed % 4]
            check_same_opt(K, n, src, dst, ew, vw, metric, num, den, mode, f"tiny {seed} {metric} {num}/{den} {mode}")


def test_optimised_threshold_and_strict_trimming(K):
    from test_peel_pins import powerlaw_graph
    src, dst, ew, vw = powerlaw_graph(1495, 39)           # the global threshold changes the rounds here
    for mode in ("gpo", "lpo"):
        check_same_opt(K, 39, src, dst, ew, vw, "DW", 1, 10, mode, f"powerlaw 1495 {mode}")
    # vertex weights only (FD with no edges): 22 zeros, then 1, 4, 7; two trims
    e = np.zeros(0, np.int32)
    vw = np.array([0] * 22 + [1, 4, 7], np.int64)
    check_same_opt(K, 25, e, e, np.zeros(0, np.int64), vw, "FD", 0, 1, "lpo", "strict trimming")
    G = K.PeelGraph(25, e, e, "FD", vertex_w=vw)
    _, _, _, sm = G.peel(2, 0, 1, mode="lpo")
    G.close()
    assert sm["trims"] == 2


@pytest.mark.parametrize("name,scale", [("peel_chunglu10k", None), ("peel_rmat20", 14), ("peel_rmat20", 16)])
def test_optimised_synthetic_graphs(K, name, scale):
    inp = workloads.peel_input(name, scale=scale)
    for metric in oracle.METRICS:
        for mode in ("gpo", "lpo"):
            for num, den in [(1, 10), (1, 2)]:
                say(name, scale, metric, mode, num, den)
                check_same_opt(K, inp["n"], inp["src"], inp["dst"], inp["edge_w"], inp["vertex_w"], metric, num, den,
                               mode, f"{name} {scale} {metric} {mode} {num}/{den}")


def test_optimised_rmat24_full_scale(K):
    inp = workloads.peel_input("peel_rmat24")
    n = inp["n"]
    c, a = oracle.metric_weights("DG", inp["src"], inp["dst"], n)
    for mode in ("gpo", "lpo"):
        say("peel rmat24", mode)
        check_same_opt(K, n, inp["src"], inp["dst"], inp["edge_w"], inp["vertex_w"], "DG", 1, 10, mode,
                       f"rmat24 DG {mode}", c=c, a=a)
