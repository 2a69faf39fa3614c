"""Pins of the parallel-peeling oracle (CPU only).

Nothing here shares code with ``oracle/peel_oracle.c``:

* an exact re-simulation of the round structure in Python with rational
  numbers and sets, recomputing f, g and every peeling weight from the
  definition in every round, must give the same rounds, sizes, f values
  and best index on random small graphs under all three metrics and
  several eps;
* the approximation guarantee of the parallel algorithm (Section 4.2,
  Theorem 4.2: g(S^p) >= g(S*) / (k (1 + eps))) against the optimum found
  by enumerating every vertex subset;
* the sequential algorithm's guarantee (Section 2.2, Theorem 2.1: factor 2)
  for the sequential oracle, against the same optimum;
* the round bound (Section 4.2, Lemma 4.1): every round shrinks the set by
  more than a factor 1 + eps, so R - 1 < log_{1+eps} |V|;
* closed forms: complete digraphs, stars, a clique beside a path.
"""
import itertools
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
from synth import gen, workloads


def random_graph(seed, n_max=11, p_max=0.5):
    rnd = random.Random(seed)
    n = rnd.randint(1, n_max)
    p = rnd.uniform(0.05, p_max)
    src, dst = [], []
    for u in range(n):
        for v in range(n):
            if u != v and rnd.random() < p:
                src.append(u)
                dst.append(v)
                if rnd.random() < 0.1:          # a repeated edge now and then
                    src.append(u)
                    dst.append(v)
    edge_w = [rnd.randint(1, 9) for _ in src]
    vertex_w = [rnd.randint(0, 1 << 24) if rnd.random() < 0.7 else 0 for _ in range(n)]
    return n, np.array(src, np.int32), np.array(dst, np.int32), np.array(edge_w, np.int64), \
        np.array(vertex_w, np.int64)


def f_of(S, src, dst, c, a):
    return sum(int(a[u]) for u in S) + sum(int(c[e]) for e in range(len(src)) if src[e] in S and dst[e] in S)


def simulate(n, src, dst, c, a, k, eps):
    """Algorithm 2, written with sets and Fractions."""
    S = set(range(n))
    rounds_of = {}
    sizes, fs = [n], [f_of(S, src, dst, c, a)]
    i = 0
    while S:
        f = f_of(S, src, dst, c, a)
        g = Fraction(f, len(S))
        tau = k * (1 + eps) * g
        U = set()
        for u in S:
            w = f - f_of(S - {u}, src, dst, c, a)      # the decrease of f when u is peeled
            if w <= tau:
                U.add(u)
        i += 1
        for u in U:
            rounds_of[u] = i
        S = S - U
        sizes.append(len(S))
        fs.append(f_of(S, src, dst, c, a))
    best = max(range(len(sizes) - 1), key=lambda j: (Fraction(fs[j], sizes[j]), -j)) if n else 0
    return [rounds_of[u] for u in range(n)], sizes, fs, best


def optimum(n, src, dst, c, a):
    best = Fraction(0)
    for r in range(1, n + 1):
        for S in itertools.combinations(range(n), r):
            best = max(best, Fraction(f_of(set(S), src, dst, c, a), r))
    return best


EPS = [(0, 1), (1, 10), (1, 2), (3, 1)]


@pytest.mark.parametrize("block", range(4))
def test_oracle_matches_exact_simulation(block):
    for seed in range(block * 40, block * 40 + 40):
        n, src, dst, ew, vw = random_graph(seed)
        for metric in oracle.METRICS:
            c, a = oracle.metric_weights(metric, src, dst, n, ew, vw)
            num, den = EPS[seed % len(EPS)]
            r = oracle.peel(n, src, dst, c, a, 2, num, den)
            pr, sizes, fs, best = simulate(n, src, dst, c, a, 2, Fraction(num, den))
            assert r.peel_round.tolist() == pr, (seed, metric)
            assert r.sizes.tolist() == sizes and r.f.tolist() == fs, (seed, metric)
            assert r.best == best, (seed, metric)


def test_approximation_guarantees():
    for seed in range(300, 380):
        n, src, dst, ew, vw = random_graph(seed, n_max=10)
        for metric in oracle.METRICS:
            c, a = oracle.metric_weights(metric, src, dst, n, ew, vw)
            opt = optimum(n, src, dst, c, a)
            for num, den in EPS:
                r = oracle.peel(n, src, dst, c, a, 2, num, den)
                gp = Fraction(int(r.f[r.best]), int(r.sizes[r.best]))
                assert gp * 2 * Fraction(den + num, den) >= opt, (seed, metric, num, den)
                S = set(r.best_set().tolist())
                assert Fraction(f_of(S, src, dst, c, a), len(S)) == gp
            mask, bf, bs = oracle.peel_sequential(n, src, dst, c, a)
            assert 2 * Fraction(bf, bs) >= opt, (seed, metric)
            assert mask.sum() == bs and f_of(set(np.flatnonzero(mask).tolist()), src, dst, c, a) == bf


def test_round_bound_on_rmat():
    inp = workloads.peel_input("peel_rmat20", scale=12)
    n, src, dst = inp["n"], inp["src"], inp["dst"]
    for metric in oracle.METRICS:
        c, a = oracle.metric_weights(metric, src, dst, n, inp["edge_w"], inp["vertex_w"])
        for num, den in [(1, 10), (1, 2)]:
            r = oracle.peel(n, src, dst, c, a, 2, num, den)
            assert r.rounds - 1 < math.log(n) / math.log(1 + num / den)
            for i in range(1, r.rounds + 1):      # |S_i| (1 + eps) < |S_{i-1}|
                assert r.sizes[i] * (den + num) < r.sizes[i - 1] * den
            assert r.sizes[-1] == 0 and (r.peel_round >= 1).all() and (r.peel_round <= r.rounds).all()


def complete_digraph(n):
    src = [u for u in range(n) for v in range(n) if u != v]
    dst = [v for u in range(n) for v in range(n) if u != v]
    return np.array(src, np.int32), np.array(dst, np.int32)


def test_closed_forms():
    # complete digraph: every vertex has the same weight 2(n-1) <= 2(1+eps)(n-1):
    # one round, and the whole graph (g = n - 1) is the answer
    for n in (2, 5, 9):
        src, dst = complete_digraph(n)
        c, a = oracle.metric_weights("DG", src, dst, n)
        r = oracle.peel(n, src, dst, c, a)
        assert r.rounds == 1 and r.best == 0 and r.f[0] == n * (n - 1)
    # star (leaves -> centre): leaves go in round 1, the centre in round 2
    n = 12
    src = np.arange(1, n, dtype=np.int32)
    dst = np.zeros(n - 1, np.int32)
    c, a = oracle.metric_weights("DG", src, dst, n)
    r = oracle.peel(n, src, dst, c, a)
    assert r.rounds == 2 and r.peel_round[0] == 2 and (r.peel_round[1:] == 1).all() and r.best == 0
    # a 6-clique beside a long path: the clique is the densest set found
    cs, cd = complete_digraph(6)
    ps = np.arange(6, 40, dtype=np.int32)
    pd = ps + 1
    src = np.concatenate([cs, ps])
    dst = np.concatenate([cd, pd])
    c, a = oracle.metric_weights("DG", src, dst, 41)
    r = oracle.peel(41, src, dst, c, a)
    assert sorted(r.best_set().tolist()) == list(range(6))


def test_fd_weights_follow_the_formula():
    for d in (1, 2, 10, 1000, 123456):
        assert oracle.load().orc_fd_weight(d) == round((1 << 24) / math.log(d + 5))


def load_fd_golden():
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fd_weights.json")) as f:
        return json.load(f)


def test_fd_golden_hand_derived():
    """FD edge weights, peeling weights and rounds against literal values
    derived by hand (tests/golden/fd_weights.json): the source's total
    degree, natural log, + 5, 2^-24 units. No formula is recomputed here."""
    gd = load_fd_golden()
    n = gd["n"]
    src = np.array([e[0] for e in gd["edges"]], np.int32)
    dst = np.array([e[1] for e in gd["edges"]], np.int32)
    vw = np.array(gd["vertex_w"], np.int64)
    c, a = oracle.metric_weights("FD", src, dst, n, None, vw)
    assert c.tolist() == gd["c"]
    assert a.tolist() == gd["vertex_w"]
    for case in gd["cases"]:
        r = oracle.peel(n, src, dst, c, a, case["k"], case["eps_num"], case["eps_den"])
        assert r.peel_round.tolist() == case["peel_round"], case
        assert r.sizes.tolist() == case["sizes"] and r.f.tolist() == case["f"], case
        assert r.rounds == case["rounds"] and r.best == case["best"], case
    # the literal peeling weights are consistent with the literal c and a
    # (each edge adds to both endpoints) and with f(V)
    w = list(gd["vertex_w"])
    for (s, d), ce in zip(gd["edges"], gd["c"]):
        w[s] += ce
        w[d] += ce
    assert w == gd["w0"]
    assert sum(gd["w0"]) == 2 * sum(gd["c"]) + sum(gd["vertex_w"])
    assert gd["cases"][0]["f"][0] == sum(gd["c"]) + sum(gd["vertex_w"])


def test_threshold_below_two_is_rejected():
    """k (1 + eps) < 2 cannot guarantee progress (Algorithm 2 on a regular
    graph with k = 1, eps = 0 peels nothing: every weight is exactly 2 g),
    so both readings of it are refused; k (1 + eps) = 2 exactly is allowed."""
    n = 6
    src = np.arange(n, dtype=np.int32)
    dst = ((np.arange(n) + 1) % n).astype(np.int32)        # directed cycle: every w = 2 = 2 g
    c, a = oracle.metric_weights("DG", src, dst, n)
    for k, num, den in [(1, 0, 1), (1, 9, 10)]:
        with pytest.raises(ValueError):
            oracle.peel(n, src, dst, c, a, k, num, den)
        with pytest.raises(ValueError):
            oracle.peel_opt(n, src, dst, c, a, k, num, den, mode="lpo")
    r = oracle.peel(n, src, dst, c, a, 1, 1, 1)            # k (1 + eps) = 2: all peeled at once
    assert r.rounds == 1 and (r.peel_round == 1).all()


def test_uniform_generator():
    x = gen.uniform_i64(7, 1, 20000, 1, 1000)
    assert x.min() >= 1 and x.max() <= 1000 and abs(x.mean() - 500.5) < 10
    assert np.array_equal(x, gen.uniform_i64(7, 1, 20000, 1, 1000))
    assert not np.array_equal(x, gen.uniform_i64(7, 2, 20000, 1, 1000))


# ---- the long-tail optimisations of Section 5 (Algorithms 3 and 4)

def simulate_opt(n, src, dst, c, a, k, eps, mode):
    """Algorithms 3 (mode 'gpo') and 4 (mode 'lpo'), written with sets and Fractions."""
    S = set(range(n))
    rounds_of = {}
    sizes, fs = [n], [f_of(S, src, dst, c, a)]
    tau_max = Fraction(0)
    i, trims = 0, 0

    def w_of(S):
        f = f_of(S, src, dst, c, a)
        return {u: f - f_of(S - {u}, src, dst, c, a) for u in S}

    while S:
        f = f_of(S, src, dst, c, a)
        g = Fraction(f, len(S))
        tau_max = max(tau_max, g / (k * (1 + eps)))
        tau1 = max(tau_max, k * (1 + eps) * g)
        w = w_of(S)
        U1 = {u for u in S if w[u] <= tau1}
        i += 1
        for u in U1:
            rounds_of[u] = i
        S = S - U1
        if mode == "lpo":
            while S:
                w = w_of(S)
                gS = Fraction(f_of(S, src, dst, c, a), len(S))
                if not any(w[u] < gS for u in S):
                    break
                tau2 = max(tau_max, gS)
                U2 = {u for u in S if w[u] < tau2}
                for u in U2:
                    rounds_of[u] = i
                S = S - U2
                trims += 1
        sizes.append(len(S))
        fs.append(f_of(S, src, dst, c, a))
    best = max(range(len(sizes) - 1), key=lambda j: (Fraction(fs[j], sizes[j]), -j)) if n else 0
    return [rounds_of[u] for u in range(n)], sizes, fs, best, trims


@pytest.mark.parametrize("mode", ["gpo", "lpo"])
@pytest.mark.parametrize("block", range(3))
def test_optimised_oracle_matches_exact_simulation(mode, block):
    for seed in range(500 + block * 30, 500 + block * 30 + 30):
        n, src, dst, ew, vw = random_graph(seed, n_max=10)
        for metric in oracle.METRICS:
            c, a = oracle.metric_weights(metric, src, dst, n, ew, vw)
            num, den = EPS[seed % len(EPS)]
            r = oracle.peel_opt(n, src, dst, c, a, 2, num, den, mode=mode)
            pr, sizes, fs, best, trims = simulate_opt(n, src, dst, c, a, 2, Fraction(num, den), mode)
            assert r.peel_round.tolist() == pr, (seed, metric, mode)
            assert r.sizes.tolist() == sizes and r.f.tolist() == fs, (seed, metric, mode)
            assert r.best == best and r.trims == trims, (seed, metric, mode)


def test_plain_mode_is_algorithm_2():
    for seed in range(600, 660):
        n, src, dst, ew, vw = random_graph(seed)
        for metric in oracle.METRICS:
            c, a = oracle.metric_weights(metric, src, dst, n, ew, vw)
            num, den = EPS[seed % len(EPS)]
            r0 = oracle.peel(n, src, dst, c, a, 2, num, den)
            r1 = oracle.peel_opt(n, src, dst, c, a, 2, num, den, mode="plain")
            assert np.array_equal(r0.peel_round, r1.peel_round) and np.array_equal(r0.f, r1.f)
            assert r0.best == r1.best and r1.trims == 0


def test_optimisations_keep_the_guarantee():
    # the paper's claim that the approximation ratio of Theorem 4.2 holds for
    # both optimisations (Lemmas 5.1 and 5.3), against brute-force optima
    for seed in range(700, 760):
        n, src, dst, ew, vw = random_graph(seed, n_max=10)
        for metric in oracle.METRICS:
            c, a = oracle.metric_weights(metric, src, dst, n, ew, vw)
            opt = optimum(n, src, dst, c, a)
            for num, den in EPS:
                for mode in ("gpo", "lpo"):
                    r = oracle.peel_opt(n, src, dst, c, a, 2, num, den, mode=mode)
                    gp = Fraction(int(r.f[r.best]), int(r.sizes[r.best]))
                    assert gp * 2 * Fraction(den + num, den) >= opt, (seed, metric, mode, num, den)
                    S = set(r.best_set().tolist())
                    assert Fraction(f_of(S, src, dst, c, a), len(S)) == gp


def test_trimmed_sets_have_no_light_vertex():
    # the trimming loop stops only when no vertex of S_i weighs less than g(S_i)
    inp = workloads.peel_input("peel_rmat20", scale=12)
    n, src, dst = inp["n"], inp["src"].astype(np.int64), inp["dst"].astype(np.int64)
    for metric in oracle.METRICS:
        c, a = oracle.metric_weights(metric, inp["src"], inp["dst"], n, inp["edge_w"], inp["vertex_w"])
        r = oracle.peel_opt(n, inp["src"], inp["dst"], c, a, 2, 1, 10, mode="lpo")
        assert r.trims > 0
        for i in range(1, r.rounds):
            alive = r.peel_round > i
            both = alive[src] & alive[dst]
            w = a.astype(np.int64) + np.bincount(src[both], weights=c[both], minlength=n).astype(np.int64) + \
                np.bincount(dst[both], weights=c[both], minlength=n).astype(np.int64)
            s = int(alive.sum())
            f = int(a[alive].sum()) + int(c[both].sum())
            assert s == r.sizes[i] and f == r.f[i]
            assert (w[alive] * s >= f).all(), (metric, i)


def simulate_opt_fast(n, src, dst, c, a, k, num, den, mode):
    """Algorithms 3 and 4 again, vectorised: per-vertex weights by bin counts
    and the thresholds as exact integer floors and ceilings (w <= t for an
    integer w is w <= floor(t); w < t is w < ceil(t))."""
    src = src.astype(np.int64)
    dst = dst.astype(np.int64)
    alive = np.ones(n, bool)
    peel_round = np.zeros(n, np.int64)
    K = k * (den + num)                         # k (1 + eps) = K / den
    tA, tB = 0, 1                               # tau_max = tA / tB
    i, trims = 0, 0

    def state():
        both = alive[src] & alive[dst]
        w = a.astype(np.int64) + np.bincount(src[both], weights=c[both], minlength=n).astype(np.int64) + \
            np.bincount(dst[both], weights=c[both], minlength=n).astype(np.int64)
        return w, int(a[alive].sum()) + int(c[both].sum()), int(alive.sum())

    w, f, s = state()
    sizes, fs = [s], [f]
    while s:
        if mode != "plain" and f * den * tB > tA * s * K:
            tA, tB = f * den, s * K
        thr1 = max(tA // tB, (K * f) // (s * den))
        i += 1
        cut = alive & (w <= thr1)
        peel_round[cut] = i
        alive &= ~cut
        w, f, s = state()
        while mode == "lpo" and s and int(w[alive].min()) * s < f:
            thr2 = max(-(-tA // tB), -(-f // s))
            cut = alive & (w < thr2)
            peel_round[cut] = i
            alive &= ~cut
            trims += 1
            w, f, s = state()
        sizes.append(s)
        fs.append(f)
    best = max(range(len(sizes) - 1), key=lambda j: (Fraction(fs[j], sizes[j]), -j)) if n else 0
    return peel_round, sizes, fs, best, trims


def test_optimised_oracle_on_long_tails():
    # inputs with tails long enough for tau_max to bind (GPO changes the rounds)
    gpo_binds = False
    for name, scale in [("peel_chunglu10k", None), ("peel_rmat20", 14)]:
        inp = workloads.peel_input(name, scale=scale)
        n = inp["n"]
        for metric in oracle.METRICS:
            c, a = oracle.metric_weights(metric, inp["src"], inp["dst"], n, inp["edge_w"], inp["vertex_w"])
            plain = oracle.peel(n, inp["src"], inp["dst"], c, a, 2, 1, 10)
            for mode in ("gpo", "lpo"):
                r = oracle.peel_opt(n, inp["src"], inp["dst"], c, a, 2, 1, 10, mode=mode)
                pr, sizes, fs, best, trims = simulate_opt_fast(n, inp["src"], inp["dst"], c, a, 2, 1, 10, mode)
                assert np.array_equal(r.peel_round, pr), (name, metric, mode)
                assert r.sizes.tolist() == sizes and r.f.tolist() == fs, (name, metric, mode)
                assert r.best == best and r.trims == trims, (name, metric, mode)
                if mode == "gpo" and not np.array_equal(r.peel_round, plain.peel_round):
                    gpo_binds = True
                if mode == "lpo":
                    assert trims > 0
    assert gpo_binds


def powerlaw_graph(seed, n):
    """Skewed degrees and weights: long tails where the global threshold binds."""
    rnd = random.Random(seed)
    wts = [(i + 1) ** -0.8 for i in range(n)]
    rnd.shuffle(wts)
    src, dst = [], []
    m = rnd.randint(2 * n, 5 * n)
    while len(src) < m:
        u = rnd.choices(range(n), weights=wts)[0]
        v = rnd.choices(range(n), weights=wts)[0]
        if u != v:
            src.append(u)
            dst.append(v)
    ew = [rnd.choice([1, 2, 3, 5, 8, 50, 200]) for _ in src]
    vw = [rnd.randint(0, 1 << 24) if rnd.random() < 0.5 else 0 for _ in range(n)]
    return np.array(src, np.int32), np.array(dst, np.int32), np.array(ew, np.int64), np.array(vw, np.int64)


def test_global_threshold_reading():
    # an input on which g / (k (1 + eps)) and g / k as the refined threshold
    # give different rounds (found by search): the oracle must follow the
    # first, as the exact simulation does
    src, dst, ew, vw = powerlaw_graph(1495, 39)
    c, a = oracle.metric_weights("DW", src, dst, 39, ew, vw)
    r = oracle.peel_opt(39, src, dst, c, a, 2, 1, 10, mode="gpo")
    pr, sizes, fs, best, _ = simulate_opt(39, src, dst, c, a, 2, Fraction(1, 10), "gpo")
    assert r.peel_round.tolist() == pr and r.sizes.tolist() == sizes and r.best == best
    assert not np.array_equal(r.peel_round, oracle.peel(39, src, dst, c, a, 2, 1, 10).peel_round)


def test_trimming_is_strict():
    # no edges, vertex weights 0 (22 vertices), 1, 4, 7; k = 2, eps = 0.
    # Round 1: g = 12/25, the threshold 24/25 peels the 22 zeros; trimming
    # S = {1, 4, 7} (g = 4) removes only the 1 (4 is not below g), then
    # {4, 7} (g = 5.5) loses the 4: two trimming steps, S_1 = {7}.
    n = 25
    e = np.zeros(0, np.int32)
    a = np.array([0] * 22 + [1, 4, 7], np.int64)
    r = oracle.peel_opt(n, e, e, np.zeros(0, np.int64), a, 2, 0, 1, mode="lpo")
    assert r.trims == 2 and r.rounds == 2 and r.best == 1
    assert r.sizes.tolist() == [25, 1, 0] and r.f.tolist() == [12, 7, 0]
    assert r.peel_round.tolist() == [1] * 24 + [2]
