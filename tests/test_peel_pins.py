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


def test_uniform_generator():
    x = gen.uniform_i64(7, 1, 20000, 1, 1000)
    assert x.min() >= 1 and x.max() <= 1000 and abs(x.mean() - 500.5) < 10
    assert np.array_equal(x, gen.uniform_i64(7, 1, 20000, 1, 1000))
    assert not np.array_equal(x, gen.uniform_i64(7, 2, 20000, 1, 1000))
