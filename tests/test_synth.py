"""The seeded generators: determinism, the RNG against its published
definition, and the structural promises each workload recipe makes."""
import numpy as np

from synth import gen, workloads

M64 = (1 << 64) - 1


def _splitmix64_next(state):
    # SplitMix64 (Steele, Lea, Flood 2014): advance by the golden gamma, then mix
    state = (state + 0x9E3779B97F4A7C15) & M64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return state, z ^ (z >> 31)


def test_counter_rng_is_splitmix64_sequence():
    # published reference value: state 0 -> first output 0xE220A8397B1DCDAF
    assert _splitmix64_next(0)[1] == 0xE220A8397B1DCDAF
    # counter c of a stream = the c-th output of sequential SplitMix64 seeded with the stream key
    for seed, stream in [(0, 1), (0x5EED0002, 7), (123456789, 15)]:
        state = gen.stream_key(seed, stream)
        for c in range(6):
            state, z = _splitmix64_next(state)
            assert gen.u64(seed, stream, c) == z


def test_generators_deterministic():
    a = gen.rmat_csr(12, 16 << 12, seed=5)
    b = gen.rmat_csr(12, 16 << 12, seed=5)
    c = gen.rmat_csr(12, 16 << 12, seed=6)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[1][:1000], c[1][:1000])
    la = gen.labels_zipf(1000, 50, 1.0, 1, 3, 9)
    lb = gen.labels_zipf(1000, 50, 1.0, 1, 3, 9)
    assert all(np.array_equal(x, y) for x, y in zip(la, lb))


def test_rmat_structure():
    rp, col = gen.rmat_csr(14, 16 << 14, seed=0x5EED0002)
    n = 1 << 14
    assert rp[0] == 0 and rp[-1] == col.shape[0] and np.all(np.diff(rp) >= 0)
    src = np.repeat(np.arange(n), np.diff(rp))
    assert not np.any(src == col)                      # no self-loops
    key = src.astype(np.int64) * n + col
    assert np.all(np.diff(key) > 0)                    # rows sorted, no duplicates
    assert 0.8 * (16 << 14) < col.shape[0] <= 16 << 14
    deg = np.bincount(col, minlength=n)
    assert deg.max() > 50 * deg.mean()                 # power-law hubs


def test_chung_lu_exact_edges():
    g = workloads.chunglu10k()
    assert g.n == 10_000 and g.m == 50_000
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    assert not np.any(src == g.col)
    assert np.unique(src.astype(np.int64) * g.n + g.col).shape[0] == 50_000


def test_labels_recipe():
    lp, lab = gen.labels_zipf(20_000, 500, 1.1, 1, 3, 0x5EED0101)
    cnt = np.diff(lp)
    assert cnt.min() == 1 and cnt.max() == 3
    assert abs(cnt.mean() - 2.0) < 0.05
    for v in range(0, 20_000, 997):
        row = lab[lp[v]:lp[v + 1]]
        assert np.all(np.diff(row) > 0) and row.min() >= 0 and row.max() < 500
    freq = np.sort(np.bincount(lab, minlength=500))[::-1]
    h = np.sum(1.0 / np.arange(1, 501) ** 1.1)
    # the most frequent label's share of first draws is 1/h (distinctness lowers it a little)
    assert 0.6 / h < freq[0] / lab.shape[0] < 1.2 / h


def test_type_tree_recipe():
    parent, leaves = gen.type_tree(8, 6, 0x5EED0104)
    assert parent.shape[0] == 299_593 and leaves.shape[0] == 262_144
    assert (parent == -1).sum() == 1
    # every leaf is at depth 6
    for leaf in leaves[:: 9973]:
        d, x = 0, int(leaf)
        while parent[x] >= 0:
            x, d = int(parent[x]), d + 1
        assert d == 6
    kids = np.bincount(parent[parent >= 0], minlength=parent.shape[0])
    assert set(np.unique(kids).tolist()) == {0, 8}


def test_queries_recipe():
    qs = workloads.rmat_flat_queries(256, 2, 8, [2, 3, 4], 20, cfg=2, qcfg=3)
    sizes = [len(q.kw) for q in qs]
    assert min(sizes) == 2 and max(sizes) == 8
    assert all(len(set(q.kw)) == len(q.kw) for q in qs)
    assert {q.d_max for q in qs} == {2, 3, 4}
    parent, leaves = gen.type_tree(8, 6, 0x5EED0104)
    hq = workloads.rmat_hier_queries(parent, leaves, 64)
    for q in hq:
        for t in q.kw:
            d, x = 0, t
            while parent[x] >= 0:
                x, d = int(parent[x]), d + 1
            assert 2 <= d <= 6


def test_arrivals_rate():
    t = gen.arrivals(20_000, 500.0, 3)
    assert np.all(np.diff(t) > 0)
    assert abs(20_000 / t[-1] - 500.0) < 25.0
