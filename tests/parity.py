"""Helpers shared by the GPU parity tests: run the oracle, compare results."""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle


def oracle_results(o, queries, workers: int = None):
    """Oracle answers for many queries; ctypes releases the GIL, so threads run in parallel."""
    workers = workers or min(16, os.cpu_count() or 1)
    if len(queries) <= 1 or workers <= 1:
        return [o.search(q.kw, q.d_max, q.k) for q in queries]
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda q: o.search(q.kw, q.d_max, q.k), queries))


def assert_same(got, want, ctx="", te=True):
    """Bit-exact comparison of one GPU result against the oracle's (te
    excluded when te=False: a query stopped early scans fewer edges)."""
    assert got.kw == want.kw, (ctx, "kw", got.kw, want.kw)
    assert np.array_equal(got.roots, want.roots), (ctx, "roots", got.roots[:20], want.roots[:20])
    assert np.array_equal(got.scores, want.scores), (ctx, "scores")
    assert np.array_equal(got.kw_dist, want.kw_dist), (ctx, "kw_dist")
    assert np.array_equal(got.edge_ptr, want.edge_ptr), (ctx, "edge_ptr", got.edge_ptr, want.edge_ptr)
    assert np.array_equal(got.edge_src, want.edge_src), (ctx, "edge_src")
    assert np.array_equal(got.edge_dst, want.edge_dst), (ctx, "edge_dst")
    if te:
        assert got.te == want.te, (ctx, "te", got.te, want.te)


def assert_all_same(gots, wants, ctx="", te=True):
    assert len(gots) == len(wants)
    for i, (a, b) in enumerate(zip(gots, wants)):
        assert_same(a, b, f"{ctx} query {i}", te=te)
