"""Small seeded graphs and queries for exhaustive checks.

Random tiny graphs keep the awkward cases in: self-loops, multi-edges,
isolated and unlabelled vertices, labels shared by many vertices, type
forests, duplicate query keywords, d_max from 0 up, and k of 0 or beyond n.
Plus a few hand-shaped graphs (path, complete digraph, no edges).
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from .gen import Graph, Query


def _csr(n: int, src, dst) -> Tuple[np.ndarray, np.ndarray]:
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    row_ptr = np.zeros(n + 1, np.int32)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return row_ptr, dst.astype(np.int32)


def from_edges(n: int, edges, labels: List[List[int]], n_labels: int, parent=None,
               name: str = "") -> Graph:
    src = [e[0] for e in edges]
    dst = [e[1] for e in edges]
    row_ptr, col = _csr(n, src, dst)
    lab_ptr = np.zeros(n + 1, np.int32)
    for v in range(n):
        lab_ptr[v + 1] = lab_ptr[v] + len(labels[v])
    lab = np.array([x for ls in labels for x in ls], np.int32)
    par = None if parent is None else np.asarray(parent, np.int32)
    return Graph(row_ptr, col, n_labels, lab_ptr, lab, par, name)


def random_forest(n_types: int, rng: np.random.Generator) -> np.ndarray:
    """Random type forest: parent[t] < t in a hidden order, then renamed."""
    order = rng.permutation(n_types)
    parent = np.full(n_types, -1, np.int32)
    for i in range(1, n_types):
        if rng.random() < 0.85:
            parent[order[i]] = order[rng.integers(0, i)]
    return parent


def random_graph(seed: int, n_max: int = 48, hier: bool = None) -> Graph:
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, n_max + 1))
    density = rng.choice([0.0, 0.03, 0.08, 0.2, 0.5])
    m = int(rng.poisson(density * n * n)) if density > 0 else 0
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    # some multi-edges and self-loops on purpose
    if m and rng.random() < 0.5:
        extra = rng.integers(0, m, max(1, m // 5))
        src = np.concatenate([src, src[extra]])
        dst = np.concatenate([dst, dst[extra]])
    if n and rng.random() < 0.5:
        v = rng.integers(0, n, 3)
        src = np.concatenate([src, v])
        dst = np.concatenate([dst, v])
    if hier is None:
        hier = bool(rng.random() < 0.4)
    n_labels = int(rng.integers(1, 9))
    parent = random_forest(n_labels, rng) if hier else None
    labels = []
    for _ in range(n):
        c = int(rng.choice([0, 1, 1, 2, 3]))
        c = min(c, n_labels)
        labels.append(sorted(rng.choice(n_labels, c, replace=False).tolist()))
    return from_edges(n, list(zip(src.tolist(), dst.tolist())), labels, n_labels, parent,
                      f"tiny{seed}")


def random_queries(g: Graph, seed: int, count: int = 4) -> List[Query]:
    rng = np.random.default_rng(seed ^ 0xABCDEF)
    out = []
    for _ in range(count):
        nk = int(rng.integers(1, 5))
        kw = rng.integers(0, g.n_labels, nk).tolist()
        if rng.random() < 0.3:
            kw.append(kw[0])            # duplicate keyword
        d_max = int(rng.choice([0, 1, 2, 3, 4, 6]))
        k = int(rng.choice([0, 1, 3, 10, g.n + 2]))
        out.append(Query(kw, d_max, k))
    return out


def path_graph(n: int) -> Graph:
    """0 -> 1 -> ... -> n-1, label 0 only on vertex n-1."""
    labels = [[] for _ in range(n)]
    labels[n - 1] = [0]
    return from_edges(n, [(i, i + 1) for i in range(n - 1)], labels, 1, name=f"path{n}")


def complete_digraph(n: int, seeds) -> Graph:
    """Every ordered pair (u, v), u != v; label 0 on the vertices in seeds."""
    labels = [[0] if v in seeds else [] for v in range(n)]
    edges = [(u, v) for u in range(n) for v in range(n) if u != v]
    return from_edges(n, edges, labels, 1, name=f"complete{n}")


def no_edges(n: int, labels: List[List[int]], n_labels: int) -> Graph:
    return from_edges(n, [], labels, n_labels, name=f"empty{n}")
