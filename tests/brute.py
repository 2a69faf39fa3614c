"""Independent checks for the oracle: brute force and a BFS certificate.

None of this shares code with ``oracle/``. The brute force walks the graph
the other way round (a breadth-first search *forward* from every vertex,
all pairs), finds keyword sets by walking the type tree *downwards*, and
does the ranking with Python's sort.
"""
from __future__ import annotations

from collections import deque

import numpy as np

INF = 255


def out_lists(g):
    rp, col = g.row_ptr, g.col
    return [col[rp[u]:rp[u + 1]].tolist() for u in range(g.n)]


def all_pairs(g):
    """D[r][v] = hop count of a shortest directed path r -> v (None if none)."""
    adj = out_lists(g)
    D = []
    for r in range(g.n):
        d = [None] * g.n
        d[r] = 0
        dq = deque([r])
        while dq:
            x = dq.popleft()
            for y in adj[x]:
                if d[y] is None:
                    d[y] = d[x] + 1
                    dq.append(y)
        D.append(d)
    return D


def descendants(parent, t):
    """t and every type below it, found top-down over child lists."""
    if parent is None:
        return {t}
    children = {}
    for c, p in enumerate(parent.tolist()):
        if p >= 0:
            children.setdefault(p, []).append(c)
    out, stack = set(), [t]
    while stack:
        x = stack.pop()
        if x in out:
            continue
        out.add(x)
        stack.extend(children.get(x, []))
    return out


def keyword_set(g, t):
    ok = descendants(g.type_parent, t)
    return {v for v in range(g.n)
            if any(int(l) in ok for l in g.lab[g.lab_ptr[v]:g.lab_ptr[v + 1]])}


def search(g, kw, d_max, k, D=None):
    """Full result by brute force: dict with kw, roots, scores, kw_dist, edges, te."""
    if D is None:
        D = all_pairs(g)
    K = sorted(set(int(x) for x in kw))
    adj = out_lists(g)
    indeg = np.bincount(g.col, minlength=g.n) if g.m else np.zeros(g.n, np.int64)
    dist = {}
    te = 0
    for t in K:
        S = keyword_set(g, t)
        d = []
        for r in range(g.n):
            best = min((D[r][v] for v in S if D[r][v] is not None), default=None)
            d.append(best if best is not None and best <= d_max else INF)
        dist[t] = d
        te += sum(int(indeg[x]) for x in range(g.n) if d[x] < d_max)
    roots = [r for r in range(g.n) if all(dist[t][r] <= d_max for t in K)]
    ranked = sorted(roots, key=lambda r: (sum(dist[t][r] for t in K), r))[:k]
    edges = []
    for r in ranked:
        es = set()
        for t in K:
            x = r
            while dist[t][x] > 0:
                y = min(w for w in adj[x] if dist[t][w] == dist[t][x] - 1)
                es.add((x, y))
                x = y
        edges.append(sorted(es))
    return dict(kw=K, roots=ranked, scores=[sum(dist[t][r] for t in K) for r in ranked],
                kw_dist=[[dist[t][r] for t in K] for r in ranked], edges=edges, te=te)


def certificate(row_ptr, col, in_set, dist, d_max):
    """Check that dist[] are the truncated BFS distances to in_set.

    The four conditions below hold for the true distances and, by
    induction on the level, only for them:
      1. dist == 0 exactly on in_set;
      2. every value is in {0..d_max} or INF;
      3. for every edge u -> w with dist[w] < d_max: dist[u] <= dist[w] + 1;
      4. every u with 0 < dist[u] <= d_max has an out-neighbour w with
         dist[w] == dist[u] - 1.
    Returns a list of violated condition numbers (empty = certified).
    """
    dist = np.asarray(dist).astype(np.int16)
    in_set = np.asarray(in_set, bool)
    n = dist.shape[0]
    bad = []
    if not np.array_equal(dist == 0, in_set):
        bad.append(1)
    if not np.all((dist <= d_max) | (dist == INF)):
        bad.append(2)
    row_ptr = np.asarray(row_ptr, np.int64)
    has = np.zeros(n, bool)
    chunk = 1 << 24                     # vertices per slice, keeps memory bounded at 1B edges
    for v0 in range(0, n, chunk):
        v1 = min(n, v0 + chunk)
        a, b = int(row_ptr[v0]), int(row_ptr[v1])
        src = np.repeat(np.arange(v0, v1, dtype=np.int64), np.diff(row_ptr[v0:v1 + 1]))
        dst = np.asarray(col[a:b], np.int64)
        dw, du = dist[dst], dist[src]
        sel = dw < d_max
        if 3 not in bad and np.any(du[sel] > dw[sel] + 1):
            bad.append(3)
        good_edge = (du >= 1) & (du <= d_max) & (dw == du - 1)
        has[src[good_edge]] = True
    need = (dist >= 1) & (dist <= d_max)
    if np.any(need & ~has):
        bad.append(4)
    return sorted(bad)
