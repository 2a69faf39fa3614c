"""The named synthetic workloads (graph + labels + queries), fully seeded.

Recipes (sizes, distributions and seeds):

* ``chunglu10k``: directed Chung-Lu, exponent 2.1, 10,000 vertices and
  exactly 50,000 distinct non-loop edges; 500 labels Zipf(1.1), 1-3 per
  vertex; queries of 2 keywords, d_max=3, k=10 (the first is "the" query,
  the next 100 are for statistics).
* ``rmat20``: R-MAT(.57,.19,.19,.05), 2^20 vertices, 2^24 sampled edges
  (self-loops and duplicates dropped), seeded vertex permutation; 10,000
  labels Zipf(1.0), 1-3 per vertex.
    - ``rmat20_q4``: 100 queries x 4 keywords, d_max=3, k=20.
    - ``rmat20_batch256``: 256 queries, 2-8 keywords, d_max in {2,3,4}, k=20.
* ``rmat24_hier``: R-MAT 2^24 vertices, 2^28 samples; labels are leaves of a
  complete 8-ary type tree of depth 6 (299,593 types, 262,144 leaves), Zipf(1.0)
  over a permutation of the leaves, 1-3 per vertex; 512 queries of 2-6
  keywords, each the ancestor at depth U{2..6} of a Zipf-drawn leaf,
  d_max=3, k=50.
* ``rmat26_serve``: R-MAT 2^26 vertices, 2^30 samples; labels as rmat20;
  a Poisson stream of queries with 2-8 keywords, d_max in {2,3,4}, k=20.

``scale`` overrides shrink the R-MAT graphs for fast tests (same recipe,
fewer vertices; edge factor 16).

Peeling (densest-subgraph) inputs reuse these graphs as directed edge
lists and add weights from their own seed (graph seed + 0x400): DW edge
weights uniform on 1..1000 (stream 1), FD vertex weights uniform on
[0, 2^24) (stream 2, i.e. [0, 1) in 2^-24 units).

* ``peel_chunglu10k``: the chunglu10k graph.
* ``peel_rmat20``: the rmat20 graph (16,086,343 edges).
* ``peel_rmat24``: R-MAT 2^24 vertices, 2^28 samples (cfg 4 seeds).
"""
from __future__ import annotations

from typing import List, Optional, Tuple

from . import gen
from .gen import Graph, Query

SEED_BASE = 0x5EED0000
TREE_FANOUT, TREE_DEPTH = 8, 6


def _seeds(cfg: int):
    g = SEED_BASE + cfg
    return g, g + 0x100, g + 0x200, g + 0x300


def chunglu10k() -> Graph:
    sg, sl, _, _ = _seeds(1)
    rp, col = gen.chung_lu_csr(10_000, 50_000, 2.1, sg)
    lp, lab = gen.labels_zipf(10_000, 500, 1.1, 1, 3, sl)
    return Graph(rp, col, 500, lp, lab, None, "chunglu10k")


def chunglu10k_queries(count: int = 101) -> List[Query]:
    _, sl, sq, _ = _seeds(1)
    return gen.queries(count, 500, 1.1, 2, 2, [3], 10, sl, sq)


def rmat_flat(scale: int = 20, cfg: int = 2, n_labels: int = 10_000) -> Graph:
    sg, sl, _, _ = _seeds(cfg)
    rp, col = gen.rmat_csr(scale, 16 << scale, 0.57, 0.19, 0.19, sg)
    lp, lab = gen.labels_zipf(1 << scale, n_labels, 1.0, 1, 3, sl)
    return Graph(rp, col, n_labels, lp, lab, None, f"rmat{scale}")


def rmat_flat_queries(nq: int, mq_lo: int, mq_hi: int, dmax_set, k: int, cfg: int = 2,
                      qcfg: Optional[int] = None, n_labels: int = 10_000) -> List[Query]:
    _, sl, _, _ = _seeds(cfg)
    _, _, sq, _ = _seeds(cfg if qcfg is None else qcfg)
    return gen.queries(nq, n_labels, 1.0, mq_lo, mq_hi, dmax_set, k, sl, sq)


def rmat20_q4(scale: int = 20, nq: int = 100) -> Tuple[Graph, List[Query]]:
    g = rmat_flat(scale, 2)
    return g, rmat_flat_queries(nq, 4, 4, [3], 20, cfg=2)


def rmat20_batch256(scale: int = 20, nq: int = 256) -> Tuple[Graph, List[Query]]:
    g = rmat_flat(scale, 2)
    return g, rmat_flat_queries(nq, 2, 8, [2, 3, 4], 20, cfg=2, qcfg=3)


def rmat_hier(scale: int = 24, cfg: int = 4, fanout: int = TREE_FANOUT,
              depth: int = TREE_DEPTH) -> Tuple[Graph, "object"]:
    sg, sl, _, _ = _seeds(cfg)
    parent, leaves = gen.type_tree(fanout, depth, sl)
    rp, col = gen.rmat_csr(scale, 16 << scale, 0.57, 0.19, 0.19, sg)
    lp, leaf_idx = gen.labels_zipf(1 << scale, leaves.shape[0], 1.0, 1, 3, sl)
    lab = leaves[leaf_idx]
    g = Graph(rp, col, int(parent.shape[0]), lp, lab, parent, f"rmat{scale}_hier")
    return g, leaves


def rmat_hier_queries(parent, leaves, nq: int = 512, cfg: int = 4, k: int = 50,
                      depth: int = TREE_DEPTH) -> List[Query]:
    _, sl, sq, _ = _seeds(cfg)
    return gen.queries(nq, int(leaves.shape[0]), 1.0, 2, 6, [3], k, sl, sq,
                       leaf_ids=leaves, parent=parent, leaf_depth=depth,
                       hd_lo=min(2, depth), hd_hi=depth)


def rmat24_hier(scale: int = 24, nq: int = 512) -> Tuple[Graph, List[Query]]:
    g, leaves = rmat_hier(scale, 4)
    return g, rmat_hier_queries(g.type_parent, leaves, nq, 4)


def rmat26_serve(scale: int = 26, nq: int = 4096) -> Tuple[Graph, List[Query]]:
    g = rmat_flat(scale, 5)
    return g, rmat_flat_queries(nq, 2, 8, [2, 3, 4], 20, cfg=5)


def serve_arrivals(count: int, lam: float):
    _, _, _, sa = _seeds(5)
    return gen.arrivals(count, lam, sa)


# ---------------------------------------------------------------- peeling

def peel_input(name: str, scale: Optional[int] = None) -> dict:
    """A peeling input: n, src, dst (int32 edge list), edge_w (DW), vertex_w (FD)."""
    import numpy as np
    if name == "peel_chunglu10k":
        g, cfg = chunglu10k(), 1
    elif name == "peel_rmat20":
        sc = scale or 20
        cfg = 2
        gs, _, _, _ = _seeds(cfg)
        rp, col = gen.rmat_csr(sc, 16 << sc, seed=gs)
        g = Graph(rp, col, 1, np.zeros(rp.shape[0], np.int32), np.zeros(0, np.int32), None, f"rmat{sc}")
    elif name == "peel_rmat24":
        sc = scale or 24
        cfg = 4
        gs, _, _, _ = _seeds(cfg)
        rp, col = gen.rmat_csr(sc, 16 << sc, seed=gs)
        g = Graph(rp, col, 1, np.zeros(rp.shape[0], np.int32), np.zeros(0, np.int32), None, f"rmat{sc}")
    else:
        raise ValueError(name)
    n = g.n
    src = np.repeat(np.arange(n, dtype=np.int32), np.diff(g.row_ptr).astype(np.int64))
    dst = np.ascontiguousarray(g.col, np.int32)
    ws = SEED_BASE + cfg + 0x400
    return dict(name=name, n=n, src=src, dst=dst,
                edge_w=gen.uniform_i64(ws, 1, src.shape[0], 1, 1000),
                vertex_w=gen.uniform_i64(ws, 2, n, 0, (1 << 24) - 1))
