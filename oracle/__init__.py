"""TEST INFRASTRUCTURE: the CPU oracles for distance-bounded keyword search
and for parallel peeling (densest subgraph discovery).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU
baseline may import this package. The GPU library never does, and the two
share no code. The arithmetic lives in ``kws_oracle.c`` (plain C, one
thread, one keyword at a time) and ``peel_oracle.c`` (plain C, one thread,
every round's sums recomputed from scratch); this module only marshals
arguments.

The definitions they implement, and the readings they adopt where the
paper is silent, are stated at the top of each C file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import List

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kws_oracle.c")
_SRC_PEEL = os.path.join(_HERE, "peel_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True, out: str = _LIB, defines=()) -> str:
    """Compile the oracle with gcc into ``out`` (in place by default)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, _SRC, _SRC_PEEL, "-lm"]
        cmd += ["-D" + d for d in defines]
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    return out


def _bind(lib):
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    lib.orc_graph_new.restype = C.c_void_p
    lib.orc_graph_new.argtypes = [C.c_int32, i32p, i32p, C.c_int32, i32p, i32p, C.c_void_p]
    lib.orc_graph_free.restype = None
    lib.orc_graph_free.argtypes = [C.c_void_p]
    lib.orc_keyword_set.restype = None
    lib.orc_keyword_set.argtypes = [C.c_void_p, C.c_int32, u8p]
    lib.orc_distances.restype = C.c_int64
    lib.orc_distances.argtypes = [C.c_void_p, C.c_int32, C.c_int32, u8p]
    lib.orc_search.restype = C.c_int
    lib.orc_search.argtypes = [C.c_void_p, i32p, C.c_int32, C.c_int32, C.c_int32,
                               C.POINTER(C.c_int32), i32p, C.POINTER(C.c_int32), i32p, i32p,
                               u8p, i64p, i32p, i32p, C.c_int64, C.POINTER(C.c_int64)]
    lib.orc_fd_weight.restype = C.c_int64
    lib.orc_fd_weight.argtypes = [C.c_int64]
    lib.orc_peel.restype = C.c_int
    lib.orc_peel.argtypes = [C.c_int32, C.c_int64, i32p, i32p, i64p, i64p, C.c_int32, C.c_int32, C.c_int32,
                             i32p, i64p, i64p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.orc_peel_opt.restype = C.c_int
    lib.orc_peel_opt.argtypes = [C.c_int32, C.c_int64, i32p, i32p, i64p, i64p, C.c_int32, C.c_int32, C.c_int32,
                                 C.c_int32, i32p, i64p, i64p, C.c_int32, C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.orc_peel_sequential.restype = C.c_int
    lib.orc_peel_sequential.argtypes = [C.c_int32, C.c_int64, i32p, i32p, i64p, i64p, u8p,
                                        C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    return lib


def load(path: str = _LIB):
    """Load (building if needed) an oracle shared library."""
    global _lib
    if path == _LIB:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=True)
            _lib = _bind(C.CDLL(_LIB))
        return _lib
    return _bind(C.CDLL(path))


@dataclass
class Result:
    """One query's answer, in the same shape the GPU library returns."""
    kw: List[int]             # unique keywords, ascending
    roots: np.ndarray         # int32 [n_roots], ordered by (score, id)
    scores: np.ndarray        # int32 [n_roots]
    kw_dist: np.ndarray       # uint8 [n_roots, len(kw)]
    edge_ptr: np.ndarray      # int64 [n_roots + 1]
    edge_src: np.ndarray      # int32
    edge_dst: np.ndarray      # int32
    te: int                   # scanned reverse edges (GTEPS numerator)

    def edges_of(self, i: int):
        a, b = int(self.edge_ptr[i]), int(self.edge_ptr[i + 1])
        return list(zip(self.edge_src[a:b].tolist(), self.edge_dst[a:b].tolist()))


class Oracle:
    """Owns an oracle-side copy of one graph (with its own reverse CSR)."""

    def __init__(self, graph, lib=None):
        self.lib = lib if lib is not None else load()
        self.g = graph
        rp = np.ascontiguousarray(graph.row_ptr, np.int32)
        col = np.ascontiguousarray(graph.col, np.int32)
        lp = np.ascontiguousarray(graph.lab_ptr, np.int32)
        lab = np.ascontiguousarray(graph.lab, np.int32)
        if col.shape[0] == 0:
            col = np.zeros(1, np.int32)
        if lab.shape[0] == 0:
            lab = np.zeros(1, np.int32)
        par = None
        if graph.type_parent is not None:
            self._par = np.ascontiguousarray(graph.type_parent, np.int32)
            par = self._par.ctypes.data
        self.h = self.lib.orc_graph_new(graph.n, rp, col, graph.n_labels, lp, lab, par)
        if not self.h:
            raise ValueError("oracle rejected the graph")

    def close(self):
        if self.h:
            self.lib.orc_graph_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def keyword_set(self, t: int) -> np.ndarray:
        out = np.empty(max(self.g.n, 1), np.uint8)
        self.lib.orc_keyword_set(self.h, t, out)
        return out[: self.g.n].astype(bool)

    def distances(self, t: int, d_max: int):
        """(dist uint8[n] with 255 = beyond d_max, scanned reverse edges)."""
        out = np.empty(max(self.g.n, 1), np.uint8)
        te = self.lib.orc_distances(self.h, t, d_max, out)
        return out[: self.g.n], int(te)

    def search(self, kw, d_max: int, k: int) -> Result:
        kwa = np.ascontiguousarray(np.asarray(kw, np.int32))
        nk = max(kwa.shape[0], 1)
        kk = max(k, 1)
        ukw = np.empty(nk, np.int32)
        roots = np.empty(kk, np.int32)
        scores = np.empty(kk, np.int32)
        kw_dist = np.empty(kk * nk, np.uint8)
        edge_ptr = np.zeros(kk + 1, np.int64)
        cap = kk * nk * max(d_max, 1) + 1
        es = np.empty(cap, np.int32)
        ed = np.empty(cap, np.int32)
        n_ukw, n_roots, te = C.c_int32(0), C.c_int32(0), C.c_int64(0)
        if kwa.shape[0] == 0:
            kwa = np.zeros(1, np.int32)
            nkw = 0
        else:
            nkw = kwa.shape[0]
        rc = self.lib.orc_search(self.h, kwa, nkw, d_max, k, C.byref(n_ukw), ukw, C.byref(n_roots),
                                 roots, scores, kw_dist, edge_ptr, es, ed, cap, C.byref(te))
        if rc != 0:
            raise ValueError(f"oracle search failed ({rc})")
        nr, nu = n_roots.value, n_ukw.value
        ne = int(edge_ptr[nr])
        return Result([int(x) for x in ukw[:nu]], roots[:nr].copy(), scores[:nr].copy(),
                      kw_dist[: nr * nu].reshape(nr, nu).copy(), edge_ptr[: nr + 1].copy(),
                      es[:ne].copy(), ed[:ne].copy(), int(te.value))


# ---------------------------------------------------------------- peeling

PEEL_ALIVE = 0x7FFFFFFF
METRICS = ("DG", "DW", "FD")


def fd_edge_weights(src: np.ndarray, dst: np.ndarray, n: int) -> np.ndarray:
    """FD edge weights (see peel_oracle.c): 1/ln(deg(src)+5) in 2^-24 units."""
    lib = load()
    deg = np.bincount(src, minlength=n) + np.bincount(dst, minlength=n)
    table = {}
    out = np.empty(src.shape[0], np.int64)
    for e, s in enumerate(src.tolist()):
        d = int(deg[s])
        if d not in table:
            table[d] = int(lib.orc_fd_weight(d))
        out[e] = table[d]
    return out


def metric_weights(metric: str, src, dst, n: int, edge_w=None, vertex_w=None):
    """(c, a) for a metric: DG unit edges; DW the given edge weights; FD
    the log-degree edge weights and the given vertex weights."""
    m = src.shape[0]
    if metric == "DG":
        return np.ones(m, np.int64), np.zeros(n, np.int64)
    if metric == "DW":
        return np.ascontiguousarray(edge_w, np.int64), np.zeros(n, np.int64)
    if metric == "FD":
        return fd_edge_weights(src, dst, n), np.ascontiguousarray(vertex_w, np.int64)
    raise ValueError(metric)


@dataclass
class PeelResult:
    peel_round: np.ndarray    # int32 [n], round in which each vertex is peeled (1-based)
    sizes: np.ndarray         # int64 [rounds + 1], |S_i|
    f: np.ndarray             # int64 [rounds + 1], f(S_i)
    rounds: int
    best: int                 # index i of the densest S_i

    def best_set(self) -> np.ndarray:
        return np.flatnonzero(self.peel_round > self.best).astype(np.int32)


def peel(n: int, src, dst, c, a, k: int = 2, eps_num: int = 1, eps_den: int = 10, cap: int = 0) -> PeelResult:
    """Parallel peeling rounds (peel_oracle.c: orc_peel)."""
    lib = load()
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    c = np.ascontiguousarray(c, np.int64)
    a = np.ascontiguousarray(a, np.int64)
    cap = cap or n + 2
    pr = np.empty(max(n, 1), np.int32)
    sizes = np.empty(cap, np.int64)
    fs = np.empty(cap, np.int64)
    r, b = C.c_int32(), C.c_int32()
    st = lib.orc_peel(n, src.shape[0], src, dst, c, a, k, eps_num, eps_den, pr, sizes, fs, cap,
                      C.byref(r), C.byref(b))
    if st != 0:
        raise ValueError(f"orc_peel failed ({st})")
    R = int(r.value)
    return PeelResult(pr[:n].copy(), sizes[:R + 1].copy(), fs[:R + 1].copy(), R, int(b.value))


PEEL_MODES = {"plain": 0, "gpo": 1, "lpo": 2}


def peel_opt(n: int, src, dst, c, a, k: int = 2, eps_num: int = 1, eps_den: int = 10, mode: str = "lpo",
             cap: int = 0) -> PeelResult:
    """Peeling with the global threshold (gpo, Algorithm 3) and the local
    trimming loop (lpo, Algorithm 4) (peel_oracle.c: orc_peel_opt); the
    result's ``trims`` attribute counts the trimming steps."""
    lib = load()
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    c = np.ascontiguousarray(c, np.int64)
    a = np.ascontiguousarray(a, np.int64)
    cap = cap or n + 2
    pr = np.empty(max(n, 1), np.int32)
    sizes = np.empty(cap, np.int64)
    fs = np.empty(cap, np.int64)
    r, b, t = C.c_int32(), C.c_int32(), C.c_int32()
    st = lib.orc_peel_opt(n, src.shape[0], src, dst, c, a, k, eps_num, eps_den, PEEL_MODES[mode], pr, sizes, fs,
                          cap, C.byref(r), C.byref(b), C.byref(t))
    if st != 0:
        raise ValueError(f"orc_peel_opt failed ({st})")
    R = int(r.value)
    res = PeelResult(pr[:n].copy(), sizes[:R + 1].copy(), fs[:R + 1].copy(), R, int(b.value))
    res.trims = int(t.value)
    return res


def peel_sequential(n: int, src, dst, c, a):
    """Sequential peeling (orc_peel_sequential): (set mask, f, size) of the result."""
    lib = load()
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    c = np.ascontiguousarray(c, np.int64)
    a = np.ascontiguousarray(a, np.int64)
    mask = np.empty(max(n, 1), np.uint8)
    bf, bs = C.c_int64(), C.c_int64()
    if lib.orc_peel_sequential(n, src.shape[0], src, dst, c, a, mask, C.byref(bf), C.byref(bs)) != 0:
        raise ValueError("orc_peel_sequential failed")
    return mask[:n].astype(bool), int(bf.value), int(bs.value)
