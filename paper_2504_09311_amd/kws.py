"""Thin ctypes binding of ``libkws.so`` (declared in ``include/kws.h``).

Argument marshalling only: every step of a search runs in the library's
HIP kernels. The names follow the C entry points without the ``kws_``
prefix. Importing this module never falls back to anything else: if the
built library is missing, ``load_library`` raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkws.so")

OK, EINVAL, ENOMEM, EDEVICE, EOVERFLOW, EBUSY, ECANCELLED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EOVERFLOW", -5: "EBUSY",
                -6: "ECANCELLED"}
MAX_KW, MAX_DMAX, MAX_K, DIST_INF = 64, 15, 65536, 255
MAX_LEVELS = 15


class KwsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class GraphDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int64), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("n_labels", C.c_int32), ("lab_ptr", C.c_void_p), ("lab", C.c_void_p),
                ("type_parent", C.c_void_p)]


class QueryC(C.Structure):
    _fields_ = [("kw", C.c_void_p), ("n_kw", C.c_int32), ("d_max", C.c_int32), ("k", C.c_int32)]


class ResultC(C.Structure):
    _fields_ = [("n_roots", C.c_int32), ("n_kw", C.c_int32), ("kw", C.POINTER(C.c_int32)),
                ("roots", C.POINTER(C.c_int32)), ("scores", C.POINTER(C.c_int32)),
                ("kw_dist", C.POINTER(C.c_uint8)), ("edge_ptr", C.POINTER(C.c_int64)),
                ("edge_src", C.POINTER(C.c_int32)), ("edge_dst", C.POINTER(C.c_int32)),
                ("te", C.c_int64)]


class BatchResultC(C.Structure):
    _fields_ = [("nq", C.c_int32), ("total_roots", C.c_int64), ("root_ptr", C.POINTER(C.c_int64)),
                ("roots", C.POINTER(C.c_int32)), ("scores", C.POINTER(C.c_int32)),
                ("kw_ptr", C.POINTER(C.c_int64)), ("kw", C.POINTER(C.c_int32)),
                ("dist_ptr", C.POINTER(C.c_int64)), ("kw_dist", C.POINTER(C.c_uint8)),
                ("edge_ptr", C.POINTER(C.c_int64)), ("edge_src", C.POINTER(C.c_int32)),
                ("edge_dst", C.POINTER(C.c_int32)), ("te", C.POINTER(C.c_int64))]


class Options(C.Structure):
    _fields_ = [("direction", C.c_int32), ("alpha", C.c_float), ("tile_words", C.c_int32),
                ("block", C.c_int32), ("use_graph", C.c_int32), ("share_lanes", C.c_int32),
                ("count_te", C.c_int32), ("seed_mode", C.c_int32), ("fused_pull", C.c_int32),
                ("early_stop", C.c_int32), ("seed_table", C.c_int32)]


class DsdDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int64), ("src", C.c_void_p), ("dst", C.c_void_p),
                ("edge_w", C.c_void_p), ("vertex_w", C.c_void_p), ("metric", C.c_int32)]


class DsdParams(C.Structure):
    _fields_ = [("k", C.c_int32), ("eps_num", C.c_int32), ("eps_den", C.c_int32), ("profile", C.c_int32),
                ("mode", C.c_int32), ("profile_classes", C.c_int32)]


class DsdSummary(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("best", C.c_int32), ("best_size", C.c_int64), ("best_f", C.c_int64),
                ("incidences", C.c_int64), ("decide_ms", C.c_double), ("update_ms", C.c_double),
                ("reduce_ms", C.c_double), ("decide_launches", C.c_int64), ("update_launches", C.c_int64),
                ("reduce_launches", C.c_int64), ("trims", C.c_int64), ("steps", C.c_int64)]


class TuneReport(C.Structure):
    _fields_ = [("configs_tried", C.c_int32), ("best_ms", C.c_double), ("default_ms", C.c_double),
                ("from_cache", C.c_int32)]


class GraphInfo(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int64), ("n_labels", C.c_int32), ("hierarchical", C.c_int32),
                ("device_bytes", C.c_int64), ("max_out_degree", C.c_int32), ("max_in_degree", C.c_int32),
                ("graph_captures", C.c_int64), ("graph_replays", C.c_int64)]


class BatchStats(C.Structure):
    _fields_ = [("queries", C.c_int32), ("lanes", C.c_int32), ("lane_slots", C.c_int32),
                ("words", C.c_int32), ("words_padded", C.c_int32), ("tiles", C.c_int32),
                ("tile_words", C.c_int32), ("levels", C.c_int32), ("passes", C.c_int32),
                ("pulled", C.c_int32 * (MAX_LEVELS + 1)), ("frontier", C.c_int64 * (MAX_LEVELS + 1)),
                ("frontier_edges", C.c_int64 * (MAX_LEVELS + 1)),
                ("unfinished_edges", C.c_int64 * (MAX_LEVELS + 1)),
                ("fused_pull", C.c_int32), ("early_stopped", C.c_int64), ("levels_skipped", C.c_int64),
                ("seed_table", C.c_int32)]

    def as_dict(self):
        L = self.levels
        return dict(queries=self.queries, lanes=self.lanes, lane_slots=self.lane_slots, words=self.words,
                    words_padded=self.words_padded, tiles=self.tiles, tile_words=self.tile_words,
                    levels=L, passes=self.passes, pulled=list(self.pulled[:L]),
                    frontier=list(self.frontier[:L + 1]), frontier_edges=list(self.frontier_edges[:L + 1]),
                    unfinished_edges=list(self.unfinished_edges[:L + 1]),
                    fused_pull=self.fused_pull, early_stopped=self.early_stopped,
                    levels_skipped=self.levels_skipped, seed_table=self.seed_table)


class ServerOpts(C.Structure):
    _fields_ = [("max_words", C.c_int32), ("max_dmax", C.c_int32), ("queue_capacity", C.c_int32),
                ("tile_words", C.c_int32), ("mem_bytes", C.c_int64)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("cancelled", C.c_int64),
                ("rejected", C.c_int64), ("steps", C.c_int64), ("queued", C.c_int32),
                ("active_words", C.c_int32), ("max_words", C.c_int32), ("elapsed_s", C.c_double),
                ("qps", C.c_double), ("p50_us", C.c_double), ("p99_us", C.c_double),
                ("mean_active_words", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_lib = None


def load_library(path: str = LIB_PATH):
    """Load the built HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2504_09311_amd/build.py "
                           "(or __graft_entry__.build()) before use")
    lib = C.CDLL(path)
    P = C.c_void_p
    sigs = {
        "kws_load_graph": (C.c_int, [C.POINTER(GraphDesc), C.POINTER(P)]),
        "kws_free_graph": (None, [P]),
        "kws_keyword_search": (C.c_int, [P, C.POINTER(QueryC), C.POINTER(ResultC)]),
        "kws_search_batch": (C.c_int, [P, C.POINTER(QueryC), C.c_int32, C.POINTER(ResultC)]),
        "kws_result_free": (None, [C.POINTER(ResultC)]),
        "kws_search_batch_flat": (C.c_int, [P, C.POINTER(QueryC), C.c_int32, C.POINTER(BatchResultC)]),
        "kws_batch_result_free": (None, [C.POINTER(BatchResultC)]),
        "kws_search_batch_submit": (C.c_int, [P, C.POINTER(QueryC), C.c_int32, C.POINTER(C.c_int64)]),
        "kws_search_batch_collect": (C.c_int, [P, C.c_int64, C.POINTER(BatchResultC)]),
        "kws_debug_distances": (C.c_int, [P, C.c_int32, C.c_int32, P]),
        "kws_debug_distances_noalloc": (C.c_int, [P, C.c_int32, C.c_int32, P]),
        "kws_set_options": (C.c_int, [P, C.POINTER(Options)]),
        "kws_get_options": (C.c_int, [P, C.POINTER(Options)]),
        "kws_set_stream": (C.c_int, [P, P]),
        "kws_get_stream": (P, [P]),
        "kws_set_allocator": (C.c_int, [P, P, P]),
        "kws_set_mem_limit": (C.c_int, [C.c_int64]),
        "kws_mem_in_use": (C.c_int64, []),
        "kws_graph_info_get": (C.c_int, [P, C.POINTER(GraphInfo)]),
        "kws_profile_enable": (C.c_int, [P, C.c_int32]),
        "kws_profile_reset": (C.c_int, [P]),
        "kws_profile_classes": (C.c_int, [P, C.c_uint64]),
        "kws_profile_read": (C.c_int, [P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
        "kws_profile_name": (C.c_char_p, [C.c_int32]),
        "kws_last_batch_stats": (C.c_int, [P, C.POINTER(BatchStats)]),
        "kws_last_error": (C.c_char_p, []),
        "kws_autotune": (C.c_int, [P, C.POINTER(QueryC), C.c_int32, C.c_int32, C.c_double, C.c_char_p,
                                   C.POINTER(Options), C.POINTER(TuneReport)]),
        "kws_server_create": (C.c_int, [P, C.POINTER(ServerOpts), C.POINTER(P)]),
        "kws_server_submit": (C.c_int, [P, C.POINTER(QueryC), C.POINTER(C.c_uint64)]),
        "kws_server_poll": (C.c_int, [P, C.c_uint64, C.POINTER(ResultC), C.POINTER(C.c_int32)]),
        "kws_server_wait": (C.c_int, [P, C.c_uint64, C.c_int64, C.POINTER(ResultC), C.POINTER(C.c_int32)]),
        "kws_server_cancel": (C.c_int, [P, C.c_uint64]),
        "kws_server_stats_get": (C.c_int, [P, C.POINTER(ServerStats)]),
        "kws_server_destroy": (None, [P]),
        "kws_dsd_load": (C.c_int, [C.POINTER(DsdDesc), C.POINTER(P)]),
        "kws_dsd_free": (None, [P]),
        "kws_dsd_peel": (C.c_int, [P, C.POINTER(DsdParams), P, P, P, C.c_int32, C.POINTER(DsdSummary)]),
        "kws_dsd_rounds": (C.c_int, [P, P, C.POINTER(P)]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def declared_symbols() -> List[str]:
    """The function names the headers in include/ declare (parsed from them)."""
    import re
    inc = os.path.join(os.path.dirname(HERE), "include")
    text = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    return sorted(set(re.findall(r"\b(kws_[a-z_]+)\s*\(", text)))


def set_mem_limit(nbytes: int) -> None:
    """Process-wide cap on the library's device memory (negative: no cap)."""
    _check(load_library().kws_set_mem_limit(int(nbytes)))


def mem_in_use() -> int:
    """Device bytes the library holds right now."""
    return int(load_library().kws_mem_in_use())


def last_error() -> str:
    return (load_library().kws_last_error() or b"").decode()


def _check(st: int):
    if st != OK:
        raise KwsError(st, last_error())


@dataclass
class Result:
    """One query's answer (same fields as the C kws_result, as numpy arrays)."""
    kw: List[int]
    roots: np.ndarray
    scores: np.ndarray
    kw_dist: np.ndarray
    edge_ptr: np.ndarray
    edge_src: np.ndarray
    edge_dst: np.ndarray
    te: int

    def edges_of(self, i: int):
        a, b = int(self.edge_ptr[i]), int(self.edge_ptr[i + 1])
        return list(zip(self.edge_src[a:b].tolist(), self.edge_dst[a:b].tolist()))


def _take(r: ResultC) -> Result:
    nr, nk = r.n_roots, r.n_kw
    ne = int(r.edge_ptr[nr]) if r.edge_ptr else 0

    def arr(ptr, count, dt):
        if count == 0 or not ptr:
            return np.zeros(0, dt)
        return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dt, copy=True)

    return Result([int(x) for x in arr(r.kw, nk, np.int32)], arr(r.roots, nr, np.int32),
                  arr(r.scores, nr, np.int32), arr(r.kw_dist, nr * nk, np.uint8).reshape(nr, nk),
                  arr(r.edge_ptr, nr + 1, np.int64), arr(r.edge_src, ne, np.int32),
                  arr(r.edge_dst, ne, np.int32), int(r.te))


def _queries(qs) -> tuple:
    keep, arr = [], (QueryC * max(1, len(qs)))()
    for i, q in enumerate(qs):
        kw, d_max, k = (q.kw, q.d_max, q.k) if hasattr(q, "kw") else q
        a = np.ascontiguousarray(np.asarray(kw, np.int32))
        keep.append(a)
        arr[i].kw = a.ctypes.data if a.size else None
        arr[i].n_kw = int(a.size)
        arr[i].d_max = int(d_max)
        arr[i].k = int(k)
    return arr, keep


class Graph:
    """A graph resident on the device (wraps a kws_graph handle)."""

    def __init__(self, row_ptr, col, n_labels: int, lab_ptr, lab, type_parent=None):
        lib = load_library()
        self._lib = lib
        self._arrs = [np.ascontiguousarray(np.asarray(x, np.int32)) for x in (row_ptr, col, lab_ptr, lab)]
        rp, cl, lp, lb = self._arrs
        tp = None
        if type_parent is not None:
            tp = np.ascontiguousarray(np.asarray(type_parent, np.int32))
            self._arrs.append(tp)
        d = GraphDesc(int(rp.shape[0] - 1), int(cl.shape[0]), rp.ctypes.data, cl.ctypes.data if cl.size else None,
                      int(n_labels), lp.ctypes.data, lb.ctypes.data if lb.size else None,
                      tp.ctypes.data if tp is not None else None)
        h = C.c_void_p()
        _check(lib.kws_load_graph(C.byref(d), C.byref(h)))
        self.h = h
        self._pending = {}
        self._arrs = None          # the library keeps its own copies
        self.set_options()         # binding default: count te

    @classmethod
    def from_synth(cls, g) -> "Graph":
        return cls(g.row_ptr, g.col, g.n_labels, g.lab_ptr, g.lab, g.type_parent)

    def close(self):
        if getattr(self, "h", None):
            self._lib.kws_free_graph(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- searches
    def keyword_search(self, kw: Sequence[int], d_max: int, k: int) -> Result:
        qa, keep = _queries([(kw, d_max, k)])
        r = ResultC()
        _check(self._lib.kws_keyword_search(self.h, qa, C.byref(r)))
        try:
            return _take(r)
        finally:
            self._lib.kws_result_free(C.byref(r))

    def search_batch_each(self, queries) -> List[Result]:
        """kws_search_batch: one separately allocated result per query."""
        qa, keep = _queries(queries)
        n = len(queries)
        rs = (ResultC * max(1, n))()
        _check(self._lib.kws_search_batch(self.h, qa, n, rs))
        try:
            return [_take(rs[i]) for i in range(n)]
        finally:
            for i in range(n):
                self._lib.kws_result_free(C.byref(rs[i]))

    def search_batch_flat(self, queries) -> dict:
        """kws_search_batch_flat: the whole batch as flat numpy arrays."""
        qa, keep = _queries(queries)
        n = len(queries)
        r = BatchResultC()
        _check(self._lib.kws_search_batch_flat(self.h, qa, n, C.byref(r)))
        return self._flat(r, n)

    def search_batch_submit(self, queries) -> int:
        """kws_search_batch_submit: enqueue a batch and return its ticket without waiting."""
        qa, keep = _queries(queries)
        t = C.c_int64()
        _check(self._lib.kws_search_batch_submit(self.h, qa, len(queries), C.byref(t)))
        self._pending[int(t.value)] = len(queries)
        return int(t.value)

    def search_batch_collect(self, ticket: int) -> dict:
        """kws_search_batch_collect: wait for a submitted batch; same layout as search_batch_flat."""
        r = BatchResultC()
        _check(self._lib.kws_search_batch_collect(self.h, int(ticket), C.byref(r)))
        return self._flat(r, self._pending.pop(int(ticket)))

    def _flat(self, r, n: int) -> dict:
        try:
            nr = int(r.total_roots)

            def arr(ptr, count, dt):
                if count == 0:
                    return np.zeros(0, dt)
                return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dt, copy=True)

            root_ptr = arr(r.root_ptr, n + 1, np.int64)
            kw_ptr = arr(r.kw_ptr, n + 1, np.int64)
            dist_ptr = arr(r.dist_ptr, n + 1, np.int64)
            edge_ptr = arr(r.edge_ptr, nr + 1, np.int64)
            ne = int(edge_ptr[-1]) if nr else 0
            return dict(root_ptr=root_ptr, roots=arr(r.roots, nr, np.int32), scores=arr(r.scores, nr, np.int32),
                        kw_ptr=kw_ptr, kw=arr(r.kw, int(kw_ptr[-1]), np.int32), dist_ptr=dist_ptr,
                        kw_dist=arr(r.kw_dist, int(dist_ptr[-1]), np.uint8), edge_ptr=edge_ptr,
                        edge_src=arr(r.edge_src, ne, np.int32), edge_dst=arr(r.edge_dst, ne, np.int32),
                        te=arr(r.te, n, np.int64))
        finally:
            self._lib.kws_batch_result_free(C.byref(r))

    @staticmethod
    def results_of(f: dict, n: int) -> List["Result"]:
        """Per-query Result views cut from a flat batch output."""
        out = []
        for q in range(n):
            a, b = int(f["root_ptr"][q]), int(f["root_ptr"][q + 1])
            kw = f["kw"][f["kw_ptr"][q]:f["kw_ptr"][q + 1]]
            kd = f["kw_dist"][f["dist_ptr"][q]:f["dist_ptr"][q + 1]].reshape(b - a, kw.shape[0])
            ep = f["edge_ptr"][a:b + 1]
            e0, e1 = int(ep[0]), int(ep[-1])
            out.append(Result([int(x) for x in kw], f["roots"][a:b], f["scores"][a:b], kd, ep - e0,
                              f["edge_src"][e0:e1], f["edge_dst"][e0:e1], int(f["te"][q])))
        return out

    def search_batch(self, queries) -> List[Result]:
        """Batched search; per-query Result views cut from the flat output."""
        return self.results_of(self.search_batch_flat(queries), len(queries))

    def debug_distances(self, kw: int, d_max: int) -> np.ndarray:
        n = self.info().n
        out = np.empty(n, np.uint8)
        _check(self._lib.kws_debug_distances(self.h, int(kw), int(d_max), out.ctypes.data))
        return out

    def debug_distances_noalloc(self, kw: int, d_max: int, dist_dev_ptr: int) -> None:
        """kws_debug_distances_noalloc: distances into a caller-owned device
        buffer of n bytes (an integer device address), allocating nothing."""
        _check(self._lib.kws_debug_distances_noalloc(self.h, int(kw), int(d_max), C.c_void_p(int(dist_dev_ptr))))

    # ---- configuration and introspection
    def set_options(self, direction: int = 0, alpha: float = 0.0, tile_words: int = 0, use_graph: int = 0,
                    share_lanes: int = 0, count_te: int = 1, seed_mode: int = 0, fused_pull: int = 0,
                    early_stop: int = -1, seed_table: int = 0):
        """Engine options (kws_set_options). count_te defaults to on and early_stop to off here, so
        that te is the full per-keyword scan count (a query that stops early counts fewer edges)."""
        o = Options(direction, alpha, tile_words, 0, use_graph, share_lanes, count_te, seed_mode, fused_pull,
                    early_stop, seed_table)
        _check(self._lib.kws_set_options(self.h, C.byref(o)))

    def autotune(self, queries, reps: int = 3, budget_ms: float = 0.0, cache_path: Optional[str] = None):
        """Time the sample batch under a grid of options, keep the fastest (see kws_autotune)."""
        qa, keep = _queries(queries)
        o, rep = Options(), TuneReport()
        _check(self._lib.kws_autotune(self.h, qa, len(queries), reps, budget_ms,
                                      cache_path.encode() if cache_path else None, C.byref(o), C.byref(rep)))
        return ({k: getattr(o, k) for k, _ in o._fields_}, {k: getattr(rep, k) for k, _ in rep._fields_})

    def get_options(self) -> Options:
        o = Options()
        _check(self._lib.kws_get_options(self.h, C.byref(o)))
        return o

    def set_stream(self, stream_ptr: Optional[int]):
        _check(self._lib.kws_set_stream(self.h, stream_ptr))

    def get_stream(self) -> int:
        return int(self._lib.kws_get_stream(self.h) or 0)

    def info(self) -> GraphInfo:
        i = GraphInfo()
        _check(self._lib.kws_graph_info_get(self.h, C.byref(i)))
        return i

    def profile_enable(self, on: bool = True):
        _check(self._lib.kws_profile_enable(self.h, 1 if on else 0))

    def profile_reset(self):
        _check(self._lib.kws_profile_reset(self.h))

    def profile_classes(self, names=None):
        """Time only these kernel classes with events (None: every class)."""
        mask = 0
        if names:
            ids = {}
            i = 0
            while True:
                nm = self._lib.kws_profile_name(i)
                if not nm:
                    break
                ids[nm.decode()] = i
                i += 1
            for n in names:
                mask |= 1 << ids[n]
        _check(self._lib.kws_profile_classes(self.h, mask))

    def profile_read(self) -> dict:
        out = {}
        i = 0
        while True:
            name = self._lib.kws_profile_name(i)
            if not name:
                break
            n, ms = C.c_int64(), C.c_double()
            _check(self._lib.kws_profile_read(self.h, i, C.byref(n), C.byref(ms)))
            out[name.decode()] = (int(n.value), float(ms.value))
            i += 1
        return out

    def last_batch_stats(self) -> BatchStats:
        s = BatchStats()
        _check(self._lib.kws_last_batch_stats(self.h, C.byref(s)))
        return s


class Server:
    """Continuous-batching server over a resident Graph (wraps kws_server)."""

    def __init__(self, graph: Graph, max_words: int = 0, max_dmax: int = 0, queue_capacity: int = 0,
                 tile_words: int = 0, mem_bytes: int = 0):
        self._lib = load_library()
        self.graph = graph
        o = ServerOpts(max_words, max_dmax, queue_capacity, tile_words, mem_bytes)
        h = C.c_void_p()
        _check(self._lib.kws_server_create(graph.h, C.byref(o), C.byref(h)))
        self.h = h

    def submit(self, kw, d_max: int, k: int) -> int:
        qa, keep = _queries([(kw, d_max, k)])
        t = C.c_uint64()
        _check(self._lib.kws_server_submit(self.h, qa, C.byref(t)))
        return int(t.value)

    def _finish(self, st, r, done):
        _check(st)
        if not done.value:
            return None
        try:
            return _take(r)
        finally:
            self._lib.kws_result_free(C.byref(r))

    def poll(self, ticket: int) -> Optional[Result]:
        r, done = ResultC(), C.c_int32()
        return self._finish(self._lib.kws_server_poll(self.h, ticket, C.byref(r), C.byref(done)), r, done)

    def wait(self, ticket: int, timeout_s: Optional[float] = None) -> Optional[Result]:
        r, done = ResultC(), C.c_int32()
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        return self._finish(self._lib.kws_server_wait(self.h, ticket, us, C.byref(r), C.byref(done)), r, done)

    def cancel(self, ticket: int):
        _check(self._lib.kws_server_cancel(self.h, ticket))

    def stats(self) -> dict:
        st = ServerStats()
        _check(self._lib.kws_server_stats_get(self.h, C.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "h", None):
            self._lib.kws_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PeelGraph:
    """Densest-subgraph discovery by parallel peeling (wraps include/dsd.h)."""
    METRICS = {"DG": 0, "DW": 1, "FD": 2}

    def __init__(self, n: int, src, dst, metric: str, edge_w=None, vertex_w=None):
        lib = load_library()
        self._lib = lib
        self.n = int(n)
        src = np.ascontiguousarray(src, np.int32)
        dst = np.ascontiguousarray(dst, np.int32)
        ew = np.ascontiguousarray(edge_w, np.int64) if edge_w is not None and metric == "DW" else None
        vw = np.ascontiguousarray(vertex_w, np.int64) if vertex_w is not None and metric == "FD" else None
        d = DsdDesc(self.n, int(src.shape[0]), src.ctypes.data if src.size else None,
                    dst.ctypes.data if dst.size else None, ew.ctypes.data if ew is not None else None,
                    vw.ctypes.data if vw is not None else None, self.METRICS[metric])
        h = C.c_void_p()
        _check(lib.kws_dsd_load(C.byref(d), C.byref(h)))
        self.h = h

    MODES = {"plain": 0, "gpo": 1, "lpo": 2}

    PROFILE_CLASSES = {"decide": 1, "update": 2, "reduce": 4}

    def peel(self, k: int = 2, eps_num: int = 1, eps_den: int = 10, profile=False, cap: int = 0,
             rounds: bool = True, mode: str = "plain"):
        """(peel_round[n], sizes[R+1], f[R+1], summary dict) of one run.

        mode: "plain" (Algorithm 2), "gpo" (global threshold, Algorithm 3)
        or "lpo" (and local trimming, Algorithm 4). profile: True times every
        kernel class with events, a list of class names times only those.
        rounds=False leaves the peel rounds in device memory (None is
        returned in their place; ``rounds()`` fetches them later)."""
        cap = cap or 65536
        sizes = np.empty(cap, np.int64)
        fs = np.empty(cap, np.int64)
        sm = DsdSummary()
        pr = np.empty(max(self.n, 1), np.int32) if rounds else None
        pmask = 0
        if profile and not isinstance(profile, bool):
            for nm in profile:
                pmask |= self.PROFILE_CLASSES[nm]
        p = DsdParams(k, eps_num, eps_den, 1 if profile else 0, self.MODES[mode], pmask)
        _check(self._lib.kws_dsd_peel(self.h, C.byref(p), pr.ctypes.data if rounds else None, sizes.ctypes.data,
                                      fs.ctypes.data, cap, C.byref(sm)))
        R = int(sm.rounds)
        return (pr[:self.n].copy() if rounds else None), sizes[:R + 1].copy(), fs[:R + 1].copy(), \
            {k2: getattr(sm, k2) for k2, _ in sm._fields_}

    def rounds(self) -> np.ndarray:
        """Peel rounds of the last run, copied from device memory."""
        pr = np.empty(max(self.n, 1), np.int32)
        _check(self._lib.kws_dsd_rounds(self.h, pr.ctypes.data, None))
        return pr[:self.n].copy()

    def device_rounds(self) -> int:
        """Device address of the last run's peel rounds (n int32, owned by the graph)."""
        d = C.c_void_p()
        _check(self._lib.kws_dsd_rounds(self.h, None, C.byref(d)))
        return d.value or 0

    def close(self):
        if getattr(self, "h", None):
            self._lib.kws_dsd_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
