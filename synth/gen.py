"""ctypes binding of ``synth.c`` plus the plain containers for graphs and queries."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``libsynth.so`` in place with gcc (OpenMP for the big graphs)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = C.CDLL(_LIB)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        i64p = C.POINTER(C.c_int64)
        lib.syn_key.restype = C.c_uint64
        lib.syn_key.argtypes = [C.c_uint64, C.c_uint64]
        lib.syn_u64.restype = C.c_uint64
        lib.syn_u64.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
        lib.syn_uniform_i64.restype = None
        lib.syn_uniform_i64.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, C.c_int64, C.c_int64,
                                        np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")]
        lib.syn_permutation.restype = None
        lib.syn_permutation.argtypes = [C.c_int64, C.c_uint64, C.c_uint64, i32p]
        lib.syn_rmat_csr.restype = C.c_int64
        lib.syn_rmat_csr.argtypes = [C.c_int32, C.c_int64, C.c_double, C.c_double, C.c_double,
                                     C.c_uint64, i32p, i32p]
        lib.syn_chung_lu_csr.restype = C.c_int64
        lib.syn_chung_lu_csr.argtypes = [C.c_int32, C.c_int64, C.c_double, C.c_uint64, i32p, i32p]
        lib.syn_labels_zipf.restype = C.c_int64
        lib.syn_labels_zipf.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                        C.c_uint64, i32p, i32p]
        lib.syn_type_tree.restype = C.c_int64
        lib.syn_type_tree.argtypes = [C.c_int32, C.c_int32, C.c_uint64, i32p, i32p, i64p]
        lib.syn_queries.restype = C.c_int32
        lib.syn_queries.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                    i32p, C.c_int32, C.c_uint64, C.c_uint64,
                                    C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                    i32p, i32p, i32p]
        lib.syn_arrivals.restype = None
        lib.syn_arrivals.argtypes = [C.c_int64, C.c_double, C.c_uint64, f64p]
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Directed graph as an int32 forward CSR plus vertex labels.

    ``row_ptr[n+1]``/``col[m]``: out-neighbours of u are
    ``col[row_ptr[u]:row_ptr[u+1]]``. ``lab_ptr``/``lab``: label ids of
    each vertex. ``type_parent`` is None for flat labels, else the parent
    type of each label id (-1 at a root).
    """
    row_ptr: np.ndarray
    col: np.ndarray
    n_labels: int
    lab_ptr: np.ndarray
    lab: np.ndarray
    type_parent: Optional[np.ndarray] = None
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.col.shape[0])


@dataclass
class Query:
    kw: List[int]
    d_max: int
    k: int
    extra: dict = field(default_factory=dict)


def stream_key(seed: int, stream: int) -> int:
    return int(_L().syn_key(seed, stream))


def u64(seed: int, stream: int, ctr: int) -> int:
    return int(_L().syn_u64(seed, stream, ctr))


def uniform_i64(seed: int, stream: int, count: int, lo: int, hi: int) -> np.ndarray:
    """count uniform integers in [lo, hi] from (seed, stream)."""
    out = np.empty(max(count, 1), np.int64)
    _L().syn_uniform_i64(seed, stream, count, lo, hi, out)
    return out[:count]


def permutation(n: int, seed: int, stream: int = 15) -> np.ndarray:
    out = np.empty(n, np.int32)
    _L().syn_permutation(n, seed, stream, out)
    return out


def rmat_csr(scale: int, n_samples: int, a=0.57, b=0.19, c=0.19, seed=0):
    n = 1 << scale
    row_ptr = np.empty(n + 1, np.int32)
    col = np.empty(max(n_samples, 1), np.int32)
    m = _L().syn_rmat_csr(scale, n_samples, a, b, c, seed, row_ptr, col)
    if m < 0:
        raise MemoryError("syn_rmat_csr failed")
    return row_ptr, col[:m].copy() if m < col.shape[0] // 2 else col[:m]


def chung_lu_csr(n: int, m: int, gamma=2.1, seed=0):
    row_ptr = np.empty(n + 1, np.int32)
    col = np.empty(m, np.int32)
    mm = _L().syn_chung_lu_csr(n, m, gamma, seed, row_ptr, col)
    if mm < 0:
        raise ValueError("chung_lu: too many edges for n")
    return row_ptr, col[:mm]


def labels_zipf(n: int, L: int, s: float, lo=1, hi=3, seed=0):
    lab_ptr = np.empty(n + 1, np.int32)
    lab = np.empty(n * hi, np.int32)
    tot = _L().syn_labels_zipf(n, L, s, lo, hi, seed, lab_ptr, lab)
    if tot < 0:
        raise ValueError("labels_zipf: bad arguments")
    return lab_ptr, lab[:tot].copy()


def type_tree(fanout: int, depth: int, seed=0):
    total = sum(fanout ** d for d in range(depth + 1))
    parent = np.empty(total, np.int32)
    leaves = np.empty(fanout ** depth, np.int32)
    nl = C.c_int64(0)
    t = _L().syn_type_tree(fanout, depth, seed, parent, leaves, C.byref(nl))
    assert t == total and nl.value == leaves.shape[0]
    return parent, leaves


def queries(nq: int, L: int, s: float, mq_lo: int, mq_hi: int, dmax_set, k: int,
            label_seed: int, seed: int, leaf_ids=None, parent=None, leaf_depth=0,
            hd_lo=0, hd_hi=0) -> List[Query]:
    kw = np.zeros(nq * mq_hi, np.int32)
    n_kw = np.zeros(nq, np.int32)
    dmx = np.zeros(nq, np.int32)
    ds = np.ascontiguousarray(np.asarray(dmax_set, np.int32))
    lp = leaf_ids.ctypes.data if leaf_ids is not None else None
    pp = parent.ctypes.data if parent is not None else None
    rc = _L().syn_queries(nq, L, s, mq_lo, mq_hi, ds, ds.shape[0], label_seed, seed,
                          lp, pp, leaf_depth, hd_lo, hd_hi, kw, n_kw, dmx)
    if rc != 0:
        raise ValueError("queries: bad arguments")
    kw = kw.reshape(nq, mq_hi)
    return [Query([int(x) for x in kw[q, :n_kw[q]]], int(dmx[q]), int(k)) for q in range(nq)]


def arrivals(count: int, lam: float, seed: int) -> np.ndarray:
    out = np.empty(count, np.float64)
    _L().syn_arrivals(count, lam, seed, out)
    return out
