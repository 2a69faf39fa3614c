"""Seeded synthetic inputs shared by the oracle's tests and the GPU library.

This package generates graphs, labels, type trees, queries and arrival
times. It holds none of the keyword-search arithmetic. The C core
(``synth.c``) draws every random number from SplitMix64 in counter mode, so
each output is a pure function of its seed. ``workloads`` names the
concrete benchmark and test inputs.
"""
from .gen import (  # noqa: F401
    build, u64, permutation, rmat_csr, chung_lu_csr, labels_zipf, type_tree,
    queries, arrivals, Graph, Query,
)
