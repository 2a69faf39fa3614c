"""MI355X (gfx950) distance-bounded graph keyword search, and densest-
subgraph discovery by parallel peeling.

The hot paths live in the HIP library ``libkws.so`` (C ABI in
``include/kws.h`` and ``include/dsd.h``); ``kws`` is its ctypes binding.
"""
from .kws import (  # noqa: F401
    Graph, Server, Result, PeelGraph, KwsError, load_library, declared_symbols, last_error,
    set_mem_limit, mem_in_use,
    OK, EINVAL, ENOMEM, EDEVICE, EOVERFLOW, EBUSY, ECANCELLED, MAX_KW, MAX_DMAX, MAX_K, DIST_INF,
)
