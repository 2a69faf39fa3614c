"""The allocation-free distance export (kws_debug_distances_noalloc) against
the allocating one (kws_debug_distances), through the C ABI.

Two calls in a row, the second on a smaller graph and radius, so stale
contents of the fixed device array from the first call would show; the
library's device-memory tally is unchanged by the calls (they allocate
nothing); a graph larger than the array is refused with ENOMEM before any
device work. The output buffers are allocated by the test through the HIP
runtime the library is linked against.
"""
import ctypes

import numpy as np
import pytest

import oracle
from synth import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import paper_2504_09311_amd as K
    K.load_library()
    return K


@pytest.fixture(scope="module")
def hip():
    h = ctypes.CDLL("libamdhip64.so.7")            # the instance libkws.so is linked against
    h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    h.hipFree.argtypes = [ctypes.c_void_p]
    h.hipMemset.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t]
    h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    h.hipDeviceSynchronize.argtypes = []
    return h


HIP_D2H = 2


def noalloc_distances(K, hip, G, n, kw, d_max):
    p = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(p), n) == 0
    try:
        assert hip.hipMemset(p, 0xAB, n) == 0         # poison: an unwritten entry would show
        assert hip.hipDeviceSynchronize() == 0
        before = K.mem_in_use()
        G.debug_distances_noalloc(kw, d_max, p.value)
        assert K.mem_in_use() == before, "the allocation-free path allocated device memory"
        out = np.empty(n, np.uint8)
        assert hip.hipMemcpy(out.ctypes.data, p, n, HIP_D2H) == 0
        return out
    finally:
        hip.hipFree(p)


def test_noalloc_equals_debug_distances(K, hip):
    # first call: 2^14 R-MAT with the type tree, radius 4, several keywords
    g1, qs1 = workloads.rmat24_hier(14, 8)
    G1 = K.Graph.from_synth(g1)
    o1 = oracle.Oracle(g1)
    kws1 = sorted({t for q in qs1 for t in q.kw})[:6]
    for t in kws1:
        want = G1.debug_distances(t, 4)
        got = noalloc_distances(K, hip, G1, g1.n, t, 4)
        assert np.array_equal(got, want), ("rmat14 hier", t)
        assert np.array_equal(got, o1.distances(t, 4)[0]), ("rmat14 hier vs oracle", t)
    G1.close()
    # second call: a smaller graph, a smaller radius
    g2 = workloads.chunglu10k()
    qs2 = workloads.chunglu10k_queries(4)
    G2 = K.Graph.from_synth(g2)
    o2 = oracle.Oracle(g2)
    for d in (2, 0):
        for t in sorted({t for q in qs2 for t in q.kw}):
            want = G2.debug_distances(t, d)
            got = noalloc_distances(K, hip, G2, g2.n, t, d)
            assert np.array_equal(got, want), ("chunglu10k", t, d)
            assert np.array_equal(got, o2.distances(t, d)[0]), ("chunglu10k vs oracle", t, d)
    G2.close()


def test_noalloc_refuses_graphs_beyond_its_array(K, hip):
    g, qs = workloads.rmat20_q4(20, 1)
    n = g.n
    # at radius 15 (four distance planes) a vertex needs 4 * 8 + 4 * 8 + 4 + 4 + 2 = 74 bytes:
    # 74 MiB at 2^20 vertices, more than the 64 MiB array, so the call is refused on the host
    assert n == 1 << 20 and 74 * n > 64 << 20
    G = K.Graph.from_synth(g)
    p = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(p), n) == 0
    try:
        before = K.mem_in_use()
        with pytest.raises(K.KwsError) as ei:
            G.debug_distances_noalloc(qs[0].kw[0], 15, p.value)
        assert ei.value.status == K.ENOMEM and "allocation-free" in str(ei.value)
        assert K.mem_in_use() == before
    finally:
        hip.hipFree(p)
    G.close()
