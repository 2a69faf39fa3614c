"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects malformed input before touching a device."""
import ctypes as C

import numpy as np
import pytest

import paper_2504_09311_amd as K
from paper_2504_09311_amd import kws as B


def test_exports_every_declared_symbol():
    lib = K.load_library()
    names = K.declared_symbols()
    assert len(names) >= 15
    for s in names:
        assert hasattr(lib, s), s


def _desc(n, row_ptr, col, n_labels, lab_ptr, lab, parent=None, m=None):
    keep = [np.ascontiguousarray(np.asarray(x, np.int32)) for x in (row_ptr, col, lab_ptr, lab)]
    rp, cl, lp, lb = keep
    tp = None if parent is None else np.ascontiguousarray(np.asarray(parent, np.int32))
    d = B.GraphDesc(n, cl.shape[0] if m is None else m, rp.ctypes.data, cl.ctypes.data if cl.size else None,
                    n_labels, lp.ctypes.data, lb.ctypes.data if lb.size else None,
                    tp.ctypes.data if tp is not None else None)
    return d, (keep, tp)


@pytest.mark.parametrize("case", [
    "n0", "rowptr0", "decreasing", "rowptr_end", "col_range", "lab_range", "cycle", "self_parent",
    "overflow",
])
def test_load_graph_rejects(case):
    lib = K.load_library()
    rp, col, lp, lab, par, n, nl, m = [0, 1, 2], [1, 0], [0, 1, 1], [0], None, 2, 2, None
    if case == "n0":
        n, rp, lp = 0, [0], [0]
        col, lab = [], []
    elif case == "rowptr0":
        rp = [1, 1, 2]
    elif case == "decreasing":
        rp = [0, 2, 1]
    elif case == "rowptr_end":
        rp = [0, 1, 1]
    elif case == "col_range":
        col = [1, 2]
    elif case == "lab_range":
        lab = [5]
    elif case == "cycle":
        par = [1, 0]
    elif case == "self_parent":
        par = [0, -1]
    elif case == "overflow":
        m = 1 << 31
    d, keep = _desc(n, rp, col, nl, lp, lab, par, m)
    h = C.c_void_p()
    st = lib.kws_load_graph(C.byref(d), C.byref(h))
    want = K.EOVERFLOW if case == "overflow" else K.EINVAL
    assert st == want, (case, st, K.last_error())
    assert not h.value
    assert K.last_error()


def test_null_arguments():
    lib = K.load_library()
    assert lib.kws_load_graph(None, None) == K.EINVAL
    assert lib.kws_set_options(None, None) == K.EINVAL
    assert lib.kws_search_batch(None, None, 0, None) == K.EINVAL
    assert lib.kws_keyword_search(None, None, None) == K.EINVAL
    assert lib.kws_debug_distances(None, 0, 0, None) == K.EINVAL
    t = C.c_int64()
    assert lib.kws_search_batch_submit(None, None, 0, C.byref(t)) == K.EINVAL
    assert lib.kws_search_batch_collect(None, 1, None) == K.EINVAL
    r = B.ResultC()
    lib.kws_result_free(C.byref(r))          # freeing a zeroed result is a no-op
    assert lib.kws_profile_name(0) == b"seed"
    assert lib.kws_profile_name(99) is None


def test_allocator_hooks_need_both():
    lib = K.load_library()
    f = B.ALLOC_FN(lambda n, c: None)
    assert lib.kws_set_allocator(C.cast(f, C.c_void_p), None, None) == K.EINVAL
    assert lib.kws_set_allocator(None, None, None) == K.OK


def test_product_path_has_no_cpu_fallback():
    # the binding must not import the oracle, and fails loudly without the library
    import paper_2504_09311_amd.kws as mod
    src = open(mod.__file__).read()
    assert "oracle" not in src.replace("no CPU", "")
    with pytest.raises(RuntimeError):
        B._lib, saved = None, B._lib
        try:
            B.load_library("/nonexistent/libkws.so")
        finally:
            B._lib = saved


def test_server_null_arguments():
    lib = K.load_library()
    t = C.c_uint64()
    assert lib.kws_server_create(None, None, None) == K.EINVAL
    assert lib.kws_server_submit(None, None, C.byref(t)) == K.EINVAL
    r, d = B.ResultC(), C.c_int32()
    assert lib.kws_server_poll(None, 1, C.byref(r), C.byref(d)) == K.EINVAL
    assert lib.kws_server_cancel(None, 1) == K.EINVAL
    lib.kws_server_destroy(None)
    lib.kws_batch_result_free(None)


def test_profile_classes_needs_a_graph():
    import ctypes as C
    lib = K.load_library()
    assert lib.kws_profile_classes(None, C.c_uint64(1)) == K.EINVAL


def test_dsd_load_rejects_bad_input():
    # validation happens on the host before any device call
    lib = K.load_library()
    h = C.c_void_p()
    src = np.array([0, 1, 2], np.int32)
    dst = np.array([1, 2, 2], np.int32)          # a self-loop
    ew = np.array([1, 1, 1], np.int64)
    d = B.DsdDesc(3, 3, src.ctypes.data, dst.ctypes.data, ew.ctypes.data, None, 1)
    assert lib.kws_dsd_load(C.byref(d), C.byref(h)) == K.EINVAL and not h.value
    dst2 = np.array([1, 2, 5], np.int32)         # out of range
    d = B.DsdDesc(3, 3, src.ctypes.data, dst2.ctypes.data, ew.ctypes.data, None, 1)
    assert lib.kws_dsd_load(C.byref(d), C.byref(h)) == K.EINVAL
    dst3 = np.array([1, 2, 0], np.int32)
    d = B.DsdDesc(3, 3, src.ctypes.data, dst3.ctypes.data, None, None, 1)   # DW without weights
    assert lib.kws_dsd_load(C.byref(d), C.byref(h)) == K.EINVAL
    d = B.DsdDesc(3, 3, src.ctypes.data, dst3.ctypes.data, None, None, 2)   # FD without vertex weights
    assert lib.kws_dsd_load(C.byref(d), C.byref(h)) == K.EINVAL
    neg = np.array([1, -1, 1], np.int64)
    d = B.DsdDesc(3, 3, src.ctypes.data, dst3.ctypes.data, neg.ctypes.data, None, 1)
    assert lib.kws_dsd_load(C.byref(d), C.byref(h)) == K.EINVAL
    d = B.DsdDesc(3, 3, src.ctypes.data, dst3.ctypes.data, None, None, 7)   # unknown metric
    assert lib.kws_dsd_load(C.byref(d), C.byref(h)) == K.EINVAL
    assert lib.kws_dsd_load(None, C.byref(h)) == K.EINVAL
    assert lib.kws_dsd_peel(None, None, None, None, None, 0, None) == K.EINVAL
    assert K.last_error()
