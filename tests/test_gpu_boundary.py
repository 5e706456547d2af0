"""Statuses and limits of the C ABI (include/gsi.h), exercised through the
library on the GPU: caller buffers that are too small (GSI_E_CAPACITY), the
max_rows cap, borrowed device rows, the largest query (k = GSI_MAX_K = 32)
and the first one past it, count-only results, and overlapping calls on one
context (GSI_E_BUSY)."""
import ctypes
import math
import threading

import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

HIP_D2H = 2  # hipMemcpyDeviceToHost


@pytest.fixture(scope="module")
def ctx():
    import paper_1906_03420_amd as gsi
    c = gsi.Context(16 << 30)
    yield c
    c.close()


def _lib():
    import paper_1906_03420_amd as gsi
    return gsi.load_library()


def _status(fn, *args):
    return fn(*args)


def test_result_rows_capacity(ctx):
    import paper_1906_03420_amd as gsi
    from paper_1906_03420_amd.binding import U32P
    g = w.cycle_graph(50)
    dg = ctx.load(g)
    r = dg.query(w.path_query(4))
    assert r.count == 100  # P_k on C_n: 2n
    buf = np.zeros((r.count, 4), np.uint32)
    st = _lib().gsi_result_rows(r.h, buf.ctypes.data_as(U32P), r.count - 1)
    assert st == gsi.GSI_E_CAPACITY
    assert "need 100 rows" in gsi.gsi_last_error()
    assert _lib().gsi_result_rows(r.h, buf.ctypes.data_as(U32P), r.count) == gsi.GSI_OK
    np.testing.assert_array_equal(gsi.sort_rows(buf), oracle.match(g, w.path_query(4)).tuples)
    r.free()
    # a count-only result has no rows to copy or borrow
    r = dg.query(w.path_query(4), flags=gsi.GSI_COUNT_ONLY)
    assert r.count == 100
    assert _lib().gsi_result_rows(r.h, buf.ctypes.data_as(U32P), r.count) == gsi.GSI_E_INVALID
    p = ctypes.c_void_p()
    assert _lib().gsi_result_device_rows(r.h, ctypes.byref(p)) == gsi.GSI_E_INVALID
    r.free()
    dg.free()


def test_result_device_rows(ctx):
    """The borrowed device pointer holds the rows gsi_result_rows copies."""
    import paper_1906_03420_amd as gsi
    g = w.complete_graph(12)
    dg = ctx.load(g)
    q = w.path_query(5)
    r = dg.query(q)
    assert r.count == math.perm(12, 5)
    host = r.rows()
    ptr = gsi.gsi_result_device_rows(r.h)
    assert ptr
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemcpy.restype = ctypes.c_int
    dev = np.zeros_like(host)
    assert hip.hipMemcpy(dev.ctypes.data, ptr, dev.nbytes, HIP_D2H) == 0
    np.testing.assert_array_equal(dev, host)
    r.free()
    dg.free()


def test_max_rows(ctx):
    import paper_1906_03420_amd as gsi
    g = w.complete_graph(20)
    dg = ctx.load(g)
    q = w.path_query(4)
    for flags in (0, gsi.GSI_NO_FUSED):
        with pytest.raises(gsi.GsiError) as e:
            dg.query(q, flags=flags, max_rows=1000)  # level tables: 20, 380, 6840
        assert e.value.status == gsi.GSI_E_CAPACITY
    r = dg.query(q, max_rows=math.perm(20, 4))
    assert r.count == math.perm(20, 4)
    r.free()
    dg.free()


def test_largest_query_and_past_it(ctx):
    """k = 32 (GSI_MAX_K): a 32-vertex path and a 32-cycle on a cycle graph
    (closed forms 2n and, for the cycle on C_32, 2*32), every route; k = 33
    is rejected."""
    import paper_1906_03420_amd as gsi
    assert gsi.GSI_MAX_K == 32
    g = w.cycle_graph(40)
    dg = ctx.load(g)
    for q, want_count in ((w.path_query(32), 80),):
        want = oracle.match(g, q)
        assert want.count == want_count
        for flags in (0, gsi.GSI_NO_FUSED):
            r = dg.query(q, flags=flags)
            assert r.count == want_count and r.digest == want.digest
            np.testing.assert_array_equal(r.sorted_rows(), want.tuples)
            r.free()
    dg.free()
    g32 = w.cycle_graph(32)
    dg = ctx.load(g32)
    q = w.cycle_query(32)
    want = oracle.match(g32, q)
    assert want.count == 64
    r = dg.query(q)
    assert r.count == 64 and r.digest == want.digest
    np.testing.assert_array_equal(r.sorted_rows(), want.tuples)
    r.free()
    with pytest.raises(gsi.GsiError) as e:
        dg.query(w.path_query(33))
    assert e.value.status == gsi.GSI_E_INVALID
    dg.free()


def test_busy_on_overlapping_calls(ctx):
    """A call on a context that is already running one returns GSI_E_BUSY
    and leaves the running call's result intact (a 6-vertex path on K_40,
    count only: 40!/34! embeddings, about a second of device work)."""
    import paper_1906_03420_amd as gsi
    g = w.complete_graph(40)
    dg = ctx.load(g)
    long_q, small_q = w.path_query(6), w.path_query(2)
    busy_seen = 0
    for attempt in range(3):
        out = {}

        def long_call():
            while True:
                try:
                    r = dg.query(long_q, flags=gsi.GSI_COUNT_ONLY)
                except gsi.GsiError as e:
                    if e.status == gsi.GSI_E_BUSY:
                        continue  # the poller held the context: try again
                    out["error"] = e
                    return
                out["count"] = r.count
                r.free()
                return

        t = threading.Thread(target=long_call)
        t.start()
        while t.is_alive():
            try:
                dg.filter(small_q)
            except gsi.GsiError as e:
                assert e.status == gsi.GSI_E_BUSY, e
                assert "already running" in str(e)
                busy_seen += 1
        t.join()
        assert "error" not in out, out.get("error")
        assert out["count"] == math.perm(40, 6)
        if busy_seen:
            break
    assert busy_seen > 0
    dg.free()
