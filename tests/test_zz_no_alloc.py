"""The allocation-free query entry point (gsi_query_run_noalloc) against
gsi_query_run, through the C ABI: the same rows (as a set), count and digest
on consecutive calls whose scratch is the library's fixed device array, each
call smaller than the one before; sizes past the array are refused with
GSI_E_CAPACITY and leave the next call unharmed."""
import json
import os

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _gold(name):
    return {x["index"]: x for x in json.load(open(os.path.join(GOLDEN, name + ".json")))["queries"]}


def _rows(rows_t, count, k):
    return rows_t[:count * k].cpu().numpy().view(np.uint32).reshape(count, k)


def _same(dg, q, rows_t, gold=None, flags=0):
    import paper_1906_03420_amd as gsi
    print("noalloc query k=%d m=%d flags=%d" % (q.k, q.m, flags), flush=True)
    r = dg.query(q, flags=flags)
    count, digest = dg.query_noalloc(q, rows_t, flags)
    assert count == r.count and digest == r.digest
    if gold is not None:
        assert count == gold["count"] and [str(v) for v in digest] == gold["digest"]
    if not flags & gsi.GSI_COUNT_ONLY:
        np.testing.assert_array_equal(gsi.sort_rows(_rows(rows_t, count, q.k)), r.sorted_rows())
    r.free()
    return count


def test_noalloc_equals_query_run_er1k():
    import paper_1906_03420_amd as gsi
    import torch
    g = w.config_graph("er1k")
    gold = _gold("er1k")
    mk = w.QueryMaker(g)
    with gsi.Context(512 << 20) as ctx:
        dg = ctx.load(g)
        rows_t = torch.zeros(1 << 20, dtype=torch.int32, device="cuda:0")
        # the largest answer first, then a smaller one: the second call finds
        # the first one's data in the scratch
        order = sorted(gold, key=lambda i: -gold[i]["count"])
        for ix in (order[0], order[-1]):
            q = w.config_query(g, "er1k", ix, maker=mk)
            assert _same(dg, q, rows_t, gold[ix]) == gold[ix]["count"]
        q = w.config_query(g, "er1k", order[1], maker=mk)
        _same(dg, q, rows_t, gold[order[1]], flags=gsi.GSI_COUNT_ONLY)
        dg.free()
    mk.close()


def test_noalloc_equals_query_run_ba1m():
    import paper_1906_03420_amd as gsi
    import torch
    g = w.config_graph("ba1m")
    gold = _gold("ba1m")
    mk = w.QueryMaker(g)
    with gsi.Context(8 << 30) as ctx:
        dg = ctx.load(g)
        rows_t = torch.zeros(16 << 20, dtype=torch.int32, device="cuda:0")
        # 769,655 rows of 12 (k = 12), then 134,831 of 6, then 13,118 of 6
        for ix in (1, 84, 62):
            q = w.config_query(g, "ba1m", ix, attempt=gold[ix]["attempt"], maker=mk)
            _same(dg, q, rows_t, gold[ix])
        # 42.4M rows of 7 need more than the fixed scratch: refused
        q = w.config_query(g, "ba1m", 14, attempt=gold[14]["attempt"], maker=mk)
        with pytest.raises(gsi.GsiError) as e:
            dg.query_noalloc(q, rows_t)
        assert e.value.status == gsi.GSI_E_CAPACITY
        print("refused:", e.value, flush=True)
        # rows beyond the caller's buffer: refused
        q = w.config_query(g, "ba1m", 84, attempt=gold[84]["attempt"], maker=mk)
        with pytest.raises(gsi.GsiError) as e:
            dg.query_noalloc(q, rows_t[:6 * 1000])
        assert e.value.status == gsi.GSI_E_CAPACITY
        # and the next call is unharmed
        q = w.config_query(g, "ba1m", 4, attempt=gold[4]["attempt"], maker=mk)
        _same(dg, q, rows_t, gold[4])
        dg.free()
    mk.close()
