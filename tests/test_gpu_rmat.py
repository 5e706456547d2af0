"""Full-size R-MAT workloads against the stored oracle values: the serving
pool on the scale-22 graph (50M edges) through the server, the
single-query path and a batch; and the scale-23 graph (100M edges) through
the single-query path.  Each test checks the queries its golden file holds
(the files are written query by query)."""
import json
import os

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu


def _gold(golden_dir, name):
    path = os.path.join(golden_dir, "%s.json" % name)
    if not os.path.exists(path):
        pytest.skip("no stored oracle values for %s" % name)
    gold = json.load(open(path))
    if not gold["queries"]:
        pytest.skip("no stored oracle values for %s" % name)
    return gold


def _load(ctx, g):
    import torch
    dev = torch.device("cuda:0")
    as_t = lambda a: torch.from_numpy(a.view(np.int32)).to(dev)
    return ctx.load_device(g.n, as_t(g.vlabel), as_t(g.src), as_t(g.dst), as_t(g.elabel))


def test_rmat22_serving_pool(golden_dir):
    import paper_1906_03420_amd as gsi
    gold = _gold(golden_dir, "rmat22_serve")["queries"]
    print("generating the scale-22 graph", flush=True)
    g = w.config_graph("rmat22_serve")
    mk = w.QueryMaker(g)
    qs = [w.config_query(g, "rmat22_serve", x["index"], attempt=x["attempt"], maker=mk) for x in gold]
    mk.close()
    want = [(x["count"], x["digest"]) for x in gold]
    with gsi.Context(96 << 30) as ctx:
        dg = _load(ctx, g)
        print("pool of", len(qs), "queries; serving", flush=True)
        srv = dg.server()
        r = np.random.default_rng(5)
        tickets, ans, i = [], {}, 0
        while len(ans) < len(qs):
            b = min(len(qs) - i, int(r.integers(0, 24)))
            tickets += [srv.submit(q) for q in qs[i:i + b]]
            i += b
            srv.step()
            for t in srv.poll():
                ans[t] = srv.answer(t)
                if ans[t]["count"] > 200_000:
                    srv.release(t)
        for t, (c, d) in zip(tickets, want):
            assert ans[t]["status"] == 0 and ans[t]["count"] == c and [str(v) for v in ans[t]["digest"]] == d
        print("server info", srv.info(), flush=True)
        srv.free()
        print("single-query path", flush=True)
        for q, (c, d) in zip(qs, want):
            res = dg.query(q, flags=gsi.GSI_COUNT_ONLY)
            assert res.count == c and [str(v) for v in res.digest] == d
            res.free()
        print("batch", flush=True)
        b = dg.batch(qs, flags=gsi.GSI_COUNT_ONLY)
        for i, (c, d) in enumerate(want):
            assert b.count(i) == c and [str(v) for v in b.digest(i)] == d
        print("batch info", b.info(), flush=True)
        b.free()
        dg.free()


def test_rmat23_single_query_path(golden_dir):
    import paper_1906_03420_amd as gsi
    gold = _gold(golden_dir, "rmat23")["queries"]
    print("generating the scale-23 graph", flush=True)
    g = w.config_graph("rmat23")
    mk = w.QueryMaker(g)
    qs = [w.config_query(g, "rmat23", x["index"], attempt=x["attempt"], maker=mk) for x in gold]
    mk.close()
    with gsi.Context(160 << 30) as ctx:
        dg = _load(ctx, g)
        for q, x in zip(qs, gold):
            print("rmat23 query", x["index"], "k", q.k, "count", x["count"], flush=True)
            res = dg.query(q)
            assert res.count == x["count"]
            assert [str(v) for v in res.digest] == x["digest"]
            res.free()
        dg.free()
