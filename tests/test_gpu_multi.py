"""Multi-labelled vertices and edges (Sec. VII-B) on the GPU against the
multi-label oracle: random multi-labelled graphs and walk / dense queries
through every join route, closed forms, and agreement with the single-label
path when every set has one label."""
import math

import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

ROUTES = [dict(), dict(flags=0x4), dict(chunk_min_rows=2, chunk_rows=3), dict(fused_max_rows=8, fused_max_slots=64)]


@pytest.fixture(scope="module")
def ctx():
    import paper_1906_03420_amd as gsi
    c = gsi.Context(4 << 30)
    yield c
    c.close()


@pytest.mark.parametrize("seed", range(8))
def test_multi_random_graphs(ctx, seed):
    r = np.random.default_rng(7000 + seed)
    n = int(r.integers(80, 400))
    g = w.random_multi_graph(n, float(r.uniform(0.02, 0.06)), int(r.integers(2, 6)), int(r.integers(1, 4)),
                             int(r.integers(1, 4)), int(r.integers(1, 3)), seed + 300)
    dg = ctx.load_multi(g)
    og = oracle.OracleMultiGraph(g)
    for t in range(4):
        k = int(r.integers(2, 7))
        try:
            q = w.multi_walk_query(g, k, seed * 50 + t, dense=bool(t % 2))
        except RuntimeError:
            continue
        want = og.match(q, threads=4, max_count=2_000_000)
        if want.status != 0:
            continue
        assert want.count >= 1
        for mode in ROUTES:
            print("multi seed", seed, "query", t, "k", k, "mode", mode, flush=True)
            res = dg.query_multi(q, **mode)
            assert (res.count, res.digest) == (want.count, want.digest)
            np.testing.assert_array_equal(res.sorted_rows(), want.tuples)
            res.free()
    og.close()
    dg.free()


def test_multi_closed_forms(ctx):
    n = 9
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
    g = w.make_mgraph(n, [[0, 1]] * n, [(a, b, l) for a, b in pairs for l in (0, 1)])
    dg = ctx.load_multi(g)
    for k in range(1, 6):
        clique = [(a, b) for a in range(k) for b in range(a + 1, k)]
        for vsets, ls in (([[0]] * k, (1,)), ([[0, 1]] * k, (0, 1))):
            r = dg.query_multi(w.make_mquery(vsets, [(a, b, l) for a, b in clique for l in ls]))
            assert r.count == math.perm(n, k)
            r.free()
        r = dg.query_multi(w.make_mquery([[0, 2]] + [[0]] * (k - 1), [(a, b, 0) for a, b in clique]))
        assert r.count == 0
        r.free()
    dg.free()
    cyc = {(min(i, (i + 1) % n), max(i, (i + 1) % n)) for i in range(n)}
    g = w.make_mgraph(n, [[0]] * n, [(a, b, 0) for a, b in pairs] + [(a, b, 1) for a, b in sorted(cyc)])
    dg = ctx.load_multi(g)
    for k in range(2, n):
        r = dg.query_multi(w.make_mquery([[0]] * k, [(i, i + 1, l) for i in range(k - 1) for l in (0, 1)]))
        assert r.count == 2 * n
        r.free()
    dg.free()


def test_multi_singleton_sets_equal_single_label_path(ctx):
    """A single-label graph loaded as a multi-labelled one, and queries with
    singleton sets, give exactly the single-label path's rows; the
    single-label query call on a multi-labelled graph reads its labels as
    singletons; the multi-label call on a single-label graph matches only
    singleton sets."""
    import paper_1906_03420_amd as gsi
    g = w.config_graph("er1k")
    mk = w.QueryMaker(g)
    plain = ctx.load(g)
    multi = ctx.load_multi(w.mgraph_from_single(g))
    for i in range(8):
        q = w.config_query(g, "er1k", i, maker=mk)
        mq = w.mquery_from_single(q)
        a, b, c, d = plain.query(q), multi.query_multi(mq), multi.query(q), plain.query_multi(mq)
        assert a.count == b.count == c.count == d.count >= 1
        assert a.digest == b.digest == c.digest == d.digest
        rows = a.sorted_rows()
        for x in (b, c, d):
            np.testing.assert_array_equal(x.sorted_rows(), rows)
        for x in (a, b, c, d):
            x.free()
        two = w.make_mquery([q.vlabel[:1].tolist() + [int(q.vlabel[0]) + 1]] + [[int(x)] for x in q.vlabel[1:]],
                            list(zip(q.src.tolist(), q.dst.tolist(), q.elabel.tolist())))
        r = plain.query_multi(two)
        assert r.count == 0
        r.free()
    with pytest.raises(gsi.GsiError):
        multi.batch([q])
    with pytest.raises(gsi.GsiError):
        multi.server()
    multi.free()
    plain.free()


def test_multi_rejects_bad_input(ctx):
    import paper_1906_03420_amd as gsi
    with pytest.raises(gsi.GsiError) as e:
        ctx.load_multi(w.make_mgraph(3, [[0], [0], [0]], [(0, 1, 0), (1, 0, 0)]))
    assert e.value.status == gsi.GSI_E_INVALID
    dg = ctx.load_multi(w.make_mgraph(3, [[0], [0, 1], [0]], [(0, 1, 0), (0, 1, 1), (1, 2, 0)]))
    with pytest.raises(gsi.GsiError):
        dg.query_multi(w.make_mquery([[0], [0]], [(0, 1, 0), (1, 0, 0)]))
    with pytest.raises(gsi.GsiError):
        dg.query_multi(w.make_mquery([[0], [0], [0]], [(0, 1, 0)]))
    r = dg.query_multi(w.make_mquery([[0], [1]], [(0, 1, 0), (0, 1, 1)]))
    assert r.count == 1 and r.rows().tolist() == [[0, 1]]
    r.free()
    dg.free()
