"""The serving loop: every answer equals the oracle's, and the one the
single-query path gives for the same query alone, whatever else was in
flight when it ran (tolerance 0: count, digest and rows)."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1906_03420_amd as gsi
    c = gsi.Context(16 << 30)
    yield c
    c.close()


def _small_set(seed, nq):
    r = np.random.default_rng(seed)
    n = int(r.integers(100, 500))
    g = w.random_small_graph(n, float(r.uniform(0.01, 0.04)), int(r.integers(1, 4)), int(r.integers(1, 3)), seed)
    og = oracle.OracleGraph(g)
    qs, want = [], []
    t = 0
    while len(qs) < nq:
        q = w.random_connected_query(int(r.integers(1, 9)), int(r.integers(0, 3)), int(g.vlabel.max()) + 1,
                                     int(g.elabel.max()) + 1, seed * 1000 + t)
        t += 1
        res = og.match(q, threads=4, max_count=2_000_000)
        if res.status != 0:
            continue
        qs.append(q)
        want.append(res)
    return g, qs, want


def drive(srv, qs, seed, burst=6):
    """Submits the queries in seeded bursts between steps, so that queries
    arrive while others are in flight, and steps until every one is
    answered.  Returns the tickets (in query order) and their answers."""
    r = np.random.default_rng(seed)
    tickets, answers = [], {}
    i = steps = 0
    while len(answers) < len(qs):
        if i < len(qs):
            b = min(len(qs) - i, int(r.integers(0, burst + 1)))
            tickets += [srv.submit(q) for q in qs[i:i + b]]
            i += b
        srv.step()
        steps += 1
        for t in srv.poll():
            answers[t] = srv.answer(t)
        assert steps < 200 * len(qs) + 1000, "server made no progress"
    return tickets, answers


@pytest.mark.parametrize("opts", [dict(), dict(table_budget=1, max_admit=1, flags=2), dict(max_inflight=3, max_admit=2),
                                  dict(threads=64, grid_scale=4, flags=2), dict(solo_queue=1000),
                                  dict(flags=2, engine_tiles=8)])
def test_server_matches_oracle(ctx, opts):
    for seed in (5, 6):
        g, qs, want = _small_set(seed, 50)
        dg = ctx.load(g)
        print("server seed", seed, "options", opts, flush=True)
        srv = dg.server(**opts)
        tickets, ans = drive(srv, qs, seed)
        paths = {}
        for q, t, wnt in zip(qs, tickets, want):
            a = ans[t]
            assert a["status"] == 0 and a["k"] == q.k
            assert (a["count"], a["digest"]) == (wnt.count, wnt.digest), t
            np.testing.assert_array_equal(srv.sorted_rows(t), wnt.tuples)
            assert a["admit_ms"] >= a["submit_ms"] and a["done_ms"] >= a["admit_ms"]
            paths[a["path"]] = paths.get(a["path"], 0) + 1
            srv.release(t)
        info = srv.info()
        print("paths", paths, "info", info, flush=True)
        assert info["answered"] == info["admitted"] == info["submitted"] == len(qs)
        if opts.get("flags", 0) & 2:
            assert info["solo"] == 0 and "solo" not in paths
        if opts.get("solo_queue") == 1000:
            # nothing is ever in flight: every request is answered alone
            assert paths == {"solo": len(qs)}
        assert info["waiting"] == 0 and info["in_flight"] == 0
        if opts.get("table_budget") == 1:
            # nothing is admitted beside a query still in the level engine
            assert info["admit_rounds"] >= paths.get("levels", 0)
        srv.free()
        dg.free()
    assert ctx.memory()[0] == 0


def test_server_count_only_and_errors(ctx):
    import paper_1906_03420_amd as gsi
    g, qs, want = _small_set(7, 30)
    dg = ctx.load(g)
    srv = dg.server(flags=gsi.GSI_COUNT_ONLY)
    t0 = srv.submit(qs[0])
    with pytest.raises(gsi.GsiError) as e:
        srv.answer(t0)  # not answered yet
    assert e.value.status == gsi.GSI_E_INVALID
    with pytest.raises(gsi.GsiError):
        srv.submit(w.make_query([0, 0, 0], [(0, 1)], [0]))  # disconnected
    tickets = [t0] + [srv.submit(q) for q in qs[1:]]
    ans = {}
    for _ in range(100 * len(qs)):
        if len(ans) == len(tickets):
            break
        srv.step()
        for t in srv.poll():
            ans[t] = srv.answer(t)
    assert len(ans) == len(tickets)
    for t, wnt in zip(tickets, want):
        assert (ans[t]["count"], ans[t]["digest"]) == (wnt.count, wnt.digest)
    with pytest.raises(gsi.GsiError):
        gsi.gsi_server_rows(srv.h, tickets[0], qs[0].k, ans[tickets[0]]["count"])
    srv.release(tickets[0])
    with pytest.raises(gsi.GsiError):
        srv.release(tickets[0])
    with pytest.raises(gsi.GsiError):
        srv.answer(10 ** 9)
    srv.free()
    dg.free()


def test_server_query_too_large_for_the_arena():
    """A query whose table cannot fit even alone is answered with
    GSI_E_NOMEM; the queries around it are answered normally."""
    import paper_1906_03420_amd as gsi
    g = w.complete_graph(40)
    big = w.clique_query(7)      # 40!/33! rows; level 5 alone needs ~1.6 GB
    small = w.path_query(3)      # 40*39*38 rows
    og = oracle.OracleGraph(g)
    ws = og.match(small, threads=2)
    with gsi.Context(256 << 20) as c:
        dg = c.load(g)
        for flags, path in ((gsi.GSI_SERVER_NO_SOLO, "levels"), (0, "solo")):
            srv = dg.server(flags=flags)
            tb, ts = srv.submit(big), srv.submit(small)
            ans = {}
            for _ in range(200):
                srv.step()
                for t in srv.poll():
                    ans[t] = srv.answer(t)
                if len(ans) == 2:
                    break
            assert ans[tb]["status"] == gsi.GSI_E_NOMEM and ans[tb]["path"] == path
            assert ans[ts]["status"] == 0 and ans[ts]["count"] == 40 * 39 * 38 == ws.count
            assert ans[ts]["digest"] == ws.digest
            np.testing.assert_array_equal(srv.sorted_rows(ts), og.match(small, threads=2, tuples=True).tuples)
            srv.release(tb)
            srv.release(ts)
            srv.free()
        dg.free()
        assert c.memory()[0] == 0


def test_server_ba1m_mix_equals_alone(golden_dir):
    """600 mixed BA-1M queries arriving in bursts: each answer equals the
    stored oracle count and digest, and, on a sample, the single-query path
    and a server holding that query alone (rows compared as sets)."""
    import torch
    import paper_1906_03420_amd as gsi
    gold = json.load(open(os.path.join(golden_dir, "ba1m_batch.json")))["queries"][:600]
    g = w.config_graph("ba1m_batch")
    mk = w.QueryMaker(g)
    qs = [w.config_query(g, "ba1m_batch", x["index"], attempt=x["attempt"], maker=mk) for x in gold]
    dev = torch.device("cuda:0")
    as_t = lambda a: torch.from_numpy(a.view(np.int32)).to(dev)
    with gsi.Context(64 << 30) as c:
        dg = c.load_device(g.n, as_t(g.vlabel), as_t(g.src), as_t(g.dst), as_t(g.elabel))
        srv = dg.server()
        tickets, ans = drive(srv, qs, 11, burst=40)
        info = srv.info()
        print("server info", info, flush=True)
        paths = {}
        for x, t in zip(gold, tickets):
            a = ans[t]
            paths[a["path"]] = paths.get(a["path"], 0) + 1
            assert a["status"] == 0
            assert a["count"] == x["count"], x["index"]
            assert [str(v) for v in a["digest"]] == x["digest"], x["index"]
        print("paths", paths, flush=True)
        assert paths.get("levels", 0) > 0 and paths.get("tier1", 0) > 0
        for i in range(0, len(qs), 41):
            t = tickets[i]
            r = dg.query(qs[i])
            assert (r.count, r.digest) == (ans[t]["count"], ans[t]["digest"])
            if r.count <= 200_000:
                np.testing.assert_array_equal(r.sorted_rows(), srv.sorted_rows(t))
            r.free()
            alone = dg.server()
            ta = alone.submit(qs[i])
            while not alone.poll():
                alone.step()
            aa = alone.answer(ta)
            assert (aa["count"], aa["digest"]) == (ans[t]["count"], ans[t]["digest"])
            alone.free()
        for t in tickets:
            srv.release(t)
        srv.free()
        dg.free()
