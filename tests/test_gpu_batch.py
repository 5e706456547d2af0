"""The batched path: every query's result equals the oracle's and the
single-query path's, under every schedule and with forced tier overflow."""
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
        q = w.random_connected_query(int(r.integers(1, 8)), int(r.integers(0, 3)), int(g.vlabel.max()) + 1,
                                     int(g.elabel.max()) + 1, seed * 1000 + t)
        t += 1
        res = og.match(q, threads=4, max_count=2_000_000)
        if res.status != 0:
            continue
        qs.append(q)
        want.append(res)
    return g, qs, want


@pytest.mark.parametrize("threads,grid_scale,flags,tiles", [(64, 8, 0, 0), (256, 8, 0, 0), (1024, 8, 0, 0),
                                                           (64, 1, 0, 0), (256, 4, 0, 0), (256, 8, 8, 0),
                                                           (256, 8, 8, 1), (256, 8, 8, 2), (256, 8, 8, 8),
                                                           (64, 8, 0, 8)])
def test_batch_matches_oracle(ctx, threads, grid_scale, flags, tiles):
    for seed in (3, 4):
        g, qs, want = _small_set(seed, 60)
        dg = ctx.load(g)
        print("batch seed", seed, "threads", threads, "flags", flags, "engine tiles", tiles, flush=True)
        b = dg.batch(qs, flags=flags, threads=threads, grid_scale=grid_scale, engine_tiles=tiles)
        assert b.info()["schedule"]["engine_tiles"] == tiles
        info = b.info()
        assert info["queries"] == len(qs)
        assert info["empty"] + info["tier1"] + info["tier2"] + info["per_level"] == len(qs)
        for i, (q, wnt) in enumerate(zip(qs, want)):
            assert b.count(i) == wnt.count
            assert b.digest(i) == wnt.digest
            np.testing.assert_array_equal(b.sorted_rows(i), wnt.tuples)
        b.free()
        dg.free()


def test_batch_count_only_and_tune(ctx):
    import paper_1906_03420_amd as gsi
    g, qs, want = _small_set(9, 80)
    dg = ctx.load(g)
    sched = dg.tune(qs, sample=40)
    assert sched["threads"] in (64, 256, 1024) and sched["grid_scale"] in (4, 8)
    assert sched["engine_tiles"] in (1, 2, 4, 8)
    with pytest.raises(gsi.GsiError):
        dg.batch(qs, threads=256, grid_scale=8, engine_tiles=3)
    b = dg.batch(qs, flags=gsi.GSI_COUNT_ONLY)  # tuned schedule
    assert b.info()["schedule"]["threads"] == sched["threads"]
    for i, wnt in enumerate(want):
        assert (b.count(i), b.digest(i)) == (wnt.count, wnt.digest)
    with pytest.raises(gsi.GsiError):
        b.rows(0)
    with pytest.raises(gsi.GsiError):
        b.count(len(qs))
    b.free()
    # an invalid query names its index
    bad = qs[:3] + [w.make_query([0, 0, 0], [(0, 1)], [0])]
    with pytest.raises(gsi.GsiError) as e:
        dg.batch(bad)
    assert "query 3" in str(e.value)
    dg.free()
    assert ctx.memory()[0] == 0


BA1M_BATCH_PARTS = 4


@pytest.fixture(scope="module")
def ba1m_batch(golden_dir):
    """The batched BA-1M workload (1,024 mixed queries) run once as a batch
    with rows written; the graph and results stay resident for the tests."""
    import torch
    import paper_1906_03420_amd as gsi
    gold = json.load(open(os.path.join(golden_dir, "ba1m_batch.json")))
    g = w.config_graph("ba1m_batch")
    mk = w.QueryMaker(g)
    qs = [w.config_query(g, "ba1m_batch", x["index"], attempt=x["attempt"], maker=mk) for x in gold["queries"]]
    dev = torch.device("cuda:0")
    as_t = lambda a: torch.from_numpy(a.view(np.int32)).to(dev)
    ctx = gsi.Context(64 << 30)
    dg = ctx.load_device(g.n, as_t(g.vlabel), as_t(g.src), as_t(g.dst), as_t(g.elabel))
    b = dg.batch(qs)
    print("batch info", b.info(), flush=True)
    state = dict(g=g, qs=qs, gold=gold["queries"], ctx=ctx, dg=dg, b=b, og=None)
    yield state
    if state["og"] is not None:
        state["og"].close()
    b.free()
    dg.free()
    ctx.close()


def test_batch_ba1m_mixed_full(ba1m_batch):
    """The batched BA-1M workload against the stored oracle counts and
    digests (fused tiers + engine, and the engine alone), and against the
    single-query path."""
    import paper_1906_03420_amd as gsi
    qs, gold, dg, b = ba1m_batch["qs"], ba1m_batch["gold"], ba1m_batch["dg"], ba1m_batch["b"]
    lv = dg.batch(qs, flags=gsi.GSI_BATCH_LEVELS_ONLY | gsi.GSI_COUNT_ONLY)
    print("levels-only batch info", lv.info(), flush=True)
    for i, x in enumerate(gold):
        assert lv.count(i) == x["count"], i
        assert [str(v) for v in lv.digest(i)] == x["digest"], i
    lv.free()
    for i, x in enumerate(gold):
        assert b.count(i) == x["count"], i
        assert [str(v) for v in b.digest(i)] == x["digest"], i
    # single-query path on a sample: identical counts, digests and tuples
    for i in range(0, len(qs), 37):
        r = dg.query(qs[i])
        assert (r.count, r.digest) == (b.count(i), b.digest(i))
        if r.count <= 200_000:
            np.testing.assert_array_equal(r.sorted_rows(), b.sorted_rows(i))
        r.free()


@pytest.mark.parametrize("part", range(BA1M_BATCH_PARTS))
def test_batch_ba1m_tuples(ba1m_batch, part):
    """Sorted tuples of every batched query whose output is at most 2 GiB
    equal the live oracle's (queries split in parts by index)."""
    if ba1m_batch["og"] is None:
        ba1m_batch["og"] = oracle.OracleGraph(ba1m_batch["g"])
    og, qs, gold, b = ba1m_batch["og"], ba1m_batch["qs"], ba1m_batch["gold"], ba1m_batch["b"]
    threads = max(1, min(16, os.cpu_count() or 1))
    n = 0
    for i in range(part, len(qs), BA1M_BATCH_PARTS):
        x = gold[i]
        if x["count"] * x["k"] * 4 > (2 << 30):
            continue
        want = og.match(qs[i], threads=threads)
        assert want.status == oracle.OR_OK and want.count == x["count"], i
        np.testing.assert_array_equal(b.sorted_rows(i), want.tuples)
        n += 1
    print("part", part, "compared", n, "queries tuple by tuple", flush=True)
