"""GPU parity: every step of the HIP path against the CPU oracle, through the
C ABI.  Integer work, so every comparison is bit-exact."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import spec
import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1906_03420_amd as gsi
    c = gsi.Context(8 << 30)
    yield c
    c.close()


def _sorted(a):
    return a[np.lexsort(a.T[::-1])] if len(a) else a


def check_query(dg, g, q, og=None, threads=4, **kw):
    print("query k=%d m=%d" % (q.k, q.m), flush=True)
    r = dg.query(q, **kw)
    want = (og or oracle.OracleGraph(g)).match(q, threads=threads)
    assert want.status == 0
    assert r.count == want.count
    if not kw.get("flags", 0) & 1:
        np.testing.assert_array_equal(r.sorted_rows(), want.tuples)
    assert r.digest == want.digest
    st = r.stats()
    r.free()
    return st


# ------------------------------------------------------------ structures
@pytest.mark.parametrize("name,flags", [("er1k", 0), ("er1k", 1), ("rand", 0), ("rand", 1), ("star", 0),
                                        ("example", 0)])
def test_pcsr_and_signatures_bit_exact(ctx, name, flags):
    if name == "er1k":
        g = w.config_graph("er1k")
    elif name == "rand":
        g = w.random_small_graph(300, 0.05, 3, 5, 11)
    elif name == "star":
        g = w.star_graph(700)
    else:
        g, _ = w.paper_example()
    print("graph", name, flags, flush=True)
    dg = ctx.load(g, flags)
    want = spec.pcsr(g, degenerate=bool(flags))
    info = dg.info()
    assert info["n_edge_labels"] == int(g.elabel.max()) + 1
    assert info["total_groups"] == sum(gl.shape[0] for gl, _ in want.values())
    for l in range(info["n_edge_labels"]):
        gl, ci = dg.pcsr(l)
        if l not in want:
            assert gl.shape[0] == 0 and ci.shape[0] == 0
            continue
        np.testing.assert_array_equal(gl, want[l][0])
        np.testing.assert_array_equal(ci, want[l][1])
    if flags:
        assert info["max_chain"] > 1
    np.testing.assert_array_equal(dg.signatures(), spec.signature_table(g))
    dg.free()


def test_filter_bit_exact(ctx):
    g = w.config_graph("er1k")
    dg = ctx.load(g)
    sig = spec.signature_table(g)
    mk = w.QueryMaker(g)
    for i in range(8):
        q = w.config_query(g, "er1k", i, maker=mk)
        bits, cnt = dg.filter(q)
        cands = spec.filter_candidates(sig, spec.query_signatures(q))
        np.testing.assert_array_equal(bits, spec.filter_bitsets(cands, g.n))
        assert cnt.tolist() == [len(c) for c in cands]
    dg.free()


# ------------------------------------------------------------- end to end
def test_er1k_all_queries(ctx):
    g = w.config_graph("er1k")
    dg = ctx.load(g)
    og = oracle.OracleGraph(g)
    mk = w.QueryMaker(g)
    for i in range(8):
        q = w.config_query(g, "er1k", i, maker=mk)
        check_query(dg, g, q, og)
    dg.free()


@pytest.mark.parametrize("seed", range(25))
def test_random_graphs(ctx, seed):
    r = np.random.default_rng(seed)
    n = int(r.integers(5, 400))
    g = w.random_small_graph(n, float(r.uniform(0.02, 0.4)) if n < 100 else 0.03, int(r.integers(1, 4)),
                             int(r.integers(1, 4)), seed)
    if g.m == 0:
        return
    dg = ctx.load(g)
    og = oracle.OracleGraph(g)
    for t in range(3):
        k = int(r.integers(1, 7))
        q = w.random_connected_query(k, int(r.integers(0, 4)), int(g.vlabel.max()) + 1, int(g.elabel.max()) + 1,
                                     seed * 100 + t)
        check_query(dg, g, q, og)
    dg.free()


def test_closed_forms(ctx):
    perm = lambda n, k: math.factorial(n) // math.factorial(n - k)
    g = w.complete_graph(9)
    dg = ctx.load(g)
    for k in range(1, 8):
        for q in (w.clique_query(k), w.path_query(k), w.star_query(k)):
            r = dg.query(q)
            assert r.count == perm(9, k)
            r.free()
    dg.free()
    g = w.cycle_graph(40)
    dg = ctx.load(g)
    for k in (2, 5, 17, 32):
        r = dg.query(w.path_query(k))
        assert r.count == 80
        r.free()
    r = dg.query(w.cycle_query(7))
    assert r.count == 0
    r.free()
    dg.free()
    g = w.complete_bipartite(4, 6, 0, 1)
    dg = ctx.load(g)
    r = dg.query(w.star_query(5, 0, 1))
    assert r.count == 4 * math.factorial(6) // math.factorial(2)
    r.free()
    dg.free()


def test_dense_queries_past_the_inline_plan(ctx):
    """K_12 has 66 linking edges, more than a plan passed as a kernel argument
    holds (64): the fused workgroup then reads its plan from device memory.
    K_11 (55 edges) takes the argument route.  Both against the oracle."""
    r = np.random.default_rng(77)
    n_cl, n_rest = 14, 200
    vl = list(range(12)) + [0, 1] + [int(x) for x in r.integers(0, 12, n_rest)]
    edges = [(a, b) for a in range(n_cl) for b in range(a + 1, n_cl)]
    seen = set(edges)
    while len(edges) < 91 + 600:  # the clique's 91 edges and 600 random ones
        a, b = sorted(int(x) for x in r.integers(0, n_cl + n_rest, 2))
        if a != b and (a, b) not in seen:
            seen.add((a, b))
            edges.append((a, b))
    g = w.make_graph(n_cl + n_rest, vl, edges, [0] * len(edges))
    dg = ctx.load(g)
    og = oracle.OracleGraph(g)
    import paper_1906_03420_amd as gsi
    for k in (11, 12):
        e = [(a, b) for a in range(k) for b in range(a + 1, k)]
        q = w.make_query(list(range(k)), e, [0] * len(e))
        for flags in (0, gsi.GSI_NO_FUSED, gsi.GSI_COUNT_ONLY):
            st = check_query(dg, g, q, og, flags=flags)
            assert st["k"] == k
    dg.free()


def test_edge_cases(ctx):
    import paper_1906_03420_amd as gsi
    g = w.config_graph("er1k")
    dg = ctx.load(g)
    og = oracle.OracleGraph(g)
    # k = 1: all vertices of the label
    q = w.make_query([2], [], [])
    st = check_query(dg, g, q, og)
    assert st["cand"][0] == int((g.vlabel == 2).sum())
    # absent edge label / absent vertex label -> 0 rows
    for q in (w.make_query([0, 1], [(0, 1)], [5]), w.make_query([0, 9], [(0, 1)], [0])):
        r = dg.query(q)
        assert r.count == 0 and r.rows().shape == (0, 2)
        r.free()
    # invalid queries
    for bad in (w.make_query([0, 0, 0], [(0, 1)], [0]),          # disconnected
                w.make_query([0, 0], [(0, 0)], [0]),              # self-loop
                w.make_query([0, 0], [(0, 1), (1, 0)], [0, 0])):  # repeated pair
        with pytest.raises(gsi.GsiError) as e:
            dg.query(bad)
        assert e.value.status == gsi.GSI_E_INVALID
    # count-only keeps count and digest
    mk = w.QueryMaker(g)
    q = w.config_query(g, "er1k", 0, maker=mk)
    a = dg.query(q)
    b = dg.query(q, flags=gsi.GSI_COUNT_ONLY)
    assert (a.count, a.digest) == (b.count, b.digest)
    with pytest.raises(gsi.GsiError):
        b.rows()
    a.free(); b.free()
    dg.free()
    # invalid graphs
    for bad in (w.make_graph(3, [0, 0, 0], [(0, 0)], [0]), w.make_graph(3, [0, 0, 0], [(0, 1), (1, 0)], [0, 1]),
                w.make_graph(3, [0, 0, 0], [(0, 5)], [0])):
        with pytest.raises(gsi.GsiError) as e:
            ctx.load(bad)
        assert e.value.status == gsi.GSI_E_INVALID
    live, _ = ctx.memory()
    assert live == 0


def test_levels_match_spec(ctx):
    import paper_1906_03420_amd as gsi
    g = w.config_graph("er1k")
    dg = ctx.load(g)
    sig = spec.signature_table(g)
    mk = w.QueryMaker(g)
    nb = spec.neighbour_lists(g)
    for i in range(8):
        q = w.config_query(g, "er1k", i, maker=mk)
        cands = spec.filter_candidates(sig, spec.query_signatures(q))
        order, e0 = spec.plan(q, [len(c) for c in cands], spec.label_frequency(g))
        # Algorithm 4's first edge for every row, then each row's shortest list
        for flags, per_row in ((gsi.GSI_LEVEL_FIRST_EDGE, False), (0, True)):
            r = dg.query(q, flags=flags | gsi.GSI_NO_LIST_FILTER)
            st = r.stats()
            assert st["order"] == order
            assert st["first_edge"][1:] == e0[1:]
            M, lev = spec.join_levels(g, q, cands, order, e0, nb, per_row=per_row)
            for j, L in enumerate(lev, start=1):
                assert (st["rows"][j], st["gba"][j], st["survivors"][j]) == (L["R"], L["GBA"], L["S"])
            np.testing.assert_array_equal(r.rows(), spec.to_query_order(M, order))
            r.free()
    dg.free()


def test_paper_example_join_numbers(ctx, golden_dir):
    import paper_1906_03420_amd as gsi
    gold = json.load(open(os.path.join(golden_dir, "paper_example.json")))
    g, q = w.paper_example()
    dg = ctx.load(g)
    for e0_u2, key in ((1, "gba_e0_label_a"), (0, "gba_e0_label_b")):
        r = dg.query(q, flags=gsi.GSI_FILTER_LABEL_ONLY, order=[0, 1, 2, 3], first_edge=[None, 0, e0_u2, 1])
        st = r.stats()
        assert st["cand"] == [1, 100, 101, 101]
        assert st["gba"][2] == gold[key]["value"]
        assert r.rows().tolist() == [gold["single_match"]["tuple"]]
        r.free()
    r = dg.query(q)
    assert r.rows().tolist() == [gold["single_match"]["tuple"]]
    r.free()
    dg.free()


NO_CHUNKS = 0x10
FUSED_MODES = [dict(), dict(flags=4), dict(flags=NO_CHUNKS),
               dict(flags=NO_CHUNKS, fused_max_rows=64, fused_max_slots=128),
               dict(flags=NO_CHUNKS, fused_max_rows=300, fused_max_slots=64),
               dict(flags=NO_CHUNKS, fused_max_rows=8, fused_max_slots=4096),
               dict(chunk_min_rows=1), dict(chunk_min_rows=1, chunk_rows=1), dict(chunk_min_rows=1, chunk_rows=7)]


def test_root_chunks_partly_left_to_the_per_level_kernels(ctx):
    """Root chunks that cannot hold a level (roots in a 40-clique) finish
    with the per-level kernels while the others (roots on a long cycle)
    finish in their chunks; the merged result is the oracle's."""
    import paper_1906_03420_amd as gsi
    n_cyc, n_cl = 200, 40
    src = list(range(n_cyc))
    dst = [(i + 1) % n_cyc for i in range(n_cyc)]
    for a in range(n_cl):
        for b in range(a + 1, n_cl):
            src.append(n_cyc + a)
            dst.append(n_cyc + b)
    n = n_cyc + n_cl
    g = w.make_graph(n, np.zeros(n, np.uint32), list(zip(src, dst)), np.zeros(len(src), np.uint32))
    q = w.path_query(4)
    og = oracle.OracleGraph(g)
    want = og.match(q, threads=4, tuples=True)
    assert want.count == 2 * n_cyc + n_cl * (n_cl - 1) * (n_cl - 2) * (n_cl - 3)
    dg = ctx.load(g)
    for mode in (dict(chunk_rows=1), dict(chunk_rows=3), dict()):
        mode = dict(mode, chunk_min_rows=1, flags=gsi.GSI_NO_LIST_FILTER)
        print("chunk mode", mode, flush=True)
        res = dg.query(q, **mode)
        stt = res.stats()
        print("chunks", stt["chunks"], "left", stt["chunks_left"], flush=True)
        assert stt["chunks"] > 0
        if "chunk_rows" in mode:
            assert 0 < stt["chunks_left"] < stt["chunks"]
        assert res.count == want.count and res.digest == want.digest
        np.testing.assert_array_equal(res.sorted_rows(), want.tuples)
        ref = dg.query(q, flags=gsi.GSI_NO_FUSED | gsi.GSI_NO_LIST_FILTER)
        assert (stt["rows"], stt["gba"], stt["survivors"]) == (ref.stats()["rows"], ref.stats()["gba"],
                                                               ref.stats()["survivors"])
        ref.free()
        res.free()
        co = dg.query(q, **dict(mode, flags=mode["flags"] | gsi.GSI_COUNT_ONLY))
        assert (co.count, co.digest) == (want.count, want.digest)
        co.free()
    dg.free()


@pytest.mark.parametrize("seed", range(10))
def test_fused_and_per_level_paths_agree(ctx, seed):
    """The fused small-table workgroup, the per-level kernels, and every mix
    forced by low fused capacities give the oracle's result and the same
    per-level sizes."""
    r = np.random.default_rng(1000 + seed)
    n = int(r.integers(50, 400))
    g = w.random_small_graph(n, float(r.uniform(0.01, 0.05)), int(r.integers(1, 3)), int(r.integers(1, 3)), seed + 5)
    if g.m == 0:
        return
    dg = ctx.load(g)
    og = oracle.OracleGraph(g)
    for t in range(3):
        k = int(r.integers(2, 8))
        q = w.random_connected_query(k, int(r.integers(0, 3)), int(g.vlabel.max()) + 1, int(g.elabel.max()) + 1,
                                     seed * 31 + t)
        want = og.match(q, threads=4, max_count=3_000_000)
        if want.status != 0:  # more than 3M embeddings: too large for a tuple-level check
            continue
        ref = None
        for mode in FUSED_MODES:
            print("seed", seed, "query", t, "k", k, "mode", mode, flush=True)
            # per-level sizes are compared as Algorithm 4 defines them
            res = dg.query(q, **dict(mode, flags=mode.get("flags", 0) | 0x8000))
            assert res.count == want.count
            np.testing.assert_array_equal(res.sorted_rows(), want.tuples)
            assert res.digest == want.digest
            stt = res.stats()
            sizes = (stt["rows"], stt["gba"], stt["survivors"])
            if ref is None:
                ref = sizes
            else:
                assert sizes == ref
            res.free()
    dg.free()


def test_profiling_context_gives_identical_results():
    """A context that times every launch (GSI_CTX_PROFILE) gives the same
    answers on every route: per-level kernels with and without list
    filtering, small and large scans, the fused workgroup and root chunks
    (regression: a profiling reduction once overwrote |GBA| in the mailbox
    after k_locate's last workgroup had scanned the row bounds)."""
    import paper_1906_03420_amd as gsi
    pc = gsi.Context(2 << 30, flags=gsi.GSI_CTX_PROFILE)
    try:
        for seed in range(4):
            r = np.random.default_rng(2000 + seed)
            n = int(r.integers(300, 2000))
            g = w.random_small_graph(n, float(r.uniform(0.005, 0.02)), 2, 2, seed + 77)
            if g.m == 0:
                continue
            dg = pc.load(g)
            og = oracle.OracleGraph(g)
            for t in range(3):
                q = w.random_connected_query(int(r.integers(3, 7)), 1, 2, 2, seed * 17 + t)
                want = og.match(q, threads=4, max_count=2_000_000)
                if want.status != 0:
                    continue
                for mode in (dict(flags=4), dict(flags=4 | 0x8000), dict(), dict(chunk_min_rows=1)):
                    print("seed", seed, "query", t, "mode", mode, flush=True)
                    res = dg.query(q, **mode)
                    assert res.count == want.count
                    np.testing.assert_array_equal(res.sorted_rows(), want.tuples)
                    assert res.digest == want.digest
                    res.free()
            dg.free()
        assert any(k["launches"] for k in pc.kernel_stats())
    finally:
        pc.close()


def test_fused_path_er1k_and_count_only(ctx):
    import paper_1906_03420_amd as gsi
    g = w.config_graph("er1k")
    dg = ctx.load(g)
    og = oracle.OracleGraph(g)
    mk = w.QueryMaker(g)
    for i in range(8):
        q = w.config_query(g, "er1k", i, maker=mk)
        want = og.match(q, threads=4)
        for mode in FUSED_MODES:
            a = dg.query(q, **mode)
            b = dg.query(q, flags=mode.get("flags", 0) | gsi.GSI_COUNT_ONLY,
                         **{k2: v for k2, v in mode.items() if k2 != "flags"})
            assert a.count == b.count == want.count
            assert a.digest == b.digest == want.digest
            np.testing.assert_array_equal(a.sorted_rows(), want.tuples)
            a.free(); b.free()
    live, _ = ctx.memory()
    dg.free()


# ------------------------------------------------------------- homomorphism
@pytest.mark.parametrize("seed", range(8))
def test_homomorphism_matches_oracle(ctx, seed):
    """Homomorphism semantics (Sec. VII-A) through every join route."""
    import paper_1906_03420_amd as gsi
    r = np.random.default_rng(3000 + seed)
    n = int(r.integers(20, 200))
    g = w.random_small_graph(n, float(r.uniform(0.03, 0.12)), int(r.integers(1, 3)), int(r.integers(1, 3)), seed + 40)
    if g.m == 0:
        return
    dg = ctx.load(g)
    og = oracle.OracleGraph(g)
    H = gsi.GSI_HOMOMORPHISM
    for t in range(3):
        q = w.random_connected_query(int(r.integers(2, 7)), int(r.integers(0, 3)), int(g.vlabel.max()) + 1,
                                     int(g.elabel.max()) + 1, seed * 100 + t + 7)
        want = og.match(q, threads=4, homomorphism=True, max_count=3_000_000)
        if want.status != 0:
            continue
        for mode in (dict(flags=H), dict(flags=H | 4), dict(flags=H | NO_CHUNKS, fused_max_rows=64,
                     fused_max_slots=128), dict(flags=H, chunk_min_rows=1, chunk_rows=2),
                     dict(flags=H | gsi.GSI_LEVEL_FIRST_EDGE)):
            print("homomorphism seed", seed, "query", t, "k", q.k, "mode", mode, flush=True)
            res = dg.query(q, **mode)
            assert (res.count, res.digest) == (want.count, want.digest)
            np.testing.assert_array_equal(res.sorted_rows(), want.tuples)
            res.free()
    dg.free()


def test_homomorphism_closed_forms(ctx):
    import paper_1906_03420_amd as gsi
    H = gsi.GSI_HOMOMORPHISM
    n = 9
    dg = ctx.load(w.complete_graph(n))
    for k in range(2, 8):
        for q in (w.path_query(k), w.star_query(k)):
            r = dg.query(q, flags=H | gsi.GSI_COUNT_ONLY)
            assert r.count == n * (n - 1) ** (k - 1)
            r.free()
        if k >= 3:
            r = dg.query(w.cycle_query(k), flags=H | gsi.GSI_COUNT_ONLY)
            assert r.count == (n - 1) ** k + (-1) ** k * (n - 1)
            r.free()
    dg.free()
    dg = ctx.load(w.cycle_graph(12))
    for k in (2, 5, 11):
        r = dg.query(w.path_query(k), flags=H)
        assert r.count == 12 * 2 ** (k - 1)
        r.free()
    dg.free()


# ------------------------------------------------------------------ ablations
def JOIN_ABLATIONS(gsi):
    return [gsi.GSI_ABL_NAIVE_SETOPS, gsi.GSI_ABL_ROW_PER_WAVE, gsi.GSI_ABL_ROW_PER_WAVE | gsi.GSI_ABL_DUP_REMOVAL,
            gsi.GSI_ABL_FOUR_LAYER, gsi.GSI_ABL_FOUR_LAYER | gsi.GSI_ABL_DUP_REMOVAL,
            gsi.GSI_ABL_NAIVE_SETOPS | gsi.GSI_LEVEL_FIRST_EDGE, gsi.GSI_ABL_FOUR_LAYER | gsi.GSI_HOMOMORPHISM]


def hub_graph(degrees, every=50):
    """Hubs 0..h-1 of the given degrees over shared leaves h, h+1, ...: hub
    t is joined to the first degrees[t] leaves.  Hubs and leaves have vertex
    label 0, except every `every`-th leaf (label 1); one edge label."""
    h = len(degrees)
    edges = [(t, h + x) for t, d in enumerate(degrees) for x in range(d)]
    n = h + max(degrees)
    vl = [0] * h + [1 if x % every == 0 else 0 for x in range(n - h)]
    return w.make_graph(n, vl, edges, [0] * len(edges), "hubs")


def test_join_ablations_on_hub_rows(ctx):
    """Rows whose scanned lists cross every threshold of the 4-layer balance
    (over W1 = 4096, over W2 = 1024, over W3 = 256, short), with rows that
    scan the same hub list close together (shared by duplicate removal):
    every join variant gives the oracle's rows for the path label 0 - label
    0 - label 1 (closed form: the sum over hubs of their label-0 times their
    label-1 neighbours) and the same per-level sizes."""
    import paper_1906_03420_amd as gsi
    degs = [5000, 2000, 600, 100]
    g = hub_graph(degs)
    closed = sum((d - (d + 49) // 50) * ((d + 49) // 50) for d in degs)
    q = w.make_query([0, 0, 1], [(0, 1), (1, 2)], [0, 0])
    want = oracle.match(g, q, threads=8)
    assert want.count == closed == 575652
    dg = ctx.load(g)
    ref = None
    for f in [gsi.GSI_NO_FUSED] + JOIN_ABLATIONS(gsi):
        for co in (gsi.GSI_COUNT_ONLY, 0):
            print("hub rows, flags", hex(f | co), flush=True)
            r = dg.query(q, flags=f | co)
            assert (r.count, r.digest) == (want.count, want.digest), hex(f)
            if not co:
                np.testing.assert_array_equal(r.sorted_rows(), want.tuples)
            st = r.stats()
            sizes = (st["rows"], st["gba"], st["survivors"])
            if f == gsi.GSI_NO_FUSED:
                # the level-wide filtered lists: level 2's rows scan the
                # label-0 leaves of their hub only
                assert st["filtered_levels"] == 1 << 2
                assert st["gba"][2] == closed
                r.free()
                continue
            if not f & gsi.GSI_LEVEL_FIRST_EDGE:
                ref = ref or sizes
                assert sizes == ref
            r.free()
    assert max(ref[1]) > 4096 * 100  # the heavy rows were there
    with pytest.raises(gsi.GsiError):
        dg.query(q, flags=gsi.GSI_ABL_DUP_REMOVAL)
    with pytest.raises(gsi.GsiError):
        dg.query(q, flags=gsi.GSI_ABL_NAIVE_SETOPS | gsi.GSI_ABL_FOUR_LAYER)
    dg.free()


def test_ablations_give_identical_results(ctx):
    """Compressed-representation lookup, two-step output, unstaged row
    writes and the join ablations change only how the per-level kernels
    work, never the result (under either semantics)."""
    import paper_1906_03420_amd as gsi
    modes = [dict(flags=gsi.GSI_ABL_CR), dict(flags=gsi.GSI_ABL_TWO_STEP), dict(flags=gsi.GSI_ABL_NO_STAGING),
             dict(flags=gsi.GSI_ABL_CR | gsi.GSI_ABL_TWO_STEP | gsi.GSI_ABL_NO_STAGING | gsi.GSI_COUNT_ONLY)]
    modes += [dict(flags=f) for f in JOIN_ABLATIONS(gsi)]
    for seed in range(6):
        r = np.random.default_rng(4000 + seed)
        n = int(r.integers(50, 400))
        g = w.random_small_graph(n, float(r.uniform(0.01, 0.05)), int(r.integers(1, 3)), int(r.integers(1, 3)),
                                 seed + 60)
        if g.m == 0:
            continue
        dg = ctx.load(g, gsi.GSI_GRAPH_KEEP_CR)
        plain = ctx.load(g)
        og = oracle.OracleGraph(g)
        for t in range(3):
            q = w.random_connected_query(int(r.integers(2, 8)), int(r.integers(0, 3)), int(g.vlabel.max()) + 1,
                                         int(g.elabel.max()) + 1, seed * 100 + t + 9)
            want = og.match(q, threads=4, max_count=3_000_000)
            if want.status != 0:
                continue
            # a homomorphism mode is held to the oracle's homomorphism mode
            want_h = None
            for mode in modes:
                print("ablation seed", seed, "query", t, "mode", mode, flush=True)
                ref = want
                if mode["flags"] & gsi.GSI_HOMOMORPHISM:
                    if want_h is None:
                        want_h = og.match(q, threads=4, homomorphism=True, max_count=3_000_000)
                    if want_h.status != 0:
                        continue
                    ref = want_h
                res = dg.query(q, **mode)
                assert (res.count, res.digest) == (ref.count, ref.digest)
                if not mode["flags"] & gsi.GSI_COUNT_ONLY:
                    np.testing.assert_array_equal(res.sorted_rows(), ref.tuples)
                res.free()
            with pytest.raises(gsi.GsiError):
                plain.query(q, flags=gsi.GSI_ABL_CR)
        plain.free()
        dg.free()


@pytest.mark.parametrize("seed", range(4))
def test_single_pass_last_level_and_list_filter(ctx, seed):
    """The one-pass last level (decoupled look-back) and the level-wide
    filtered lists give the same rows in the same order as the separate
    join / scan / link launches on unfiltered lists, and the oracle's set."""
    import paper_1906_03420_amd as gsi
    r = np.random.default_rng(9000 + seed)
    n = int(r.integers(200, 2000))
    g = w.random_small_graph(n, float(r.uniform(0.005, 0.03)), int(r.integers(1, 3)), int(r.integers(1, 3)),
                             seed + 90)
    if g.m == 0:
        return
    dg = ctx.load(g)
    og = oracle.OracleGraph(g)
    base = gsi.GSI_NO_FUSED
    for t in range(4):
        q = w.random_connected_query(int(r.integers(2, 7)), int(r.integers(0, 3)), int(g.vlabel.max()) + 1,
                                     int(g.elabel.max()) + 1, seed * 77 + t)
        want = og.match(q, threads=4, max_count=3_000_000)
        if want.status != 0:
            continue
        ref = dg.query(q, flags=base | gsi.GSI_NO_LIST_FILTER)
        rows = ref.rows()
        for f in (base, base | gsi.GSI_SINGLE_PASS, base | gsi.GSI_SINGLE_PASS | gsi.GSI_NO_LIST_FILTER, 0,
                  gsi.GSI_SINGLE_PASS):
            res = dg.query(q, flags=f)
            assert (res.count, res.digest) == (want.count, want.digest)
            if f & gsi.GSI_NO_FUSED:
                np.testing.assert_array_equal(res.rows(), rows)  # same order
            np.testing.assert_array_equal(res.sorted_rows(), want.tuples)
            res.free()
            co = dg.query(q, flags=f | gsi.GSI_COUNT_ONLY)
            assert (co.count, co.digest) == (want.count, want.digest)
            co.free()
        ref.free()
    dg.free()


def test_one_pass_levels_on_a_clique(ctx):
    """K_20 and a 5-vertex path (20!/15! embeddings): levels 2-4 rescan the
    same 19-element lists, so all three filter them level-wide and run in one
    pass (levels 2-3 write the next table at |GBA| rows per column, level 4
    the rows); rows in the same order as the separate launches, the oracle's
    set."""
    import paper_1906_03420_amd as gsi
    g = w.complete_graph(20)
    q = w.path_query(5)
    want = oracle.match(g, q, threads=4)
    assert want.count == math.perm(20, 5)
    dg = ctx.load(g)
    ref = dg.query(q, flags=gsi.GSI_NO_FUSED | gsi.GSI_NO_LIST_FILTER)
    r = dg.query(q, flags=gsi.GSI_NO_FUSED | gsi.GSI_SINGLE_PASS)
    st = r.stats()
    assert st["filtered_levels"] == 0b11100
    # every vertex is a candidate here, so the filtered lists are whole
    assert st["gba"][4] == math.perm(20, 4) * 19
    assert (st["rows"], st["gba"], st["survivors"]) == (ref.stats()["rows"], ref.stats()["gba"],
                                                       ref.stats()["survivors"])
    np.testing.assert_array_equal(r.rows(), ref.rows())
    np.testing.assert_array_equal(r.sorted_rows(), want.tuples)
    assert r.digest == want.digest
    r.free()
    ref.free()
    dg.free()
