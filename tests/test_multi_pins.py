"""CPU pins of the multi-label oracle (Sec. VII-B semantics): brute force over
all injective maps on tiny graphs, agreement with the separately written
single-label oracle when every set has one label, and closed forms."""
import itertools
import math

import numpy as np
import pytest

import oracle
import workloads as w


def brute_multi(g, q):
    """Every injective map f with L(u) within L(f(u)) and the labels of every
    query pair within the labels of its image pair, by enumeration."""
    elab = {}
    for a, b, l in zip(g.src.tolist(), g.dst.tolist(), g.elabel.tolist()):
        elab.setdefault(frozenset((a, b)), set()).add(l)
    need = {}
    for a, b, l in zip(q.src.tolist(), q.dst.tolist(), q.elabel.tolist()):
        need.setdefault((a, b), set()).add(l)
    out = []
    for f in itertools.permutations(range(g.n), q.k):
        if not all(set(q.labels(u)) <= set(g.labels(f[u])) for u in range(q.k)):
            continue
        if all(ls <= elab.get(frozenset((f[a], f[b])), set()) for (a, b), ls in need.items()):
            out.append(f)
    return np.array(sorted(out), np.uint32).reshape(-1, q.k)


@pytest.mark.parametrize("seed", range(30))
def test_multi_oracle_brute_force(seed):
    r = np.random.default_rng(seed)
    n = int(r.integers(3, 8))
    g = w.random_multi_graph(n, float(r.uniform(0.3, 0.9)), 3, 3, 2, 2, seed)
    if g.m == 0:
        return
    k = int(r.integers(1, min(n, 4) + 1))
    try:
        q = w.multi_walk_query(g, k, seed + 100, dense=bool(seed % 2))
    except RuntimeError:
        return
    want = brute_multi(g, q)
    for threads in (1, 3):
        got = oracle.match_multi(g, q, threads=threads)
        assert got.status == 0
        assert got.count == len(want) >= 1
        np.testing.assert_array_equal(got.tuples, want)
        assert got.digest == oracle.digest_rows(want)


def test_multi_oracle_equals_single_label_oracle():
    """Singleton label sets: the multi-label oracle (multi.c) and the
    single-label oracle (match.c), written separately, agree exactly."""
    for seed in range(6):
        g = w.random_small_graph(120, 0.05, 3, 2, seed + 40)
        mg = w.mgraph_from_single(g)
        og, om = oracle.OracleGraph(g), oracle.OracleMultiGraph(mg)
        for t in range(4):
            q = w.random_connected_query(int(2 + t), t % 2, 3, 2, seed * 10 + t)
            a = og.match(q, threads=2)
            b = om.match(w.mquery_from_single(q), threads=2)
            assert (a.status, b.status) == (0, 0)
            assert a.count == b.count and a.digest == b.digest
            np.testing.assert_array_equal(a.tuples, b.tuples)
    g = w.config_graph("er1k")
    mk = w.QueryMaker(g)
    og, om = oracle.OracleGraph(g), oracle.OracleMultiGraph(w.mgraph_from_single(g))
    for i in range(8):
        q = w.config_query(g, "er1k", i, maker=mk)
        a, b = og.match(q), om.match(w.mquery_from_single(q))
        assert a.count == b.count and a.digest == b.digest


def test_multi_oracle_closed_forms():
    n = 7
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
    # K_n, every vertex labelled {0, 1}, every pair labelled {0, 1}
    g = w.make_mgraph(n, [[0, 1]] * n, [(a, b, l) for a, b in pairs for l in (0, 1)])
    for k in range(1, 5):
        clique = [(a, b) for a in range(k) for b in range(a + 1, k)]
        for vsets, ls in (([[0]] * k, (1,)), ([[0, 1]] * k, (0, 1)), ([[1]] * k, (0,))):
            q = w.make_mquery(vsets, [(a, b, l) for a, b in clique for l in ls])
            assert oracle.match_multi(g, q).count == math.perm(n, k)
        # a label no vertex has
        q = w.make_mquery([[0, 2]] + [[0]] * (k - 1), [(a, b, 0) for a, b in clique])
        assert oracle.match_multi(g, q).count == 0
    # K_n with label 0 on every pair and label 1 only on the cycle pairs
    # (i, i+1 mod n): a k-path asking both labels on every edge follows the
    # cycle (2n maps for 2 <= k < n)
    cyc = {(min(i, (i + 1) % n), max(i, (i + 1) % n)) for i in range(n)}
    g = w.make_mgraph(n, [[0]] * n, [(a, b, 0) for a, b in pairs] + [(a, b, 1) for a, b in sorted(cyc)])
    for k in range(2, n):
        q = w.make_mquery([[0]] * k, [(i, i + 1, l) for i in range(k - 1) for l in (0, 1)])
        assert oracle.match_multi(g, q).count == 2 * n
        q = w.make_mquery([[0]] * k, [(i, i + 1, 0) for i in range(k - 1)])
        assert oracle.match_multi(g, q).count == math.perm(n, k)


def test_multi_oracle_rejects_bad_input():
    g = w.make_mgraph(3, [[0], [0], [0]], [(0, 1, 0), (0, 1, 0)])
    with pytest.raises(ValueError):
        oracle.OracleMultiGraph(g)
    g = w.make_mgraph(3, [[0], [0], [0]], [(0, 1, 0), (0, 1, 1), (1, 2, 0)])
    og = oracle.OracleMultiGraph(g)
    q = w.make_mquery([[0], [0], [0]], [(0, 1, 0)])  # disconnected
    assert og.match(q).status == oracle.OR_INVALID
    q = w.make_mquery([[0], [0]], [(0, 1, 0), (1, 0, 0)])  # same pair and label twice
    assert og.match(q).status == oracle.OR_INVALID
    q = w.make_mquery([[0], [0]], [(0, 1, 0), (1, 0, 1)])  # two labels on one pair
    assert og.match(q).count == 2
