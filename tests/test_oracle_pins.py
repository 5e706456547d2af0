"""Pins of the CPU oracle against things other than itself: brute force,
closed forms, linear algebra, the paper's worked example, published hash test
vectors.  CPU only."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as w


def brute_force(g, q):
    """Every injective map V(Q)->V(G) checked against Definitions 1-3."""
    E = {}
    for a, b, l in zip(g.src.tolist(), g.dst.tolist(), g.elabel.tolist()):
        E[frozenset((a, b))] = l
    out = []
    for f in itertools.permutations(range(g.n), q.k):
        if any(int(g.vlabel[f[u]]) != int(q.vlabel[u]) for u in range(q.k)):
            continue
        ok = True
        for a, b, l in zip(q.src.tolist(), q.dst.tolist(), q.elabel.tolist()):
            if E.get(frozenset((f[a], f[b]))) != l:
                ok = False
                break
        if ok:
            out.append(f)
    return np.array(sorted(out), np.uint32).reshape(-1, q.k)


@pytest.mark.parametrize("seed", range(40))
def test_oracle_matches_brute_force(seed):
    r = np.random.default_rng(seed)
    n = int(r.integers(4, 9))
    g = w.random_small_graph(n, float(r.uniform(0.3, 0.9)), int(r.integers(1, 3)), int(r.integers(1, 3)), seed)
    k = int(r.integers(1, min(n, 5) + 1))
    q = w.random_connected_query(k, int(r.integers(0, 3)), int(g.vlabel.max()) + 1, int(g.elabel.max()) + 1 if g.m else 1, seed + 1000)
    want = brute_force(g, q)
    for threads in (1, 3):
        got = oracle.match(g, q, threads=threads)
        assert got.status == oracle.OR_OK
        assert got.count == len(want)
        np.testing.assert_array_equal(got.tuples, want)
        assert got.digest == oracle.digest_rows(want)


def perm(n, k):
    return math.factorial(n) // math.factorial(n - k)


@pytest.mark.parametrize("n,k", [(5, 1), (5, 2), (6, 3), (7, 4), (8, 5), (9, 6)])
def test_closed_form_cliques(n, k):
    # any connected k-vertex query on K_n (uniform labels): n!/(n-k)! embeddings
    g = w.complete_graph(n)
    for q in (w.clique_query(k), w.path_query(k), w.star_query(k)):
        assert oracle.match(g, q, tuples=False, threads=2).count == perm(n, k)


@pytest.mark.parametrize("n", [3, 5, 8, 13])
def test_closed_form_cycles(n):
    g = w.cycle_graph(n)
    for k in range(2, n + 1):
        assert oracle.match(g, w.path_query(k), tuples=False).count == 2 * n
    for k in range(3, n):
        assert oracle.match(g, w.cycle_query(k), tuples=False).count == 0
    assert oracle.match(g, w.cycle_query(n), tuples=False).count == 2 * n


@pytest.mark.parametrize("n,k", [(4, 3), (6, 3), (6, 5), (9, 4)])
def test_closed_form_stars(n, k):
    g = w.star_graph(n)
    assert oracle.match(g, w.star_query(k), tuples=False).count == math.factorial(n - 1) // math.factorial(n - k)


@pytest.mark.parametrize("a,b,k", [(3, 4, 3), (2, 5, 4), (4, 6, 5)])
def test_closed_form_bipartite_star(a, b, k):
    g = w.complete_bipartite(a, b, 0, 1)
    q = w.star_query(k, 0, 1)
    assert oracle.match(g, q, tuples=False).count == a * math.factorial(b) // math.factorial(b - k + 1)


def test_absent_edge_label_gives_zero():
    g = w.complete_graph(6)
    q = w.make_query([0, 0, 0], [(0, 1), (1, 2)], [0, 7])
    assert oracle.match(g, q).count == 0


def test_single_edge_count_is_twice_edges():
    g = w.config_graph("er1k")
    g.vlabel[:] = 0
    g.elabel[:] = 0
    q = w.path_query(2)
    assert oracle.match(g, q, tuples=False, threads=4).count == 2 * g.m


def _adj(g, lab=None, vl=None):
    A = np.zeros((g.n, g.n), np.int64)
    for a, b, l in zip(g.src, g.dst, g.elabel):
        if lab is None or l == lab:
            A[a, b] = A[b, a] = 1
    return A


def test_algebra_uniform_triangles():
    g = w.random_small_graph(60, 0.2, 1, 1, 7)
    A = _adj(g)
    assert oracle.match(g, w.clique_query(3), tuples=False, threads=4).count == int(np.trace(A @ A @ A))


def test_algebra_labelled_triangle_and_two_path():
    g = w.config_graph("er1k")
    A = [_adj(g, l) for l in range(2)]
    mask = [np.diag((g.vlabel == x).astype(np.int64)) for x in range(4)]
    # labelled triangle u0(x)-u1(y)-u2(z) with edge labels l01, l12, l20
    x, y, z, l01, l12, l20 = 0, 1, 0, 0, 1, 1
    P = mask[x] @ A[l01] @ mask[y] @ A[l12] @ mask[z] @ A[l20] @ mask[x]
    q = w.make_query([x, y, z], [(0, 1), (1, 2), (0, 2)], [l01, l12, l20])
    assert oracle.match(g, q, tuples=False, threads=4).count == int(np.trace(P))
    # labelled 2-path u0(x) -l1- u1(y) -l2- u2(zz): sum over centres of degree products
    for (x, y, zz, l1, l2) in [(0, 1, 2, 0, 1), (3, 3, 3, 0, 0), (2, 1, 2, 1, 1)]:
        d1 = A[l1] @ (g.vlabel == x).astype(np.int64)
        d2 = A[l2] @ (g.vlabel == zz).astype(np.int64)
        cen = g.vlabel == y
        expect = int(np.sum(d1[cen] * d2[cen]))
        if x == zz and l1 == l2:
            expect -= int(np.sum(d1[cen]))  # the two ends may not coincide
        q = w.make_query([x, y, zz], [(0, 1), (1, 2)], [l1, l2])
        assert oracle.match(g, q, tuples=False).count == expect


def test_paper_example(golden_dir):
    gold = json.load(open(os.path.join(golden_dir, "paper_example.json")))
    g, q = w.paper_example()
    r = oracle.match(g, q)
    assert r.count == 1
    assert r.tuples.tolist() == [gold["single_match"]["tuple"]]


def test_hash_test_vectors():
    # FNV-1a 64-bit published test vectors (Fowler/Noll/Vo)
    assert oracle.fnv1a64(b"") == 0xCBF29CE484222325
    assert oracle.fnv1a64(b"a") == 0xAF63DC4C8601EC8C
    assert oracle.fnv1a64(b"foobar") == 0x85944171F73967E8
    # first SplitMix64 output from state 0 = finalizer(golden gamma)
    assert oracle.splitmix64_finalize(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF
    # FNV-1a over 32-bit symbols is the octet form when every symbol is
    # below 256: the published vectors again, through the word function
    assert oracle.fnv1a64_words([]) == 0xCBF29CE484222325
    assert oracle.fnv1a64_words([ord("a")]) == 0xAF63DC4C8601EC8C
    assert oracle.fnv1a64_words([ord(c) for c in "foobar"]) == 0x85944171F73967E8


def test_digest_is_order_independent_and_sensitive():
    rng = np.random.default_rng(3)
    rows = rng.integers(0, 1 << 32, (500, 5), dtype=np.uint64).astype(np.uint32)
    d = oracle.digest_rows(rows)
    assert oracle.digest_rows(rows[::-1]) == d
    rows2 = rows.copy()
    rows2[17, 3] ^= 1
    assert oracle.digest_rows(rows2) != d
    # the tuple hash takes the k values as FNV symbols in query-vertex order:
    # with values below 256, the octet FNV-1a of those values
    t = np.array([1, 2], np.uint32)
    assert oracle.tuple_hash(t) == oracle.splitmix64_finalize(oracle.fnv1a64(b"\x01\x02"))
    assert oracle.tuple_hash(np.array([2, 1], np.uint32)) != oracle.tuple_hash(t)
    # a value's high bits count: 0x100 is not 0x00
    assert oracle.tuple_hash(np.array([0x100], np.uint32)) != oracle.tuple_hash(np.array([0], np.uint32))


def test_invalid_inputs_rejected():
    with pytest.raises(ValueError):
        oracle.OracleGraph(w.make_graph(3, [0, 0, 0], [(0, 0)], [0]))
    with pytest.raises(ValueError):
        oracle.OracleGraph(w.make_graph(3, [0, 0, 0], [(0, 1), (1, 0)], [0, 1]))
    g = w.complete_graph(5)
    q = w.make_query([0, 0, 0, 0], [(0, 1), (2, 3)], [0, 0])  # disconnected
    assert oracle.match(g, q).status == oracle.OR_INVALID


def test_vertex_relabelling_invariance():
    g = w.config_graph("er1k")
    mk = w.QueryMaker(g)
    q = w.config_query(g, "er1k", 3, maker=mk)
    r0 = oracle.match(g, q, threads=2)
    p = np.random.default_rng(5).permutation(g.n).astype(np.uint32)
    inv = np.argsort(p).astype(np.uint32)
    g2 = w.Graph(g.n, g.vlabel[inv], p[g.src], p[g.dst], g.elabel.copy())
    r1 = oracle.match(g2, q, threads=2)
    back = np.sort(inv[r1.tuples].view([("", np.uint32)] * q.k), axis=0).view(np.uint32).reshape(-1, q.k)
    np.testing.assert_array_equal(back, r0.tuples)


def test_walk_query_contains_its_source():
    g = w.config_graph("er1k")
    mk = w.QueryMaker(g)
    for i in range(8):
        q = w.config_query(g, "er1k", i, maker=mk)
        r = oracle.match(g, q)
        assert r.count >= 1
        assert any((r.tuples == q.source).all(axis=1))


# ------------------------------------------------------------ homomorphism
def brute_force_hom(g, q):
    """Every map V(Q)->V(G), injective or not, that keeps vertex labels and
    maps each query edge onto a data edge of the same label (Sec. VII-A)."""
    E = {}
    for a, b, l in zip(g.src.tolist(), g.dst.tolist(), g.elabel.tolist()):
        E[frozenset((a, b))] = l
    out = []
    for f in itertools.product(range(g.n), repeat=q.k):
        if any(int(g.vlabel[f[u]]) != int(q.vlabel[u]) for u in range(q.k)):
            continue
        if all(f[a] != f[b] and E.get(frozenset((f[a], f[b]))) == l
               for a, b, l in zip(q.src.tolist(), q.dst.tolist(), q.elabel.tolist())):
            out.append(f)
    return np.array(sorted(out), np.uint32).reshape(-1, q.k)


@pytest.mark.parametrize("seed", range(30))
def test_oracle_homomorphism_matches_brute_force(seed):
    r = np.random.default_rng(500 + seed)
    n = int(r.integers(3, 7))
    g = w.random_small_graph(n, float(r.uniform(0.3, 0.9)), int(r.integers(1, 3)), int(r.integers(1, 3)), seed)
    k = int(r.integers(1, 5))
    q = w.random_connected_query(k, int(r.integers(0, 3)), int(g.vlabel.max()) + 1, int(g.elabel.max()) + 1 if g.m else 1, seed + 2000)
    want = brute_force_hom(g, q)
    for threads in (1, 2):
        got = oracle.match(g, q, threads=threads, homomorphism=True)
        assert got.status == oracle.OR_OK
        np.testing.assert_array_equal(got.tuples, want)
        assert got.digest == oracle.digest_rows(want)
    # every embedding is a homomorphism
    inj = oracle.match(g, q)
    assert inj.count <= len(want)


@pytest.mark.parametrize("n", [3, 4, 6, 9])
def test_homomorphism_closed_forms(n):
    g = w.complete_graph(n)
    for k in range(1, 6):
        # trees into K_n: n (n-1)^(k-1); cycles: the chromatic polynomial of C_k
        assert oracle.match(g, w.path_query(k), tuples=False, homomorphism=True).count == n * (n - 1) ** (k - 1)
        assert oracle.match(g, w.star_query(k), tuples=False, homomorphism=True).count == n * (n - 1) ** (k - 1)
        if k >= 3:
            want = (n - 1) ** k + (-1) ** k * (n - 1)
            assert oracle.match(g, w.cycle_query(k), tuples=False, homomorphism=True).count == want
    c = w.cycle_graph(n + 2)
    for k in range(1, 7):
        # a walk of k vertices on a cycle: a start, then two ways each step
        assert oracle.match(c, w.path_query(k), tuples=False, homomorphism=True).count == (n + 2) * 2 ** (k - 1)
