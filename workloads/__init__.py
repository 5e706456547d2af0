"""Seeded synthetic inputs: labelled data graphs and random-walk query graphs.

This module is the only code shared by the CPU oracle side (tests, the bench's
CPU baseline) and the GPU library side: it *generates* inputs and holds none
of the matching method's arithmetic.  Every generator is deterministic in its
seed.  Graph models and PRNG are documented in ``gen.c``.

Workload recipes (the paper's datasets, Sec. VIII-A / Table III, are not
available; these synthetic graphs stand in for them, with power-law labels as
in Sec. VIII-A and random-walk queries as in the same section):

  ER-1K     Erdos-Renyi, 1,000 vertices, 5,000 edges, 4 vertex labels and
            2 edge labels uniform; 8 walk queries with 4 vertices.
  BA-1M     Barabasi-Albert (Batagelj-Brandes), 1,000,000 vertices, seed K_11
            and 10 attachments per vertex (9,999,945 edges); 32 vertex labels
            Zipf(1.1), 8 edge labels uniform; 100 walk queries, 6..12 vertices.
  BA-1M-B   the BA-1M graph with 1,024 queries of 4..16 vertices, shapes tree,
            walk with a cycle (|E(Q)| >= |V(Q)|) and dense (all data edges among
            the walk's vertices), for the batched path.
  RMAT-23   R-MAT scale 23, 100M edges, (a,b,c) = (0.57,0.19,0.19); 100 vertex
            labels and 20 edge labels Zipf(1.1); 50 queries of 12 vertices
            (25 walk + 25 dense).
  RMAT-22-S R-MAT scale 22, 50M edges, the same (a,b,c); 64 vertex labels and
            16 edge labels Zipf(1.1); a pool of 512 queries of 4..24 vertices
            with the BA-1M-B shapes, for the serving loop: each offered rate
            serves 2,000 requests drawn from the pool (``request_stream``),
            arriving as a Poisson process (unit-rate gaps from
            ``arrival_gaps``, scaled by the caller to the offered rate).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libgen.so")
_lib = None

U32P = ctypes.POINTER(ctypes.c_uint32)


def build(force: bool = False) -> str:
    """Compile gen.c into libgen.so (gcc, host code only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.gen_er.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, U32P, U32P]
        lib.gen_er.restype = ctypes.c_int
        lib.gen_ba_edge_count.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        lib.gen_ba_edge_count.restype = ctypes.c_uint64
        lib.gen_ba.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, U32P, U32P]
        lib.gen_ba.restype = ctypes.c_int
        lib.gen_rmat.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_uint64, U32P, U32P]
        lib.gen_rmat.restype = ctypes.c_int
        lib.gen_labels_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, U32P]
        lib.gen_labels_uniform.restype = None
        lib.gen_labels_zipf.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_uint64, U32P]
        lib.gen_labels_zipf.restype = None
        lib.gen_qctx_create.argtypes = [ctypes.c_uint32, U32P, ctypes.c_uint64, U32P, U32P, U32P]
        lib.gen_qctx_create.restype = ctypes.c_void_p
        lib.gen_qctx_free.argtypes = [ctypes.c_void_p]
        lib.gen_qctx_free.restype = None
        lib.gen_query.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint64,
                                  U32P, U32P, U32P, U32P, U32P]
        lib.gen_query.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.uint32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(U32P)


@dataclass
class Graph:
    """Undirected labelled graph: one label per vertex and per edge."""
    n: int
    vlabel: np.ndarray  # uint32[n]
    src: np.ndarray     # uint32[m]
    dst: np.ndarray     # uint32[m]
    elabel: np.ndarray  # uint32[m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


@dataclass
class Query:
    """Connected query graph with vertices 0..k-1."""
    k: int
    vlabel: np.ndarray
    src: np.ndarray
    dst: np.ndarray
    elabel: np.ndarray
    mode: str = ""
    seed: int = 0
    source: np.ndarray = field(default_factory=lambda: np.zeros(0, np.uint32))

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def _u32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint32))


def make_graph(n, vlabel, edges, elabel, name="") -> Graph:
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    return Graph(int(n), _u32(vlabel), _u32(e[:, 0]), _u32(e[:, 1]), _u32(elabel), name)


def make_query(vlabel, edges, elabel, mode="manual") -> Query:
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    return Query(len(vlabel), _u32(vlabel), _u32(e[:, 0]), _u32(e[:, 1]), _u32(elabel), mode)


# ------------------------------------------------------------------ labels
def labels_uniform(n: int, nl: int, seed: int) -> np.ndarray:
    out = np.empty(n, np.uint32)
    _load().gen_labels_uniform(n, nl, seed, _p(out))
    return out


def labels_zipf(n: int, nl: int, s: float, seed: int) -> np.ndarray:
    out = np.empty(n, np.uint32)
    _load().gen_labels_zipf(n, nl, s, seed, _p(out))
    return out


# ------------------------------------------------------------------ models
def er_edges(n: int, m: int, seed: int):
    src = np.empty(m, np.uint32)
    dst = np.empty(m, np.uint32)
    rc = _load().gen_er(n, m, seed, _p(src), _p(dst))
    if rc:
        raise ValueError("gen_er failed: %d" % rc)
    return src, dst


def ba_edges(n: int, d: int, seed: int):
    lib = _load()
    m = int(lib.gen_ba_edge_count(n, d))
    src = np.empty(m, np.uint32)
    dst = np.empty(m, np.uint32)
    rc = lib.gen_ba(n, d, seed, _p(src), _p(dst))
    if rc:
        raise ValueError("gen_ba failed: %d" % rc)
    return src, dst


def rmat_edges(scale: int, m: int, a: float, b: float, c: float, seed: int):
    src = np.empty(m, np.uint32)
    dst = np.empty(m, np.uint32)
    rc = _load().gen_rmat(scale, m, a, b, c, seed, _p(src), _p(dst))
    if rc:
        raise ValueError("gen_rmat failed: %d" % rc)
    return src, dst


# ----------------------------------------------------------------- queries
MODES = {"walk": 0, "tree": 1, "dense": 2, "walk_cycle": 3}


class QueryMaker:
    """Random-walk query extraction over one data graph (Sec. VIII-A recipe)."""

    def __init__(self, g: Graph):
        self.g = g
        self._lib = _load()
        self._h = self._lib.gen_qctx_create(g.n, _p(g.vlabel), g.m, _p(g.src), _p(g.dst), _p(g.elabel))

    def close(self):
        if self._h:
            self._lib.gen_qctx_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def make(self, k: int, mode: str, seed: int) -> Query:
        cap = max(1, k * (k - 1) // 2)
        ql = np.empty(k, np.uint32)
        qs = np.empty(cap, np.uint32)
        qd = np.empty(cap, np.uint32)
        qe = np.empty(cap, np.uint32)
        srcv = np.empty(k, np.uint32)
        ne = self._lib.gen_query(self._h, k, MODES[mode], seed, _p(ql), _p(qs), _p(qd), _p(qe), _p(srcv))
        if ne < 0:
            raise RuntimeError("no random walk reached %d vertices" % k)
        return Query(k, ql, qs[:ne].copy(), qd[:ne].copy(), qe[:ne].copy(), mode, seed, srcv)


def _stream(seed: int, i: int) -> np.random.Generator:
    return np.random.default_rng([seed, i])


def query_seed(base: int, index: int, attempt: int = 0) -> int:
    """Seed of query `index` (redrawn as `attempt` grows)."""
    return (base << 32) ^ (index << 12) ^ attempt


def query_spec(base: int, index: int, kmin: int, kmax: int, modes) -> tuple:
    """(k, mode) of query `index`: k uniform in [kmin, kmax], mode uniform over `modes`."""
    r = _stream(base, index)
    k = int(r.integers(kmin, kmax + 1))
    mode = modes[int(r.integers(0, len(modes)))]
    return k, mode


# ----------------------------------------------------------------- configs
CONFIGS = {
    "er1k": dict(model="er", n=1000, m=5000, nvl=4, nel=2, vdist="uniform", edist="uniform",
                 gseed=17, lseed=2017, qseed=1017, nq=8, kmin=4, kmax=4, modes=("walk",)),
    "ba1m": dict(model="ba", n=1_000_000, d=10, nvl=32, nel=8, vdist="zipf", edist="uniform",
                 gseed=18, lseed=2018, qseed=1018, nq=100, kmin=6, kmax=12, modes=("walk",)),
    "ba1m_batch": dict(model="ba", n=1_000_000, d=10, nvl=32, nel=8, vdist="zipf", edist="uniform",
                       gseed=18, lseed=2018, qseed=1020, nq=1024, kmin=4, kmax=16,
                       modes=("tree", "walk_cycle", "dense")),
    "rmat23": dict(model="rmat", scale=23, m=100_000_000, nvl=100, nel=20, vdist="zipf", edist="zipf",
                   gseed=19, lseed=2019, qseed=1019, nq=50, kmin=12, kmax=12, modes=("walk", "dense")),
    "rmat22_serve": dict(model="rmat", scale=22, m=50_000_000, nvl=64, nel=16, vdist="zipf", edist="zipf",
                         gseed=21, lseed=2021, qseed=1021, nq=512, kmin=4, kmax=24,
                         modes=("tree", "walk_cycle", "dense"), aseed=3021, requests=2000),
}


def arrival_gaps(name: str, stream: int, n: int) -> np.ndarray:
    """Inter-arrival gaps of a unit-rate Poisson process (mean 1), seeded by
    the workload's arrival seed and a stream number (one per offered rate)."""
    return _stream(CONFIGS[name]["aseed"], stream).exponential(1.0, n)


def request_stream(name: str, stream: int, n: int, pool: int) -> np.ndarray:
    """Which pool query each of `n` requests asks (uniform, with repeats)."""
    return _stream(CONFIGS[name]["aseed"] + 1, stream).integers(0, pool, n)


def config_graph(name: str) -> Graph:
    """The named workload's data graph.  With GSI_GRAPH_CACHE set to a
    directory, the generated arrays are kept there as .npy files and later
    calls (other processes included) load them instead of regenerating."""
    cache = os.environ.get("GSI_GRAPH_CACHE")
    if cache:
        base = os.path.join(cache, "%s_" % name)
        files = [base + x + ".npy" for x in ("vl", "src", "dst", "el")]
        if all(os.path.exists(f) for f in files):
            vl, src, dst, el = (np.load(f) for f in files)
            return Graph(int(vl.shape[0]), vl, src, dst, el, name)
        g = _generate(name)
        os.makedirs(cache, exist_ok=True)
        for f, a in zip(files, (g.vlabel, g.src, g.dst, g.elabel)):
            np.save(f + ".tmp.npy", a)
            os.replace(f + ".tmp.npy", f)
        return g
    return _generate(name)


def _generate(name: str) -> Graph:
    c = CONFIGS[name]
    if c["model"] == "er":
        src, dst = er_edges(c["n"], c["m"], c["gseed"])
        n = c["n"]
    elif c["model"] == "ba":
        src, dst = ba_edges(c["n"], c["d"], c["gseed"])
        n = c["n"]
    elif c["model"] == "rmat":
        src, dst = rmat_edges(c["scale"], c["m"], 0.57, 0.19, 0.19, c["gseed"])
        n = 1 << c["scale"]
    else:
        raise KeyError(c["model"])
    m = src.shape[0]
    lseed = c["lseed"]
    if c["vdist"] == "zipf":
        vl = labels_zipf(n, c["nvl"], 1.1, lseed)
    else:
        vl = labels_uniform(n, c["nvl"], lseed)
    if c["edist"] == "zipf":
        el = labels_zipf(m, c["nel"], 1.1, lseed + 1)
    else:
        el = labels_uniform(m, c["nel"], lseed + 1)
    return Graph(n, vl, src, dst, el, name)


def config_query(g: Graph, name: str, index: int, attempt: int = 0, maker: QueryMaker | None = None) -> Query:
    c = CONFIGS[name]
    k, mode = query_spec(c["qseed"], index, c["kmin"], c["kmax"], c["modes"])
    mk = maker or QueryMaker(g)
    return mk.make(k, mode, query_seed(c["qseed"], index, attempt))


# ------------------------------------------------------- small named graphs
def complete_graph(n: int, vl: int = 0, el: int = 0) -> Graph:
    e = [(a, b) for a in range(n) for b in range(a + 1, n)]
    return make_graph(n, [vl] * n, e, [el] * len(e), "K%d" % n)


def cycle_graph(n: int) -> Graph:
    e = [(i, (i + 1) % n) for i in range(n)]
    return make_graph(n, [0] * n, e, [0] * n, "C%d" % n)


def path_query(k: int) -> Query:
    return make_query([0] * k, [(i, i + 1) for i in range(k - 1)], [0] * (k - 1), "path")


def cycle_query(k: int) -> Query:
    return make_query([0] * k, [(i, (i + 1) % k) for i in range(k)], [0] * k, "cycle")


def clique_query(k: int) -> Query:
    e = [(a, b) for a in range(k) for b in range(a + 1, k)]
    return make_query([0] * k, e, [0] * len(e), "clique")


def star_graph(n: int, center_label: int = 0, leaf_label: int = 0) -> Graph:
    """Star with centre 0 and leaves 1..n-1."""
    e = [(0, i) for i in range(1, n)]
    return make_graph(n, [center_label] + [leaf_label] * (n - 1), e, [0] * (n - 1), "S%d" % n)


def star_query(k: int, center_label: int = 0, leaf_label: int = 0) -> Query:
    e = [(0, i) for i in range(1, k)]
    return make_query([center_label] + [leaf_label] * (k - 1), e, [0] * (k - 1), "star")


def complete_bipartite(a: int, b: int, la: int = 0, lb: int = 1) -> Graph:
    e = [(i, a + j) for i in range(a) for j in range(b)]
    return make_graph(a + b, [la] * a + [lb] * b, e, [0] * len(e), "K%d,%d" % (a, b))


def random_small_graph(n: int, p: float, nvl: int, nel: int, seed: int) -> Graph:
    r = np.random.default_rng(seed)
    e = [(a, b) for a in range(n) for b in range(a + 1, n) if r.random() < p]
    return make_graph(n, r.integers(0, nvl, n), e, r.integers(0, nel, len(e)), "rand%d" % n)


def random_connected_query(k: int, extra: int, nvl: int, nel: int, seed: int) -> Query:
    """A random spanning tree on k vertices plus up to `extra` more edges."""
    r = np.random.default_rng(seed)
    edges = set()
    for v in range(1, k):
        u = int(r.integers(0, v))
        edges.add((u, v))
    for _ in range(extra):
        a, b = sorted(int(x) for x in r.integers(0, k, 2))
        if a != b:
            edges.add((a, b))
    edges = sorted(edges)
    return make_query(r.integers(0, nvl, k), edges, r.integers(0, nel, len(edges)), "random")


def paper_example():
    """A data graph and query consistent with every number the paper prints
    for its running example (Sec. III-B, Sec. IV, Sec. V, Example Fig. 1).

    Vertex labels: v0 is A(0); v1..v100 are B(1); v101..v201 are C(2).
    Edges with label a(0): (v0,vj) j=1..100; (v100,v200); (v100,v201);
    (vj, v100+j) for j=2..99.  Edges with label b(1): (v0,v201), (v1,v101).
    Query: u0:A, u1:B, u2:C, u3:C; edges u0u1:a, u0u2:b, u1u2:a, u1u3:a.
    """
    A, B, C = 0, 1, 2
    a, b = 0, 1
    vl = [A] + [B] * 100 + [C] * 101
    edges, el = [], []
    for j in range(1, 101):
        edges.append((0, j)); el.append(a)
    edges.append((100, 200)); el.append(a)
    edges.append((100, 201)); el.append(a)
    for j in range(2, 100):
        edges.append((j, 100 + j)); el.append(a)
    edges.append((0, 201)); el.append(b)
    edges.append((1, 101)); el.append(b)
    g = make_graph(202, vl, edges, el, "paper_example")
    q = make_query([A, B, C, C], [(0, 1), (0, 2), (1, 2), (1, 3)], [a, b, a, a], "paper_example")
    return g, q


# ------------------------------------------------------- multi-labelled inputs
# Sec. VII-B: a vertex may carry several labels, and a vertex pair several
# edge labels (given as one edge entry per label).  Label sets are stored as
# offsets into one label array.
@dataclass
class MGraph:
    n: int
    voff: np.ndarray   # uint64[n+1]
    vlab: np.ndarray   # uint32[voff[n]]
    src: np.ndarray    # uint32[m], one entry per (pair, label)
    dst: np.ndarray
    elabel: np.ndarray
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    def labels(self, v: int) -> list:
        return self.vlab[self.voff[v]:self.voff[v + 1]].tolist()


@dataclass
class MQuery:
    k: int
    qoff: np.ndarray   # uint32[k+1]
    qlab: np.ndarray   # uint32[qoff[k]]
    src: np.ndarray    # uint32, one entry per (pair, label)
    dst: np.ndarray
    elabel: np.ndarray
    mode: str = ""

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    def labels(self, u: int) -> list:
        return self.qlab[self.qoff[u]:self.qoff[u + 1]].tolist()


def make_mgraph(n, label_sets, edges, name="") -> MGraph:
    """label_sets[v]: labels of v; edges: (a, b, label) triples."""
    off = np.zeros(n + 1, np.uint64)
    off[1:] = np.cumsum([len(s) for s in label_sets])
    lab = _u32([x for s in label_sets for x in s])
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 3)
    return MGraph(int(n), off, lab, _u32(e[:, 0]), _u32(e[:, 1]), _u32(e[:, 2]), name)


def make_mquery(label_sets, edges, mode="manual") -> MQuery:
    k = len(label_sets)
    off = np.zeros(k + 1, np.uint32)
    off[1:] = np.cumsum([len(s) for s in label_sets])
    lab = _u32([x for s in label_sets for x in s])
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 3)
    return MQuery(k, off, lab, _u32(e[:, 0]), _u32(e[:, 1]), _u32(e[:, 2]), mode)


def mgraph_from_single(g: Graph) -> MGraph:
    """The same graph with one label per vertex and per pair."""
    return MGraph(g.n, np.arange(g.n + 1, dtype=np.uint64), g.vlabel.copy(), g.src.copy(), g.dst.copy(),
                  g.elabel.copy(), g.name)


def mquery_from_single(q: Query) -> MQuery:
    return MQuery(q.k, np.arange(q.k + 1, dtype=np.uint32), q.vlabel.copy(), q.src.copy(), q.dst.copy(),
                  q.elabel.copy(), q.mode)


def random_multi_graph(n: int, p: float, nvl: int, nel: int, max_vl: int, max_el: int, seed: int) -> MGraph:
    """Each vertex gets 1..max_vl distinct labels of nvl; each pair is an edge
    with probability p and then gets 1..max_el distinct labels of nel (at most
    nvl and nel of them)."""
    r = _stream(seed, 7)
    sets = [sorted(r.choice(nvl, size=min(nvl, int(r.integers(1, max_vl + 1))), replace=False).tolist())
            for _ in range(n)]
    a, b = np.triu_indices(n, 1)
    keep = r.random(a.shape[0]) < p
    edges = []
    for x, y in zip(a[keep].tolist(), b[keep].tolist()):
        for l in sorted(r.choice(nel, size=min(nel, int(r.integers(1, max_el + 1))), replace=False).tolist()):
            edges.append((x, y, l))
    return make_mgraph(n, sets, edges, "multi%d" % seed)


def multi_walk_query(g: MGraph, k: int, seed: int, dense: bool = False) -> MQuery:
    """A random walk over g until k distinct vertices are visited; each query
    vertex keeps a non-empty random subset of its data vertex's labels, each
    traversed pair (with dense, every pair of visited vertices joined in g)
    a non-empty random subset of the pair's labels.  The walk's own vertices
    are an embedding, so the result is never empty."""
    r = _stream(seed, 8)
    pairs = {}
    for x, y, l in zip(g.src.tolist(), g.dst.tolist(), g.elabel.tolist()):
        pairs.setdefault((min(x, y), max(x, y)), []).append(l)
    nbr = {}
    for (x, y) in pairs:
        nbr.setdefault(x, []).append(y)
        nbr.setdefault(y, []).append(x)
    starts = sorted(nbr)
    if not starts:
        raise RuntimeError("graph has no edges")
    for _ in range(100):
        v = starts[int(r.integers(0, len(starts)))]
        seen, walk = [v], set()
        for _ in range(100 * k):
            if len(seen) == k:
                break
            w = nbr[v][int(r.integers(0, len(nbr[v])))]
            walk.add((min(v, w), max(v, w)))
            if w not in seen:
                seen.append(w)
            v = w
        if len(seen) == k:
            break
    else:
        raise RuntimeError("no walk reached %d vertices" % k)
    idx = {v: i for i, v in enumerate(seen)}
    if dense:
        walk = {(x, y) for (x, y) in pairs if x in idx and y in idx}
    sets = []
    for v in seen:
        ls = g.labels(v)
        sets.append(sorted(r.choice(ls, size=int(r.integers(1, len(ls) + 1)), replace=False).tolist()))
    edges = []
    for (x, y) in sorted(walk):
        ls = pairs[(x, y)]
        for l in sorted(r.choice(ls, size=int(r.integers(1, len(ls) + 1)), replace=False).tolist()):
            edges.append((idx[x], idx[y], l))
    q = make_mquery(sets, edges, "dense" if dense else "walk")
    q.source = np.array(seen, np.uint32)
    return q
