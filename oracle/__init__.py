"""CPU ORACLE — test infrastructure, not part of the product.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import, call, link or execute anything in this package.  The
GPU library never routes through it, and it shares no code with the GPU
library: the two meet only on inputs made by ``workloads``.

Contents
  match.c   plain backtracking enumeration of all embeddings (Sec. II-A,
            Definitions 1-3) plus the order-independent result digest.
  multi.c   the same enumeration under multi-labels (Sec. VII-B): label sets
            on vertices, several labelled edges per vertex pair, containment
            instead of equality; written separately from match.c.
  spec.py   plain numpy/Python statements of the intermediate steps of the
            paper's method: vertex signatures and the signature filter
            (Sec. III-A), the PCSR layout (Sec. IV, Definition 4, Algorithm 1),
            the matching order (Algorithm 2, Algorithm 4's first-edge rule) and
            per-level join sizes (Algorithms 3-4).  Parity of the matching
            order is unpinned (it changes speed, never results).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "match.c")
_SRCS = [_SRC, os.path.join(_HERE, "multi.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

U32P = ctypes.POINTER(ctypes.c_uint32)
U64P = ctypes.POINTER(ctypes.c_uint64)

OR_OK, OR_INVALID, OR_NOMEM, OR_LIMIT = 0, 1, 2, 3


class OracleResultC(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("dsum", ctypes.c_uint64), ("dxor", ctypes.c_uint64),
                ("nodes", ctypes.c_uint64), ("tuples", ctypes.c_void_p), ("status", ctypes.c_int)]


def build(force: bool = False) -> str:
    """Compile match.c with gcc (host code only)."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fPIC", "-shared", "-pthread", "-o", tmp] + _SRCS)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_fnv1a64.argtypes = [ctypes.c_char_p, ctypes.c_uint64]
        lib.oracle_fnv1a64.restype = ctypes.c_uint64
        lib.oracle_fnv1a64_words.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        lib.oracle_fnv1a64_words.restype = ctypes.c_uint64
        lib.oracle_sm64_finalize.argtypes = [ctypes.c_uint64]
        lib.oracle_sm64_finalize.restype = ctypes.c_uint64
        lib.oracle_tuple_hash.argtypes = [U32P, ctypes.c_uint32]
        lib.oracle_tuple_hash.restype = ctypes.c_uint64
        lib.oracle_digest_rows.argtypes = [U32P, ctypes.c_uint64, ctypes.c_uint32, U64P]
        lib.oracle_digest_rows.restype = None
        lib.oracle_graph_build.argtypes = [ctypes.c_uint32, U32P, ctypes.c_uint64, U32P, U32P, U32P,
                                           ctypes.POINTER(ctypes.c_int)]
        lib.oracle_graph_build.restype = ctypes.c_void_p
        lib.oracle_graph_free.argtypes = [ctypes.c_void_p]
        lib.oracle_graph_free.restype = None
        lib.oracle_match.argtypes = [ctypes.c_void_p, ctypes.c_uint32, U32P, ctypes.c_uint32, U32P, U32P, U32P,
                                     ctypes.c_uint32, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                     ctypes.POINTER(OracleResultC)]
        lib.oracle_match.restype = ctypes.c_int
        lib.oracle_free.argtypes = [ctypes.c_void_p]
        lib.oracle_free.restype = None
        lib.oracle_mgraph_build.argtypes = [ctypes.c_uint32, U64P, U32P, ctypes.c_uint64, U32P, U32P, U32P,
                                            ctypes.POINTER(ctypes.c_int)]
        lib.oracle_mgraph_build.restype = ctypes.c_void_p
        lib.oracle_mgraph_free.argtypes = [ctypes.c_void_p]
        lib.oracle_mgraph_free.restype = None
        lib.oracle_mmatch.argtypes = [ctypes.c_void_p, ctypes.c_uint32, U32P, U32P, ctypes.c_uint32, U32P, U32P,
                                      U32P, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint64,
                                      ctypes.POINTER(OracleResultC)]
        lib.oracle_mmatch.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(U32P)


def fnv1a64(data: bytes) -> int:
    return int(_load().oracle_fnv1a64(data, len(data)))


def fnv1a64_words(words) -> int:
    """FNV-1a-64 with each 32-bit value as one symbol."""
    a = np.ascontiguousarray(words, dtype=np.uint32)
    return int(_load().oracle_fnv1a64_words(a.ctypes.data, a.shape[0]))


def splitmix64_finalize(z: int) -> int:
    return int(_load().oracle_sm64_finalize(ctypes.c_uint64(z & (2**64 - 1))))


def tuple_hash(t) -> int:
    a, p = _p(t)
    return int(_load().oracle_tuple_hash(p, a.shape[0]))


def digest_rows(rows: np.ndarray) -> tuple:
    """(sum, xor) digest of a row-major uint32 table (rows x k)."""
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    if rows.ndim != 2:
        raise ValueError("rows must be 2-D")
    out = (ctypes.c_uint64 * 2)()
    _load().oracle_digest_rows(rows.ctypes.data_as(U32P), rows.shape[0], rows.shape[1], out)
    return int(out[0]), int(out[1])


@dataclass
class MatchResult:
    status: int
    count: int
    digest: tuple
    nodes: int
    tuples: np.ndarray | None  # sorted, row-major (count x k), query-vertex order


class OracleGraph:
    """Sorted adjacency of a data graph, held by the C oracle."""

    def __init__(self, g):
        lib = _load()
        self.n = g.n
        self._keep = [_p(g.vlabel), _p(g.src), _p(g.dst), _p(g.elabel)]
        st = ctypes.c_int(0)
        self._h = lib.oracle_graph_build(g.n, self._keep[0][1], g.m, self._keep[1][1], self._keep[2][1],
                                         self._keep[3][1], ctypes.byref(st))
        self._keep = None
        if not self._h:
            raise ValueError("oracle rejected the data graph (status %d)" % st.value)

    def close(self):
        if getattr(self, "_h", None):
            _load().oracle_graph_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def match(self, q, threads: int = 1, tuples: bool = True, max_count: int = 0, max_nodes: int = 0,
              homomorphism: bool = False) -> MatchResult:
        """All embeddings of q (Definitions 1-3), or, with homomorphism, all
        label- and edge-preserving maps, injective or not (Sec. VII-A)."""
        lib = _load()
        ql, qlp = _p(q.vlabel)
        qs, qsp = _p(q.src)
        qd, qdp = _p(q.dst)
        qe, qep = _p(q.elabel)
        r = OracleResultC()
        lib.oracle_match(self._h, q.k, qlp, qs.shape[0], qsp, qdp, qep, threads, 1 if tuples else 0,
                         max_count, max_nodes, 1 if homomorphism else 0, ctypes.byref(r))
        t = None
        if r.tuples:
            if r.status == OR_OK:
                buf = (ctypes.c_uint32 * (r.count * q.k)).from_address(r.tuples)
                t = np.frombuffer(buf, dtype=np.uint32).reshape(r.count, q.k).copy()
            lib.oracle_free(r.tuples)
        elif tuples and r.status == OR_OK:
            t = np.zeros((0, q.k), np.uint32)
        return MatchResult(int(r.status), int(r.count), (int(r.dsum), int(r.dxor)), int(r.nodes), t)


def match(g, q, threads: int = 1, tuples: bool = True, **kw) -> MatchResult:
    og = OracleGraph(g)
    try:
        return og.match(q, threads=threads, tuples=tuples, **kw)
    finally:
        og.close()


class OracleMultiGraph:
    """A multi-labelled data graph (Sec. VII-B) held by the C oracle: vertex
    label sets vlab[voff[v]:voff[v+1]], one edge entry per label of a pair."""

    def __init__(self, g):
        lib = _load()
        self.n = g.n
        voff = np.ascontiguousarray(g.voff, dtype=np.uint64)
        keep = [_p(g.vlab), _p(g.src), _p(g.dst), _p(g.elabel)]
        st = ctypes.c_int(0)
        self._h = lib.oracle_mgraph_build(g.n, voff.ctypes.data_as(U64P), keep[0][1], g.m, keep[1][1], keep[2][1],
                                          keep[3][1], ctypes.byref(st))
        if not self._h:
            raise ValueError("oracle rejected the multi-labelled graph (status %d)" % st.value)

    def close(self):
        if getattr(self, "_h", None):
            _load().oracle_mgraph_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def match(self, q, threads: int = 1, tuples: bool = True, max_count: int = 0) -> MatchResult:
        """All embeddings of the multi-labelled query q: injective, each query
        vertex's labels contained in its image's, each query pair's edge
        labels contained in its image pair's."""
        lib = _load()
        qo, qop = _p(q.qoff)
        ql, qlp = _p(q.qlab)
        qs, qsp = _p(q.src)
        qd, qdp = _p(q.dst)
        qe, qep = _p(q.elabel)
        r = OracleResultC()
        lib.oracle_mmatch(self._h, q.k, qop, qlp, qs.shape[0], qsp, qdp, qep, threads, 1 if tuples else 0,
                          max_count, ctypes.byref(r))
        t = None
        if r.tuples:
            if r.status == OR_OK:
                buf = (ctypes.c_uint32 * (r.count * q.k)).from_address(r.tuples)
                t = np.frombuffer(buf, dtype=np.uint32).reshape(r.count, q.k).copy()
            lib.oracle_free(r.tuples)
        elif tuples and r.status == OR_OK:
            t = np.zeros((0, q.k), np.uint32)
        return MatchResult(int(r.status), int(r.count), (int(r.dsum), int(r.dxor)), 0, t)


def match_multi(g, q, threads: int = 1, tuples: bool = True, **kw) -> MatchResult:
    og = OracleMultiGraph(g)
    try:
        return og.match(q, threads=threads, tuples=tuples, **kw)
    finally:
        og.close()
