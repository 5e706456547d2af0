"""Plain statements of the intermediate steps of the paper's method.

CPU ORACLE — test infrastructure only (see the package docstring).  Every
function here is written for a reader to check against the paper by eye; none
is fast.  Readings of passages the paper leaves open are stated where they are
used.

Sections cited are those of the paper (GSI, arXiv 1906.03420).
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np

# --------------------------------------------------------------------------
# Vertex signatures (Sec. III-A, "Filtering Phase"; parameters N=512, K=32 as
# set in Sec. VIII-B; the vertex label is stored directly in the first K bits,
# Sec. VII-B).
#
# Reading: the K=32 label bits hold the label itself and the filter tests them
# for equality.  The remaining N-K = 480 bits are 240 two-bit groups.  Each
# (edge, neighbour) pair (e, w) of v forms the 64-bit key
#     key = L_E(e) * 2^32 + L_V(w)
# which is sent to group  g = floor(((key * A) mod 2^64 >> 32) * 240 / 2^32)
# with A = 0x9E3779B97F4A7C15 = floor(2^64 / golden ratio) (Knuth's
# multiplicative hashing; the final multiply-shift is Lemire's range
# reduction).  A group holds 00 when no pair maps to it, 01 when exactly one
# pair does and 11 when more than one does.  Group g occupies bits
# 2*(g mod 16) and 2*(g mod 16)+1 of 32-bit word 1 + g div 16; the low bit of
# the two is the "01" bit.
SIG_WORDS = 16
SIG_GROUPS = 240
KNUTH64 = 0x9E3779B97F4A7C15


def signature_group(edge_label, neighbour_label):
    """Group index in [0, 240) of the key (edge label, neighbour label)."""
    key = (np.asarray(edge_label, np.uint64) << np.uint64(32)) | np.asarray(neighbour_label, np.uint64)
    with np.errstate(over="ignore"):
        hi = (key * np.uint64(KNUTH64)) >> np.uint64(32)
    return ((hi * np.uint64(SIG_GROUPS)) >> np.uint64(32)).astype(np.int64)


def _encode(n, labels, owner, edge_label, nb_label):
    """Signature table (SIG_WORDS x n, column-first) for pairs (owner, e, w)."""
    sig = np.zeros((SIG_WORDS, n), np.uint32)
    sig[0] = labels
    if len(owner):
        g = signature_group(edge_label, nb_label)
        flat = np.asarray(owner, np.int64) * SIG_GROUPS + g
        cell, cnt = np.unique(flat, return_counts=True)
        v = cell // SIG_GROUPS
        gg = cell % SIG_GROUPS
        code = np.where(cnt == 1, 1, 3).astype(np.uint64)
        word = 1 + gg // 16
        bits = (code << (2 * (gg % 16)).astype(np.uint64)).astype(np.uint32)
        np.bitwise_or.at(sig, (word, v), bits)
    return sig


def signature_table(g) -> np.ndarray:
    """S(v) for every data vertex: uint32[16, |V|], column-first as the
    paper lays the table out (one row of the array = one 32-bit column of
    every signature)."""
    owner = np.concatenate([g.src, g.dst]).astype(np.int64)
    other = np.concatenate([g.dst, g.src]).astype(np.int64)
    el = np.concatenate([g.elabel, g.elabel])
    return _encode(g.n, g.vlabel, owner, el, g.vlabel[other])


def query_signatures(q) -> np.ndarray:
    """S(u) for every query vertex, same encoding: uint32[16, k]."""
    owner = np.concatenate([q.src, q.dst]).astype(np.int64)
    other = np.concatenate([q.dst, q.src]).astype(np.int64)
    el = np.concatenate([q.elabel, q.elabel])
    return _encode(q.k, q.vlabel, owner, el, q.vlabel[other] if len(other) else np.zeros(0, np.uint32))


def filter_candidates(sig: np.ndarray, qsig: np.ndarray) -> list:
    """C(u) for every query vertex (Sec. III-A): v is kept iff the label
    words are equal and S(v) & S(u) == S(u) on the other words.  Returns one
    sorted uint32 array per query vertex."""
    out = []
    for u in range(qsig.shape[1]):
        s = qsig[:, u:u + 1]
        ok = sig[0] == s[0, 0]
        ok &= np.all((sig[1:] & s[1:]) == s[1:], axis=0)
        out.append(np.nonzero(ok)[0].astype(np.uint32))
    return out


def filter_bitsets(cands: list, n: int) -> np.ndarray:
    """Candidate sets as bitsets: uint64[k, ceil(n/64)], bit v%64 of word v//64."""
    words = (n + 63) // 64
    out = np.zeros((len(cands), words), np.uint64)
    for u, c in enumerate(cands):
        c = np.asarray(c, np.uint64)
        np.bitwise_or.at(out[u], (c // np.uint64(64)).astype(np.int64), np.uint64(1) << (c % np.uint64(64)))
    return out


# --------------------------------------------------------------------------
# PCSR (Sec. IV, Definition 4, Algorithm 1; GPN = 16 as chosen in Sec. IV).
#
# Readings (the paper fixes neither the hash f nor where overflow keys go):
#  * P(G,l) keeps every l-labelled edge in both directions, so ci of label l
#    holds 2|E_l| entries, each vertex's neighbours ascending.
#  * |V(D)| groups of 16 (vid, offset) pairs; pairs 0..14 hold keys, pair 15
#    is (GID, END).  Home group of v: f(v) = ((v * 0x9E3779B1) mod 2^32) * H
#    >> 32, with H = |V(D)| (a test-only mode lowers H to force chains).
#  * A group's home keys are sorted ascending; the first 15 stay home.  The
#    rest go, 15 per group, to empty groups (no home key) taken in ascending
#    index order and handed to overflowing groups in ascending home index
#    order, each chain linked by GID; GID = 0xFFFFFFFF (-1) ends a chain.
#  * ci is laid out in group order, then slot order (Algorithm 1, last loop);
#    an unused slot holds (0xFFFFFFFF, END), so the list of the key in slot s
#    ends at the offset of pair s+1.
PCSR_GPN = 16
PCSR_KEYS = PCSR_GPN - 1
KNUTH32 = 0x9E3779B1
NONE = 0xFFFFFFFF


def pcsr_home(v, H: int):
    x = (np.asarray(v, np.uint64) * np.uint64(KNUTH32)) & np.uint64(0xFFFFFFFF)
    return ((x * np.uint64(H)) >> np.uint64(32)).astype(np.int64)


def neighbour_lists(g) -> dict:
    """{label: {v: sorted neighbour array}} — N(v,l) for every pair present."""
    out = defaultdict(dict)
    owner = np.concatenate([g.src, g.dst])
    other = np.concatenate([g.dst, g.src])
    el = np.concatenate([g.elabel, g.elabel])
    order = np.lexsort((other, owner, el))
    owner, other, el = owner[order], other[order], el[order]
    if len(el) == 0:
        return {}
    cut = np.nonzero((np.diff(el) != 0) | (np.diff(owner) != 0))[0] + 1
    starts = np.concatenate([[0], cut])
    ends = np.concatenate([cut, [len(el)]])
    for a, b in zip(starts, ends):
        out[int(el[a])][int(owner[a])] = other[a:b].copy()
    return dict(out)


def pcsr_label(nbrs: dict, degenerate: bool = False):
    """PCSR(G,l) = (gl, ci) for one label from {v: sorted N(v,l)}.
    gl: uint32[G, 32] (pairs interleaved vid, off); ci: uint32[...]."""
    keys = sorted(nbrs)
    G = len(keys)
    if G == 0:
        return np.zeros((0, 2 * PCSR_GPN), np.uint32), np.zeros(0, np.uint32)
    H = (G + PCSR_GPN - 1) // PCSR_GPN if degenerate else G
    home = defaultdict(list)
    for v, h in zip(keys, pcsr_home(np.array(keys, np.uint64), H)):
        home[int(h)].append(v)          # keys arrive ascending, so lists stay sorted
    empties = [i for i in range(G) if not home.get(i)]
    members = [[] for _ in range(G)]    # keys stored in each group
    gid = [NONE] * G
    take = 0
    for h in range(G):
        lst = home.get(h, [])
        if not lst:
            continue                    # an empty group may already hold overflow keys
        members[h] = lst[:PCSR_KEYS]
        prev = h
        for s in range(PCSR_KEYS, len(lst), PCSR_KEYS):
            if take >= len(empties):
                raise AssertionError("Claim 1 violated: not enough empty groups")
            e = empties[take]
            take += 1
            members[e] = lst[s:s + PCSR_KEYS]
            gid[prev] = e
            prev = e
    gl = np.zeros((G, 2 * PCSR_GPN), np.uint32)
    ci = []
    pos = 0
    for i in range(G):
        for s, v in enumerate(members[i]):
            gl[i, 2 * s] = v
            gl[i, 2 * s + 1] = pos
            ci.extend(int(x) for x in nbrs[v])
            pos += len(nbrs[v])
        for s in range(len(members[i]), PCSR_KEYS):
            gl[i, 2 * s] = NONE
            gl[i, 2 * s + 1] = pos
        gl[i, 2 * PCSR_KEYS] = gid[i]
        gl[i, 2 * PCSR_KEYS + 1] = pos
    return gl, np.array(ci, np.uint32)


def pcsr(g, degenerate: bool = False) -> dict:
    """{label: (gl, ci)} for every edge label present in G."""
    return {l: pcsr_label(nb, degenerate) for l, nb in neighbour_lists(g).items()}


def pcsr_locate(gl: np.ndarray, ci: np.ndarray, v: int, degenerate: bool = False):
    """N(v,l) read back through the structure (Sec. IV, lookup steps 1-4):
    hash to a group, probe its pairs, follow GID until found or -1."""
    G = gl.shape[0]
    if G == 0:
        return np.zeros(0, np.uint32), 0
    H = (G + PCSR_GPN - 1) // PCSR_GPN if degenerate else G
    grp = int(pcsr_home(np.array([v], np.uint64), H)[0])
    reads = 0
    while True:
        reads += 1
        row = gl[grp]
        for s in range(PCSR_KEYS):
            if int(row[2 * s]) == v:
                return ci[int(row[2 * s + 1]):int(row[2 * s + 3])], reads
        nxt = int(row[2 * PCSR_KEYS])
        if nxt == NONE:
            return np.zeros(0, np.uint32), reads
        grp = nxt


# --------------------------------------------------------------------------
# Matching order (Algorithm 2) and first edge (Algorithm 4).
#
# Readings: freq(l) = |E_l| / |E| (a ratio, so multiplying a score by it
# favours vertices with more and rarer linking edges); argmin ties go to the
# smallest query vertex id; among linking edges of equal minimum frequency
# the first edge is the one whose matched endpoint was placed earliest.
# Parity unpinned: the order changes work, never the result set.
def label_frequency(g) -> dict:
    m = max(1, g.m)
    labs, cnt = np.unique(g.elabel, return_counts=True)
    return {int(l): int(c) / m for l, c in zip(labs, cnt)}


def plan(q, cand_counts, freq: dict):
    """Returns (order, first_edge_src) where first_edge_src[j] (j >= 1) is
    the matched query vertex at the other end of the first edge e0 used to
    join order[j]."""
    k = q.k
    adj = defaultdict(dict)
    for a, b, l in zip(q.src.tolist(), q.dst.tolist(), q.elabel.tolist()):
        adj[a][b] = l
        adj[b][a] = l
    deg = [len(adj[u]) for u in range(k)]
    if k == 1:
        return [0], [None]
    score = [float(cand_counts[u]) / deg[u] for u in range(k)]
    placed = []
    e0src = [None]
    uc = min(range(k), key=lambda u: (score[u], u))
    placed.append(uc)
    for w, l in adj[uc].items():
        score[w] *= freq.get(l, 0.0)
    while len(placed) < k:
        frontier = [u for u in range(k) if u not in placed and any(w in placed for w in adj[u])]
        u = min(frontier, key=lambda x: (score[x], x))
        links = [w for w in placed if w in adj[u]]
        e0 = min(links, key=lambda w: (freq.get(adj[u][w], 0.0), placed.index(w)))
        e0src.append(e0)
        placed.append(u)
        for w, l in adj[u].items():
            score[w] *= freq.get(l, 0.0)
    return placed, e0src


# --------------------------------------------------------------------------
# Vertex-at-a-time join (Algorithm 3 with Algorithm 4's pre-allocation),
# executed row by row as written: for each row m_i the buffer is
#   buf_i = ((N(v'_i, l0) minus m_i) intersect C(u)) intersect every other N(.,l)
# and M' gets (m_i, z) for each z in buf_i.
def join_levels(g, q, cands: list, order: list, e0src: list, nbrs: dict | None = None, per_row: bool = False):
    """Returns (M, levels): the final table (rows in matching-order columns,
    produced in row order then buffer order) and per level j >= 1 a dict
    with R (rows of M), GBA (|GBA| = F[|M|]), F (the offsets of Algorithm 4)
    and S (rows of M').  With per_row, each row's buffer starts from its
    shortest linking list instead of e0's (e0's on ties): the buffer, being
    the intersection of all of them, is the same; F and |GBA| shrink."""
    nbrs = nbrs if nbrs is not None else neighbour_lists(g)
    adj = defaultdict(dict)
    for a, b, l in zip(q.src.tolist(), q.dst.tolist(), q.elabel.tolist()):
        adj[a][b] = l
        adj[b][a] = l
    empty = np.zeros(0, np.uint32)

    def N(v, l):
        return nbrs.get(l, {}).get(int(v), empty)

    M = [(int(v),) for v in cands[order[0]]]
    levels = []
    for j in range(1, len(order)):
        u = order[j]
        col = {w: order.index(w) for w in order[:j]}
        links = [w for w in order[:j] if w in adj[u]]
        w0 = e0src[j]
        l0 = adj[u][w0]
        Cu = set(int(x) for x in cands[u])
        F = [0]
        new = []
        for row in M:
            wb = w0
            base = N(row[col[w0]], l0)
            if per_row:
                for w in links:
                    if w != w0 and len(N(row[col[w]], adj[u][w])) < len(base):
                        wb, base = w, N(row[col[w]], adj[u][w])
            F.append(F[-1] + len(base))
            buf = [int(x) for x in base if int(x) not in row]
            buf = [x for x in buf if x in Cu]
            for w in links:
                if w == wb:
                    continue
                other = set(int(x) for x in N(row[col[w]], adj[u][w]))
                buf = [x for x in buf if x in other]
            new.extend(row + (x,) for x in buf)
        levels.append(dict(R=len(M), GBA=F[-1], F=F, S=len(new)))
        M = new
    return M, levels


def to_query_order(M: list, order: list) -> np.ndarray:
    """Rows in matching-order columns -> uint32 rows in query-vertex order."""
    k = len(order)
    out = np.zeros((len(M), k), np.uint32)
    for c, u in enumerate(order):
        out[:, u] = [r[c] for r in M]
    return out
