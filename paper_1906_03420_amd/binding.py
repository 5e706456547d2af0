"""ctypes binding of libgsi.so: the same entry points as include/gsi.h.

Argument marshalling only — every step of the matching path runs in the HIP
library.  There is no CPU fallback: if libgsi.so is missing or the GPU call
fails, the call raises.

PyTorch provides device memory (the arena tensor) and the stream; see
``Context``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsi.so")

GSI_OK, GSI_E_INVALID, GSI_E_NOMEM, GSI_E_DEVICE, GSI_E_CAPACITY, GSI_E_BUSY, GSI_E_INTERNAL = range(7)
GSI_MAX_K = 32
GSI_SIG_WORDS = 16
GSI_CTX_PROFILE = 0x1
GSI_GRAPH_TEST_FEW_HOME_GROUPS = 0x1
GSI_COUNT_ONLY = 0x1
GSI_FILTER_LABEL_ONLY = 0x2
GSI_NO_FUSED = 0x4
GSI_BATCH_LEVELS_ONLY = 0x8
GSI_NO_CHUNKS = 0x10
GSI_LEVEL_FIRST_EDGE = 0x20
GSI_NO_LIST_FILTER = 0x8000
GSI_SINGLE_PASS = 0x20000
GSI_HOMOMORPHISM = 0x40
GSI_ABL_CR = 0x100
GSI_ABL_TWO_STEP = 0x200
GSI_ABL_NO_STAGING = 0x400
GSI_ABL_NAIVE_SETOPS = 0x800
GSI_ABL_ROW_PER_WAVE = 0x1000
GSI_ABL_FOUR_LAYER = 0x2000
GSI_ABL_DUP_REMOVAL = 0x4000
GSI_GRAPH_KEEP_CR = 0x2
GSI_MAX_EDGE_LABELS = 65536
GSI_PCSR_GPN = 16
GSI_PATH_EMPTY, GSI_PATH_TIER1, GSI_PATH_TIER2, GSI_PATH_SINGLE, GSI_PATH_LEVELS, GSI_PATH_SOLO = range(6)
GSI_SERVER_NO_SOLO = 0x2
GSI_NOALLOC_SCRATCH_BYTES = 128 << 20

STATUS_NAMES = {0: "GSI_OK", 1: "GSI_E_INVALID", 2: "GSI_E_NOMEM", 3: "GSI_E_DEVICE", 4: "GSI_E_CAPACITY",
                5: "GSI_E_BUSY", 6: "GSI_E_INTERNAL"}

U32P = ctypes.POINTER(ctypes.c_uint32)
U64P = ctypes.POINTER(ctypes.c_uint64)
VP = ctypes.c_void_p


class GsiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class gsi_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("hip_stream", VP), ("arena_ptr", VP), ("arena_bytes", ctypes.c_uint64),
                ("flags", ctypes.c_uint32)]


class gsi_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_double)]


class gsi_graph_info(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_uint32), ("n_edges", ctypes.c_uint64), ("n_edge_labels", ctypes.c_uint32),
                ("total_groups", ctypes.c_uint64), ("max_chain", ctypes.c_uint32), ("device_bytes", ctypes.c_uint64),
                ("build_ms", ctypes.c_double)]


class gsi_query_options(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("order", U32P), ("first_edge", U32P), ("max_rows", ctypes.c_uint64),
                ("fused_max_rows", ctypes.c_uint32), ("fused_max_slots", ctypes.c_uint32),
                ("chunk_rows", ctypes.c_uint32), ("chunk_min_rows", ctypes.c_uint32)]


class gsi_stats(ctypes.Structure):
    K = GSI_MAX_K
    _fields_ = [("k", ctypes.c_uint32), ("levels", ctypes.c_uint32), ("order", ctypes.c_uint32 * K),
                ("first_edge", ctypes.c_uint32 * K), ("n_link", ctypes.c_uint32 * K), ("cand", ctypes.c_uint32 * K),
                ("rows", ctypes.c_uint64 * K), ("gba", ctypes.c_uint64 * K), ("other_elems", ctypes.c_uint64 * K),
                ("survivors", ctypes.c_uint64 * K), ("chunks", ctypes.c_uint32), ("chunks_left", ctypes.c_uint32),
                ("filter_ms", ctypes.c_double), ("join_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("filtered_levels", ctypes.c_uint32)]


class gsi_query_desc(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("vertex_labels", U32P), ("n_edges", ctypes.c_uint32), ("src", U32P),
                ("dst", U32P), ("edge_labels", U32P)]


class gsi_batch_schedule(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_uint32), ("grid_scale", ctypes.c_uint32), ("engine_tiles", ctypes.c_uint32)]


class gsi_batch_options(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("schedule", gsi_batch_schedule)]


class gsi_batch_info(ctypes.Structure):
    _fields_ = [("queries", ctypes.c_uint32), ("empty", ctypes.c_uint32), ("tier1", ctypes.c_uint32),
                ("tier2", ctypes.c_uint32), ("per_level", ctypes.c_uint32), ("schedule", gsi_batch_schedule),
                ("filter_ms", ctypes.c_double), ("tier1_ms", ctypes.c_double), ("tier2_ms", ctypes.c_double),
                ("per_level_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]


class gsi_server_options(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32), ("max_admit", ctypes.c_uint32),
                ("solo_queue", ctypes.c_uint32), ("table_budget", ctypes.c_uint64),
                ("schedule", gsi_batch_schedule)]


class gsi_server_answer(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("k", ctypes.c_uint32), ("count", ctypes.c_uint64),
                ("digest", ctypes.c_uint64 * 2), ("path", ctypes.c_uint32), ("levels", ctypes.c_uint32),
                ("predicted_bytes", ctypes.c_uint64), ("peak_table_bytes", ctypes.c_uint64),
                ("submit_ms", ctypes.c_double), ("admit_ms", ctypes.c_double), ("done_ms", ctypes.c_double)]


class gsi_server_info(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64), ("answered", ctypes.c_uint64),
                ("released", ctypes.c_uint64), ("waiting", ctypes.c_uint32), ("in_flight", ctypes.c_uint32),
                ("steps", ctypes.c_uint64), ("level_steps", ctypes.c_uint64), ("admit_rounds", ctypes.c_uint64),
                ("predicted_in_flight", ctypes.c_uint64), ("peak_predicted", ctypes.c_uint64),
                ("table_budget", ctypes.c_uint64), ("admit_ms", ctypes.c_double), ("level_ms", ctypes.c_double), ("solo", ctypes.c_uint64)]


PATH_NAMES = {GSI_PATH_EMPTY: "empty", GSI_PATH_TIER1: "tier1", GSI_PATH_TIER2: "tier2",
              GSI_PATH_SINGLE: "single", GSI_PATH_LEVELS: "levels", GSI_PATH_SOLO: "solo"}

# name -> (restype, argtypes) for every exported function of gsi.h
SIGNATURES = {
    "gsi_last_error": (ctypes.c_char_p, []),
    "gsi_version": (ctypes.c_char_p, []),
    "gsi_ctx_create": (ctypes.c_int, [ctypes.POINTER(gsi_options), ctypes.POINTER(VP)]),
    "gsi_ctx_destroy": (ctypes.c_int, [VP]),
    "gsi_ctx_memory": (ctypes.c_int, [VP, U64P, U64P]),
    "gsi_ctx_kernel_stats": (ctypes.c_int, [VP, ctypes.POINTER(gsi_kernel_stat), ctypes.c_uint32, U32P]),
    "gsi_ctx_kernel_stats_reset": (ctypes.c_int, [VP]),
    "gsi_graph_bytes_needed": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint64, U64P]),
    "gsi_graph_load": (ctypes.c_int, [VP, ctypes.c_uint32, U32P, ctypes.c_uint64, U32P, U32P, U32P, ctypes.c_uint32,
                                      ctypes.POINTER(VP)]),
    "gsi_graph_load_device": (ctypes.c_int, [VP, ctypes.c_uint32, VP, ctypes.c_uint64, VP, VP, VP, ctypes.c_uint32,
                                             ctypes.POINTER(VP)]),
    "gsi_graph_free": (ctypes.c_int, [VP]),
    "gsi_graph_load_multi": (ctypes.c_int, [VP, ctypes.c_uint32, U64P, U32P, ctypes.c_uint64, U32P, U32P, U32P,
                                            ctypes.c_uint32, ctypes.POINTER(VP)]),
    "gsi_query_run_multi": (ctypes.c_int, [VP, ctypes.c_uint32, U32P, U32P, ctypes.c_uint32, U32P, U32P, U32P,
                                           ctypes.POINTER(gsi_query_options), ctypes.POINTER(VP)]),
    "gsi_graph_get_info": (ctypes.c_int, [VP, ctypes.POINTER(gsi_graph_info)]),
    "gsi_graph_label_edges": (ctypes.c_int, [VP, ctypes.c_uint32, U64P]),
    "gsi_graph_copy_signatures": (ctypes.c_int, [VP, U32P, ctypes.c_uint64]),
    "gsi_graph_copy_pcsr": (ctypes.c_int, [VP, ctypes.c_uint32, U32P, ctypes.c_uint64, U32P, ctypes.c_uint64, U64P,
                                           U64P]),
    "gsi_query_run": (ctypes.c_int, [VP, ctypes.c_uint32, U32P, ctypes.c_uint32, U32P, U32P, U32P,
                                     ctypes.POINTER(gsi_query_options), ctypes.POINTER(VP)]),
    "gsi_query_filter": (ctypes.c_int, [VP, ctypes.c_uint32, U32P, ctypes.c_uint32, U32P, U32P, U32P, U64P,
                                        ctypes.c_uint64, U32P]),
    "gsi_query_run_noalloc": (ctypes.c_int, [VP, ctypes.c_uint32, U32P, ctypes.c_uint32, U32P, U32P, U32P,
                                             ctypes.c_uint32, VP, ctypes.c_uint64, U64P, U64P]),
    "gsi_result_count": (ctypes.c_int, [VP, U64P]),
    "gsi_result_rows": (ctypes.c_int, [VP, U32P, ctypes.c_uint64]),
    "gsi_result_device_rows": (ctypes.c_int, [VP, ctypes.POINTER(VP)]),
    "gsi_result_digest": (ctypes.c_int, [VP, U64P]),
    "gsi_result_stats": (ctypes.c_int, [VP, ctypes.POINTER(gsi_stats)]),
    "gsi_result_free": (ctypes.c_int, [VP]),
    "gsi_batch_run": (ctypes.c_int, [VP, ctypes.c_uint32, ctypes.POINTER(gsi_query_desc),
                                     ctypes.POINTER(gsi_batch_options), ctypes.POINTER(VP)]),
    "gsi_batch_count": (ctypes.c_int, [VP, ctypes.c_uint32, U64P]),
    "gsi_batch_digest": (ctypes.c_int, [VP, ctypes.c_uint32, U64P]),
    "gsi_batch_rows": (ctypes.c_int, [VP, ctypes.c_uint32, U32P, ctypes.c_uint64]),
    "gsi_batch_results": (ctypes.c_int, [VP, U64P, U64P]),
    "gsi_batch_get_info": (ctypes.c_int, [VP, ctypes.POINTER(gsi_batch_info)]),
    "gsi_batch_free": (ctypes.c_int, [VP]),
    "gsi_batch_tune": (ctypes.c_int, [VP, ctypes.c_uint32, ctypes.POINTER(gsi_query_desc), ctypes.c_uint32,
                                      ctypes.POINTER(gsi_batch_schedule), ctypes.POINTER(ctypes.c_double)]),
    "gsi_server_create": (ctypes.c_int, [VP, ctypes.POINTER(gsi_server_options), ctypes.POINTER(VP)]),
    "gsi_server_submit": (ctypes.c_int, [VP, ctypes.POINTER(gsi_query_desc), U64P]),
    "gsi_server_step": (ctypes.c_int, [VP, U32P]),
    "gsi_server_poll": (ctypes.c_int, [VP, U64P, ctypes.c_uint32, U32P]),
    "gsi_server_answer_get": (ctypes.c_int, [VP, ctypes.c_uint64, ctypes.POINTER(gsi_server_answer)]),
    "gsi_server_rows": (ctypes.c_int, [VP, ctypes.c_uint64, U32P, ctypes.c_uint64]),
    "gsi_server_release": (ctypes.c_int, [VP, ctypes.c_uint64]),
    "gsi_server_get_info": (ctypes.c_int, [VP, ctypes.POINTER(gsi_server_info)]),
    "gsi_server_free": (ctypes.c_int, [VP]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libgsi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError("libgsi.so is not built (run __graft_entry__.build()); there is no CPU fallback")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(st: int):
    if st != GSI_OK:
        raise GsiError(st, gsi_last_error())


def _u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(U32P)


# --------------------------------------------------------------- raw calls
def sort_rows(rows: np.ndarray) -> np.ndarray:
    """Rows of a (rows x k) uint32 table in lexicographic order.  Each row,
    as big-endian bytes, is one fixed-width byte string whose byte order is
    the row's lexicographic order, so one string sort orders the table (an
    order of magnitude faster than a k-key lexsort on tens of millions of
    rows).  Presentation only: the library leaves row order unspecified."""
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    if rows.ndim != 2 or rows.shape[0] <= 1 or rows.shape[1] == 0:
        return rows.copy()
    k = rows.shape[1]
    b = rows.astype(">u4").view("S%d" % (4 * k)).ravel()
    b.sort(kind="stable")
    return b.view(">u4").reshape(-1, k).astype(np.uint32)


def gsi_last_error() -> str:
    return load_library().gsi_last_error().decode()


def gsi_version() -> str:
    return load_library().gsi_version().decode()


def gsi_ctx_create(device: int, hip_stream: int, arena_ptr: int, arena_bytes: int, flags: int = 0) -> int:
    o = gsi_options(device, hip_stream or None, arena_ptr, arena_bytes, flags)
    h = VP()
    _check(load_library().gsi_ctx_create(ctypes.byref(o), ctypes.byref(h)))
    return h.value


def gsi_ctx_destroy(ctx: int):
    _check(load_library().gsi_ctx_destroy(ctx))


def gsi_ctx_memory(ctx: int):
    a, b = ctypes.c_uint64(), ctypes.c_uint64()
    _check(load_library().gsi_ctx_memory(ctx, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def gsi_ctx_kernel_stats(ctx: int) -> list:
    buf = (gsi_kernel_stat * 64)()
    n = ctypes.c_uint32()
    _check(load_library().gsi_ctx_kernel_stats(ctx, buf, 64, ctypes.byref(n)))
    return [dict(name=buf[i].name.decode(), launches=buf[i].launches, total_ms=buf[i].total_ms,
                 alg_bytes=buf[i].alg_bytes) for i in range(n.value)]


def gsi_ctx_kernel_stats_reset(ctx: int):
    _check(load_library().gsi_ctx_kernel_stats_reset(ctx))


def gsi_graph_bytes_needed(n_vertices: int, n_edges: int) -> int:
    out = ctypes.c_uint64()
    _check(load_library().gsi_graph_bytes_needed(n_vertices, n_edges, ctypes.byref(out)))
    return out.value


def gsi_graph_load(ctx: int, n_vertices: int, vertex_labels, src, dst, edge_labels, flags: int = 0) -> int:
    vl, vlp = _u32(vertex_labels)
    s, sp = _u32(src)
    d, dp = _u32(dst)
    l, lp = _u32(edge_labels)
    h = VP()
    _check(load_library().gsi_graph_load(ctx, n_vertices, vlp, s.shape[0], sp, dp, lp, flags, ctypes.byref(h)))
    return h.value


def gsi_graph_load_device(ctx: int, n_vertices: int, vertex_labels_ptr: int, n_edges: int, src_ptr: int,
                          dst_ptr: int, edge_labels_ptr: int, flags: int = 0) -> int:
    h = VP()
    _check(load_library().gsi_graph_load_device(ctx, n_vertices, vertex_labels_ptr, n_edges, src_ptr, dst_ptr,
                                                edge_labels_ptr, flags, ctypes.byref(h)))
    return h.value


def gsi_graph_load_multi(ctx: int, n_vertices: int, label_offsets, labels, src, dst, edge_labels,
                         flags: int = 0) -> int:
    off = np.ascontiguousarray(label_offsets, dtype=np.uint64)
    lab, labp = _u32(labels)
    s, sp = _u32(src)
    d, dp = _u32(dst)
    l, lp = _u32(edge_labels)
    h = VP()
    _check(load_library().gsi_graph_load_multi(ctx, n_vertices, off.ctypes.data_as(U64P), labp, s.shape[0], sp, dp,
                                               lp, flags, ctypes.byref(h)))
    return h.value


def gsi_query_run_multi(g: int, k: int, label_offsets, labels, q_src, q_dst, q_edge_labels, flags: int = 0,
                        max_rows: int = 0, fused_max_rows: int = 0, fused_max_slots: int = 0, chunk_rows: int = 0,
                        chunk_min_rows: int = 0) -> int:
    off, offp = _u32(label_offsets)
    lab, labp = _u32(labels)
    s, sp = _u32(q_src)
    d, dp = _u32(q_dst)
    l, lp = _u32(q_edge_labels)
    o = gsi_query_options(flags, None, None, max_rows, fused_max_rows, fused_max_slots, chunk_rows, chunk_min_rows)
    h = VP()
    _check(load_library().gsi_query_run_multi(g, k, offp, labp, s.shape[0], sp, dp, lp, ctypes.byref(o),
                                              ctypes.byref(h)))
    return h.value


def gsi_graph_free(g: int):
    _check(load_library().gsi_graph_free(g))


def gsi_graph_get_info(g: int) -> dict:
    i = gsi_graph_info()
    _check(load_library().gsi_graph_get_info(g, ctypes.byref(i)))
    return {f: getattr(i, f) for f, _ in gsi_graph_info._fields_}


def gsi_graph_label_edges(g: int, label: int) -> int:
    out = ctypes.c_uint64()
    _check(load_library().gsi_graph_label_edges(g, label, ctypes.byref(out)))
    return out.value


def gsi_graph_copy_signatures(g: int, n_vertices: int) -> np.ndarray:
    out = np.zeros((GSI_SIG_WORDS, n_vertices), np.uint32)
    _check(load_library().gsi_graph_copy_signatures(g, out.ctypes.data_as(U32P), out.size))
    return out


def gsi_graph_copy_pcsr(g: int, label: int):
    lib = load_library()
    ng, nc = ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib.gsi_graph_copy_pcsr(g, label, None, 0, None, 0, ctypes.byref(ng), ctypes.byref(nc)))
    gl = np.zeros((ng.value, 32), np.uint32)
    ci = np.zeros(nc.value, np.uint32)
    if ng.value or nc.value:
        _check(lib.gsi_graph_copy_pcsr(g, label, gl.ctypes.data_as(U32P), gl.size, ci.ctypes.data_as(U32P), ci.size,
                                       ctypes.byref(ng), ctypes.byref(nc)))
    return gl, ci


def gsi_query_run(g: int, k: int, q_vertex_labels, q_src, q_dst, q_edge_labels, flags: int = 0, order=None,
                  first_edge=None, max_rows: int = 0, fused_max_rows: int = 0, fused_max_slots: int = 0,
                  chunk_rows: int = 0, chunk_min_rows: int = 0) -> int:
    vl, vlp = _u32(q_vertex_labels)
    s, sp = _u32(q_src)
    d, dp = _u32(q_dst)
    l, lp = _u32(q_edge_labels)
    keep = []
    o = gsi_query_options(flags, None, None, max_rows, fused_max_rows, fused_max_slots, chunk_rows, chunk_min_rows)
    if order is not None:
        a, p = _u32(order)
        keep.append(a)
        o.order = p
    if first_edge is not None:
        fe = np.array([0xFFFFFFFF if x is None else x for x in first_edge], np.uint32)
        a, p = _u32(fe)
        keep.append(a)
        o.first_edge = p
    h = VP()
    _check(load_library().gsi_query_run(g, k, vlp, s.shape[0], sp, dp, lp, ctypes.byref(o), ctypes.byref(h)))
    return h.value


def gsi_query_filter(g: int, n_vertices: int, k: int, q_vertex_labels, q_src, q_dst, q_edge_labels):
    vl, vlp = _u32(q_vertex_labels)
    s, sp = _u32(q_src)
    d, dp = _u32(q_dst)
    l, lp = _u32(q_edge_labels)
    words = (n_vertices + 63) // 64
    bits = np.zeros((k, words), np.uint64)
    cnt = np.zeros(k, np.uint32)
    _check(load_library().gsi_query_filter(g, k, vlp, s.shape[0], sp, dp, lp, bits.ctypes.data_as(U64P), bits.size,
                                           cnt.ctypes.data_as(U32P)))
    return bits, cnt


def gsi_query_run_noalloc(g: int, k: int, q_vertex_labels, q_src, q_dst, q_edge_labels, flags: int,
                          dev_rows_ptr: int, capacity_rows: int):
    """Runs a query with no device allocation (rows into the caller's device
    buffer); returns (count, (digest sum, digest xor))."""
    vl, vlp = _u32(q_vertex_labels)
    s, sp = _u32(q_src)
    d, dp = _u32(q_dst)
    l, lp = _u32(q_edge_labels)
    cnt = ctypes.c_uint64()
    dig = (ctypes.c_uint64 * 2)()
    _check(load_library().gsi_query_run_noalloc(g, k, vlp, s.shape[0], sp, dp, lp, flags, dev_rows_ptr or None,
                                                capacity_rows, ctypes.byref(cnt), dig))
    return cnt.value, (int(dig[0]), int(dig[1]))


def gsi_result_count(r: int) -> int:
    out = ctypes.c_uint64()
    _check(load_library().gsi_result_count(r, ctypes.byref(out)))
    return out.value


def gsi_result_rows(r: int, k: int) -> np.ndarray:
    n = gsi_result_count(r)
    out = np.zeros((n, k), np.uint32)
    _check(load_library().gsi_result_rows(r, out.ctypes.data_as(U32P), n))
    return out


def gsi_result_device_rows(r: int) -> int:
    p = VP()
    _check(load_library().gsi_result_device_rows(r, ctypes.byref(p)))
    return p.value or 0


def gsi_result_digest(r: int) -> tuple:
    out = (ctypes.c_uint64 * 2)()
    _check(load_library().gsi_result_digest(r, out))
    return int(out[0]), int(out[1])


def gsi_result_stats(r: int) -> dict:
    s = gsi_stats()
    _check(load_library().gsi_result_stats(r, ctypes.byref(s)))
    k = s.k
    lv = s.levels
    return dict(k=k, levels=lv, order=list(s.order[:k]), first_edge=list(s.first_edge[:k]),
                n_link=list(s.n_link[:k]), cand=list(s.cand[:k]), rows=list(s.rows[:k]), gba=list(s.gba[:k]),
                other_elems=list(s.other_elems[:k]), survivors=list(s.survivors[:k]), chunks=s.chunks,
                chunks_left=s.chunks_left, filter_ms=s.filter_ms, join_ms=s.join_ms, total_ms=s.total_ms,
                filtered_levels=s.filtered_levels)


def gsi_result_free(r: int):
    _check(load_library().gsi_result_free(r))


def _qargs(q):
    """(vertex labels, edge count, src, dst, edge labels) of a query object as
    ctypes pointers, with the arrays that back them.  Kept on the query while
    its arrays are the same objects, so a query asked again is not marshalled
    again (a few microseconds per call)."""
    key = (id(q.vlabel), id(q.src), id(q.dst), id(q.elabel))
    c = getattr(q, "_gsi_args", None)
    if c is not None and c[0] == key:
        return c[1]
    vl, vlp = _u32(q.vlabel)
    s, sp = _u32(q.src)
    d, dp = _u32(q.dst)
    l, lp = _u32(q.elabel)
    args = (vlp, s.shape[0], sp, dp, lp, (vl, s, d, l))
    try:
        q._gsi_args = (key, args)
    except AttributeError:  # objects without attributes: no cache
        pass
    return args


def _descs(queries):
    """gsi_query_desc array for query objects (k, vlabel, src, dst, elabel);
    returns (array, keep-alive list)."""
    arr = (gsi_query_desc * max(1, len(queries)))()
    keep = []
    for i, q in enumerate(queries):
        vlp, m, sp, dp, lp, backing = _qargs(q)
        keep.append(backing)
        arr[i] = gsi_query_desc(q.k, vlp, m, sp, dp, lp)
    return arr, keep


def gsi_batch_results(b: int, nq: int):
    """(counts, digests) of every query of a batch: uint64 arrays of nq and
    nq x 2."""
    counts = np.zeros(nq, np.uint64)
    digests = np.zeros((nq, 2), np.uint64)
    _check(load_library().gsi_batch_results(b, counts.ctypes.data_as(U64P), digests.ctypes.data_as(U64P)))
    return counts, digests


def gsi_batch_run(g: int, queries, flags: int = 0, threads: int = 0, grid_scale: int = 0,
                  engine_tiles: int = 0) -> int:
    arr, keep = _descs(queries)
    o = gsi_batch_options(flags, gsi_batch_schedule(threads, grid_scale, engine_tiles))
    h = VP()
    _check(load_library().gsi_batch_run(g, len(queries), arr, ctypes.byref(o), ctypes.byref(h)))
    return h.value


def gsi_batch_count(b: int, qi: int) -> int:
    out = ctypes.c_uint64()
    _check(load_library().gsi_batch_count(b, qi, ctypes.byref(out)))
    return out.value


def gsi_batch_digest(b: int, qi: int) -> tuple:
    out = (ctypes.c_uint64 * 2)()
    _check(load_library().gsi_batch_digest(b, qi, out))
    return int(out[0]), int(out[1])


def gsi_batch_rows(b: int, qi: int, k: int) -> np.ndarray:
    n = gsi_batch_count(b, qi)
    out = np.zeros((n, k), np.uint32)
    _check(load_library().gsi_batch_rows(b, qi, out.ctypes.data_as(U32P), n))
    return out


def gsi_batch_get_info(b: int) -> dict:
    i = gsi_batch_info()
    _check(load_library().gsi_batch_get_info(b, ctypes.byref(i)))
    d = {f: getattr(i, f) for f, _ in gsi_batch_info._fields_ if f != "schedule"}
    d["schedule"] = dict(threads=i.schedule.threads, grid_scale=i.schedule.grid_scale,
                         engine_tiles=i.schedule.engine_tiles)
    return d


def gsi_batch_free(b: int):
    _check(load_library().gsi_batch_free(b))


def gsi_batch_tune(g: int, queries, sample: int = 128):
    arr, keep = _descs(queries)
    sc = gsi_batch_schedule()
    ms = ctypes.c_double()
    _check(load_library().gsi_batch_tune(g, len(queries), arr, sample, ctypes.byref(sc), ctypes.byref(ms)))
    return dict(threads=sc.threads, grid_scale=sc.grid_scale, engine_tiles=sc.engine_tiles, ms_per_query=ms.value)


def gsi_server_create(g: int, flags: int = 0, max_inflight: int = 0, max_admit: int = 0, table_budget: int = 0,
                      threads: int = 0, grid_scale: int = 0, engine_tiles: int = 0, solo_queue: int = 0) -> int:
    o = gsi_server_options(flags, max_inflight, max_admit, solo_queue, table_budget,
                           gsi_batch_schedule(threads, grid_scale, engine_tiles))
    h = VP()
    _check(load_library().gsi_server_create(g, ctypes.byref(o), ctypes.byref(h)))
    return h.value


def gsi_server_submit(s: int, q) -> int:
    arr, keep = _descs([q])
    t = ctypes.c_uint64()
    _check(load_library().gsi_server_submit(s, arr, ctypes.byref(t)))
    return t.value


def gsi_server_step(s: int) -> int:
    n = ctypes.c_uint32()
    _check(load_library().gsi_server_step(s, ctypes.byref(n)))
    return n.value


def gsi_server_poll(s: int, capacity: int = 4096) -> list:
    buf = (ctypes.c_uint64 * max(1, capacity))()
    n = ctypes.c_uint32()
    _check(load_library().gsi_server_poll(s, buf, capacity, ctypes.byref(n)))
    return [int(buf[i]) for i in range(n.value)]


def gsi_server_answer_get(s: int, ticket: int) -> dict:
    a = gsi_server_answer()
    _check(load_library().gsi_server_answer_get(s, ticket, ctypes.byref(a)))
    d = {f: getattr(a, f) for f, _ in gsi_server_answer._fields_ if f != "digest"}
    d["digest"] = (int(a.digest[0]), int(a.digest[1]))
    d["path"] = PATH_NAMES.get(a.path, str(a.path))
    return d


def gsi_server_rows(s: int, ticket: int, k: int, count: int) -> np.ndarray:
    out = np.zeros((count, k), np.uint32)
    _check(load_library().gsi_server_rows(s, ticket, out.ctypes.data_as(U32P), count))
    return out


def gsi_server_release(s: int, ticket: int):
    _check(load_library().gsi_server_release(s, ticket))


def gsi_server_get_info(s: int) -> dict:
    i = gsi_server_info()
    _check(load_library().gsi_server_get_info(s, ctypes.byref(i)))
    return {f: getattr(i, f) for f, _ in gsi_server_info._fields_}


def gsi_server_free(s: int):
    _check(load_library().gsi_server_free(s))


# ------------------------------------------------------------ conveniences
class Server:
    """Continuous-batching request loop over a resident graph; the caller
    drives it with submit / step / poll."""

    def __init__(self, h: int):
        self.h = h

    def submit(self, q) -> int:
        return gsi_server_submit(self.h, q)

    def step(self) -> int:
        return gsi_server_step(self.h)

    def poll(self, capacity: int = 4096) -> list:
        return gsi_server_poll(self.h, capacity)

    def answer(self, ticket: int) -> dict:
        return gsi_server_answer_get(self.h, ticket)

    def rows(self, ticket: int) -> np.ndarray:
        a = self.answer(ticket)
        return gsi_server_rows(self.h, ticket, a["k"], a["count"])

    def sorted_rows(self, ticket: int) -> np.ndarray:
        r = self.rows(ticket)
        return sort_rows(r)

    def release(self, ticket: int):
        gsi_server_release(self.h, ticket)

    def info(self) -> dict:
        return gsi_server_get_info(self.h)

    def free(self):
        if self.h:
            gsi_server_free(self.h)
            self.h = 0


class Batch:
    def __init__(self, h: int, ks):
        self.h, self.ks = h, list(ks)

    def count(self, qi: int) -> int:
        return gsi_batch_count(self.h, qi)

    def digest(self, qi: int) -> tuple:
        return gsi_batch_digest(self.h, qi)

    def results(self):
        """(counts, digests) of every query: uint64 arrays of nq and nq x 2."""
        return gsi_batch_results(self.h, len(self.ks))

    def rows(self, qi: int) -> np.ndarray:
        return gsi_batch_rows(self.h, qi, self.ks[qi])

    def sorted_rows(self, qi: int) -> np.ndarray:
        r = self.rows(qi)
        return sort_rows(r)

    def info(self) -> dict:
        return gsi_batch_get_info(self.h)

    def free(self):
        if self.h:
            gsi_batch_free(self.h)
            self.h = 0


class Result:
    def __init__(self, h: int, k: int):
        self.h, self.k = h, k

    @property
    def count(self) -> int:
        return gsi_result_count(self.h)

    @property
    def digest(self) -> tuple:
        return gsi_result_digest(self.h)

    def rows(self) -> np.ndarray:
        return gsi_result_rows(self.h, self.k)

    def sorted_rows(self) -> np.ndarray:
        r = self.rows()
        return sort_rows(r)

    def stats(self) -> dict:
        return gsi_result_stats(self.h)

    def free(self):
        if self.h:
            gsi_result_free(self.h)
            self.h = 0


class Graph:
    def __init__(self, ctx: "Context", h: int, n: int):
        self.ctx, self.h, self.n = ctx, h, n

    def info(self) -> dict:
        return gsi_graph_get_info(self.h)

    def signatures(self) -> np.ndarray:
        return gsi_graph_copy_signatures(self.h, self.n)

    def pcsr(self, label: int):
        return gsi_graph_copy_pcsr(self.h, label)

    def query(self, q, flags: int = 0, order=None, first_edge=None, max_rows: int = 0, fused_max_rows: int = 0,
              fused_max_slots: int = 0, chunk_rows: int = 0, chunk_min_rows: int = 0) -> Result:
        if order is None and first_edge is None:
            # the common case, with the query's marshalled arrays reused
            vlp, m, sp, dp, lp, backing = _qargs(q)
            o = gsi_query_options(flags, None, None, max_rows, fused_max_rows, fused_max_slots, chunk_rows,
                                  chunk_min_rows)
            h = VP()
            _check(load_library().gsi_query_run(self.h, q.k, vlp, m, sp, dp, lp, ctypes.byref(o), ctypes.byref(h)))
            return Result(h.value, q.k)
        h = gsi_query_run(self.h, q.k, q.vlabel, q.src, q.dst, q.elabel, flags, order, first_edge, max_rows,
                          fused_max_rows, fused_max_slots, chunk_rows, chunk_min_rows)
        return Result(h, q.k)

    def query_multi(self, q, flags: int = 0, max_rows: int = 0, fused_max_rows: int = 0, fused_max_slots: int = 0,
                    chunk_rows: int = 0, chunk_min_rows: int = 0) -> Result:
        """A multi-labelled query (label sets q.qoff / q.qlab)."""
        h = gsi_query_run_multi(self.h, q.k, q.qoff, q.qlab, q.src, q.dst, q.elabel, flags, max_rows,
                                fused_max_rows, fused_max_slots, chunk_rows, chunk_min_rows)
        return Result(h, q.k)

    def filter(self, q):
        return gsi_query_filter(self.h, self.n, q.k, q.vlabel, q.src, q.dst, q.elabel)

    def query_noalloc(self, q, rows_t, flags: int = 0):
        """Query with no device allocation: rows into `rows_t` (a device
        tensor of at least k x capacity 32-bit words, capacity = its size //
        k); returns (count, digest)."""
        cap = rows_t.numel() * rows_t.element_size() // (4 * q.k)
        return gsi_query_run_noalloc(self.h, q.k, q.vlabel, q.src, q.dst, q.elabel, flags, rows_t.data_ptr(), cap)

    def batch(self, queries, flags: int = 0, threads: int = 0, grid_scale: int = 0, engine_tiles: int = 0) -> Batch:
        # the descriptor array of the last query list is kept and reused when
        # the same queries are asked again
        key = tuple(id(q) for q in queries)
        c = getattr(self, "_last_descs", None)
        if c is None or c[0] != key:
            arr, keep = _descs(queries)
            c = (key, arr, keep, [q.k for q in queries])
            self._last_descs = c
        o = gsi_batch_options(flags, gsi_batch_schedule(threads, grid_scale, engine_tiles))
        h = VP()
        _check(load_library().gsi_batch_run(self.h, len(queries), c[1], ctypes.byref(o), ctypes.byref(h)))
        return Batch(h.value, c[3])

    def tune(self, queries, sample: int = 128) -> dict:
        return gsi_batch_tune(self.h, queries, sample)

    def server(self, flags: int = 0, max_inflight: int = 0, max_admit: int = 0, table_budget: int = 0,
               threads: int = 0, grid_scale: int = 0, engine_tiles: int = 0, solo_queue: int = 0) -> Server:
        return Server(gsi_server_create(self.h, flags, max_inflight, max_admit, table_budget, threads, grid_scale,
                                        engine_tiles, solo_queue))

    def free(self):
        if self.h:
            gsi_graph_free(self.h)
            self.h = 0


class Context:
    """A library context over a torch-allocated device arena on `device`,
    using torch's current stream of that device."""

    def __init__(self, arena_bytes: int, device: int = 0, flags: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the library has no CPU path")
        load_library()
        self.torch = torch
        self.device = device
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda:%d" % device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.h = gsi_ctx_create(device, self.stream.cuda_stream, self.arena.data_ptr(), int(arena_bytes), flags)

    def load(self, g, flags: int = 0) -> Graph:
        h = gsi_graph_load(self.h, g.n, g.vlabel, g.src, g.dst, g.elabel, flags)
        return Graph(self, h, g.n)

    def load_multi(self, g, flags: int = 0) -> Graph:
        """A multi-labelled graph (label sets g.voff / g.vlab, one edge entry
        per label of a pair)."""
        h = gsi_graph_load_multi(self.h, g.n, g.voff, g.vlab, g.src, g.dst, g.elabel, flags)
        return Graph(self, h, g.n)

    def load_device(self, n: int, vlabel_t, src_t, dst_t, elabel_t, flags: int = 0) -> Graph:
        """Graph from uint32 arrays already on the device (torch int32 tensors
        holding the uint32 bit patterns)."""
        h = gsi_graph_load_device(self.h, n, vlabel_t.data_ptr(), int(src_t.numel()), src_t.data_ptr(),
                                  dst_t.data_ptr(), elabel_t.data_ptr(), flags)
        return Graph(self, h, n)

    def memory(self):
        return gsi_ctx_memory(self.h)

    def kernel_stats(self) -> list:
        return gsi_ctx_kernel_stats(self.h)

    def kernel_stats_reset(self):
        gsi_ctx_kernel_stats_reset(self.h)

    def close(self):
        if self.h:
            gsi_ctx_destroy(self.h)
            self.h = 0
            self.arena = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
