/*
 * gsi.h — C ABI of the MI355X subgraph-isomorphism library.
 *
 * The library enumerates every label-preserving injective embedding of a
 * small connected query graph Q in a large vertex- and edge-labelled data
 * graph G (GSI, arXiv 1906.03420, Sec. II-A, Definitions 1-3; Q connected as
 * assumed in the same section).  An embedding is a map f: V(Q) -> V(G) that is
 * injective, keeps vertex labels, and maps every query edge (u1,u2) with label
 * l onto a data edge (f(u1),f(u2)) with label l.  Non-edges of Q are not
 * constrained.  The result is the table of all embeddings, one row per map,
 * column j holding f(j) (query-vertex order), or only its row count.
 *
 * Conventions
 *  - Every function returns gsi_status; nothing throws across the ABI.  On a
 *    failure gsi_last_error() returns a message for the calling thread.
 *  - Vertex ids are uint32 in [0, n_vertices); 0xFFFFFFFF is reserved.
 *    Labels are uint32; edge labels must be < GSI_MAX_EDGE_LABELS.
 *  - Graphs are simple and undirected: no self-loops and at most one edge
 *    (hence one label) per vertex pair (Definition 1).  Each undirected edge
 *    is given once.
 *  - "host" pointers are read during the call only and copied; "device"
 *    pointers are device memory on the context's GPU, read on the context's
 *    stream during the call.
 *  - All device memory the library uses is carved out of one caller-owned
 *    arena given at context creation.  The library never frees the arena and
 *    never calls hipMalloc for data; the caller keeps the arena alive until
 *    gsi_ctx_destroy returns.
 *  - Handles (context, graph, result) belong to the caller and are released
 *    with the matching *_free / *_destroy call.  A context runs one call at a
 *    time; calls on the same context from several threads must be serialised
 *    by the caller (GSI_E_BUSY is returned when they overlap).
 */
#ifndef GSI_H
#define GSI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GSI_OK = 0,
    GSI_E_INVALID = 1,   /* bad argument, graph or query */
    GSI_E_NOMEM = 2,     /* arena exhausted */
    GSI_E_DEVICE = 3,    /* a HIP runtime call failed */
    GSI_E_CAPACITY = 4,  /* caller buffer too small */
    GSI_E_BUSY = 5,      /* context already in a call */
    GSI_E_INTERNAL = 6   /* an invariant of the library failed */
} gsi_status;

#define GSI_MAX_K 32                 /* maximum query vertices */
#define GSI_MAX_EDGE_LABELS 65536    /* edge labels are < this */
#define GSI_SIG_WORDS 16             /* N = 512-bit signatures (Sec. VIII-B) */
#define GSI_PCSR_GPN 16              /* pairs per PCSR group (Sec. IV) */

/* Message for the last failure on the calling thread ("" if none). */
const char *gsi_last_error(void);
/* Library version string. */
const char *gsi_version(void);

typedef struct gsi_ctx gsi_ctx;
typedef struct gsi_graph gsi_graph;
typedef struct gsi_result gsi_result;

/* Context flags */
#define GSI_CTX_PROFILE 0x1u  /* time every kernel launch with HIP events */

typedef struct {
    int32_t device;       /* HIP device ordinal of the arena */
    void *hip_stream;     /* hipStream_t for all work; NULL = the null stream */
    void *arena_ptr;      /* device memory, 256-byte aligned, caller-owned */
    uint64_t arena_bytes; /* size of the arena */
    uint32_t flags;       /* GSI_CTX_* */
} gsi_options;

/* Creates a context over a caller-owned device arena.  Errors:
 * GSI_E_INVALID on a NULL/misaligned arena or size < 1 MiB; GSI_E_DEVICE when
 * the device cannot be selected. */
gsi_status gsi_ctx_create(const gsi_options *opts, gsi_ctx **out);
/* Releases the context (and any graph or result still alive on it). */
gsi_status gsi_ctx_destroy(gsi_ctx *ctx);
/* Arena accounting: bytes held by live graphs and results, and the peak of
 * persistent + per-call scratch bytes since creation. */
gsi_status gsi_ctx_memory(const gsi_ctx *ctx, uint64_t *live_bytes, uint64_t *peak_bytes);

/* Per-kernel timing gathered while GSI_CTX_PROFILE is set: for each kernel
 * name, the number of launches, the summed duration measured with HIP events
 * recorded on the context stream around each launch, and the summed
 * algorithmic bytes (the bytes the step must move at least, as documented per
 * kernel).  Launches of at least 16 MiB of algorithmic bytes are summed a
 * second time under "<name>@large".  Returns at most `cap` entries in `out`,
 * the number in *n. */
typedef struct {
    char name[32];
    uint64_t launches;
    double total_ms;
    double alg_bytes;
} gsi_kernel_stat;
gsi_status gsi_ctx_kernel_stats(gsi_ctx *ctx, gsi_kernel_stat *out, uint32_t cap, uint32_t *n);
gsi_status gsi_ctx_kernel_stats_reset(gsi_ctx *ctx);

/* Upper bound of arena bytes a graph of this size needs while it is built
 * (persistent structures + build scratch), so the caller can size the arena. */
gsi_status gsi_graph_bytes_needed(uint32_t n_vertices, uint64_t n_edges, uint64_t *out_bytes);

/* Graph flags */
#define GSI_GRAPH_TEST_FEW_HOME_GROUPS 0x1u  /* test only: hash PCSR keys into
    ceil(|V(D)|/16) home groups so overflow chains form (same lookups) */
#define GSI_GRAPH_KEEP_CR 0x2u  /* also keep the compressed representation
                                    (per label: ascending vertex IDs and list
                                    starts) for the GSI_ABL_CR ablation */

/*
 * Loads a data graph and builds, on the device, everything a query needs
 * (Sec. III-A offline signature table; Sec. IV PCSR for every edge label,
 * Algorithm 1):
 *   - the edge-label partitions P(G,l), each stored as PCSR(G,l) = {gl, ci}:
 *     |V(D)| groups of GPN=16 (vertex, offset) pairs, 128 bytes each, the
 *     last pair (GID, END); ci holds each vertex's l-neighbours ascending;
 *   - the column-first signature table S(v), 16 x |V| 32-bit words: word 0
 *     the vertex label, words 1..15 240 two-bit saturating groups;
 *   - |E_l| per label (for freq(l) = |E_l|/|E|, Algorithm 2).
 * vertex_labels[n_vertices]; src/dst/edge_labels[n_edges] (host memory).
 * Errors: GSI_E_INVALID for n_vertices == 0 or >= 0xFFFFFFFF, an endpoint out
 * of range, a self-loop, a repeated vertex pair, an edge label >=
 * GSI_MAX_EDGE_LABELS or more than 2^31-1 edges; GSI_E_NOMEM if the arena is
 * too small.  *out is valid only on GSI_OK.
 */
gsi_status gsi_graph_load(gsi_ctx *ctx, uint32_t n_vertices, const uint32_t *vertex_labels, uint64_t n_edges,
                          const uint32_t *src, const uint32_t *dst, const uint32_t *edge_labels, uint32_t flags,
                          gsi_graph **out);
/* Same, with the four input arrays already in device memory (not modified). */
gsi_status gsi_graph_load_device(gsi_ctx *ctx, uint32_t n_vertices, const uint32_t *vertex_labels,
                                 uint64_t n_edges, const uint32_t *src, const uint32_t *dst,
                                 const uint32_t *edge_labels, uint32_t flags, gsi_graph **out);
gsi_status gsi_graph_free(gsi_graph *g);

/*
 * Multi-labelled data graph (Sec. VII-B).  Vertex v carries the label set
 * labels[label_offsets[v] .. label_offsets[v+1]) (any order; repeats are
 * merged; label_offsets has n_vertices + 1 entries, starting at 0); a vertex
 * pair may be joined by several edges with distinct labels, one entry per
 * label (the multigraph form of a multi-labelled edge).  The structures are
 * those of gsi_graph_load: PCSR per edge label (each partition stays simple),
 * and signatures in which word 0 holds every vertex label hashed to one of
 * 32 bits and each neighbour contributes one (edge label, vertex label) pair
 * per label it carries.  Host memory.  Queries on it: gsi_query_run_multi (or
 * gsi_query_run, read as singleton label sets); the batched path and the
 * server take single-label graphs only.  Errors as gsi_graph_load, with
 * GSI_E_INVALID for the same (pair, label) given twice.
 */
gsi_status gsi_graph_load_multi(gsi_ctx *ctx, uint32_t n_vertices, const uint64_t *label_offsets,
                                const uint32_t *labels, uint64_t n_edges, const uint32_t *src, const uint32_t *dst,
                                const uint32_t *edge_labels, uint32_t flags, gsi_graph **out);

typedef struct {
    uint32_t n_vertices;
    uint64_t n_edges;
    uint32_t n_edge_labels;  /* max edge label + 1 */
    uint64_t total_groups;   /* sum over labels of |V(D)| */
    uint32_t max_chain;      /* longest PCSR group chain (1 = no overflow) */
    uint64_t device_bytes;   /* persistent bytes of PCSR + signatures */
    double build_ms;         /* device time of the build */
} gsi_graph_info;
gsi_status gsi_graph_get_info(const gsi_graph *g, gsi_graph_info *out);
/* |E_l| (undirected edges with label l); 0 for an absent label. */
gsi_status gsi_graph_label_edges(const gsi_graph *g, uint32_t label, uint64_t *out);

/* Copies the signature table (16 x n_vertices uint32, column-first: word w of
 * vertex v at [w * n_vertices + v]) to host memory of `capacity_words`. */
gsi_status gsi_graph_copy_signatures(const gsi_graph *g, uint32_t *host_dst, uint64_t capacity_words);
/* Copies PCSR(G,label): gl as groups x 32 uint32 (pairs interleaved vertex,
 * offset; offsets relative to this label's ci) and ci.  With host buffers of
 * zero capacity only the sizes are returned. GSI_E_CAPACITY if too small. */
gsi_status gsi_graph_copy_pcsr(const gsi_graph *g, uint32_t label, uint32_t *host_gl, uint64_t gl_capacity_words,
                               uint32_t *host_ci, uint64_t ci_capacity, uint64_t *out_groups, uint64_t *out_ci_len);

/* Query flags */
#define GSI_COUNT_ONLY 0x1u        /* keep count and digest, write no rows */
#define GSI_FILTER_LABEL_ONLY 0x2u /* test only: C(u) = vertices with u's label
                                      (skips the signature test) */
#define GSI_NO_FUSED 0x4u          /* run every level with the per-level kernels
                                      (no fused small-table workgroup) */
#define GSI_NO_CHUNKS 0x10u        /* no root chunks (see gsi_query_run) */
#define GSI_LEVEL_FIRST_EDGE 0x20u /* every row of a level scans the list of the
                                      level's first edge e0 (Algorithm 4), not
                                      its shortest linking list */
#define GSI_NO_LIST_FILTER 0x8000u /* no level-wide filtering of first-edge lists
                                      (see gsi_query_run) */
#define GSI_SINGLE_PASS 0x20000u    /* the last per-level level (and inner levels
                                      with filtered lists and one linking edge)
                                      in one launch with a decoupled look-back
                                      instead of separate join, scan and link
                                      launches (see gsi_query_run) */
/* Ablations (measurement and tests only; each implies GSI_NO_FUSED, since
 * they change the per-level kernels): */
#define GSI_ABL_CR 0x100u          /* N(v,l) by binary search in the compressed
                                      representation instead of PCSR (the graph
                                      needs GSI_GRAPH_KEEP_CR) */
#define GSI_ABL_TWO_STEP 0x200u    /* two-step output instead of Prealloc-
                                      Combine: the join only counts survivors,
                                      the write pass repeats the join */
#define GSI_ABL_NO_STAGING 0x400u  /* last-level rows written straight from each
                                      thread (no LDS staging) */
#define GSI_ABL_NAIVE_SETOPS 0x800u  /* one kernel per set operation (subtraction,
                                      C(u), each further linking edge) over a
                                      vertex-id buffer in GBA, instead of the
                                      fused, LDS-staged join (Sec. V) */
#define GSI_ABL_ROW_PER_WAVE 0x1000u /* one wave per row of M scans the row's list
                                      (Algorithm 3 without load balance) instead
                                      of equal tiles over the |GBA| slots */
#define GSI_ABL_FOUR_LAYER 0x2000u   /* the 4-layer load balance of Sec. VI-A
                                      (1024-thread workgroups; W1 = 4096,
                                      W2 = 1024, W3 = 256) instead of equal tiles */
#define GSI_ABL_DUP_REMOVAL 0x4000u  /* with GSI_ABL_ROW_PER_WAVE or
                                      GSI_ABL_FOUR_LAYER: waves of a workgroup
                                      whose rows scan the same list share its
                                      reads through LDS (Algorithm 5, Sec. VI-B) */
#define GSI_HOMOMORPHISM 0x40u     /* homomorphism semantics (Sec. VII-A): query
                                      vertices may share a data vertex; the join
                                      drops the subtraction of m_i and the filter
                                      asks for one neighbour per signature group */

/* Optional controls of one query run (NULL = defaults). */
typedef struct {
    uint32_t flags;            /* GSI_COUNT_ONLY | GSI_FILTER_LABEL_ONLY */
    const uint32_t *order;     /* NULL, or k query vertices: the matching order */
    const uint32_t *first_edge;/* NULL, or k entries: first_edge[j] (j >= 1) is
                                  the placed query vertex whose edge to order[j]
                                  is e0 (Algorithm 4); needs `order` */
    uint64_t max_rows;         /* 0, or a cap on rows of any intermediate table;
                                  exceeding it returns GSI_E_CAPACITY */
    uint32_t fused_max_rows;   /* 0 = default (4096); test only: a lower row
                                  capacity of the fused small-table workgroup */
    uint32_t fused_max_slots;  /* 0 = default (16384); test only: a lower |GBA|
                                  capacity of the fused workgroup */
    uint32_t chunk_rows;       /* 0 = automatic; else root rows per chunk */
    uint32_t chunk_min_rows;   /* 0 = default (4097); root chunks are used when
                                  |C(u_first)| is at least this */
} gsi_query_options;

/*
 * Runs one query (Sec. III: filtering then joining):
 *   1. query signatures S(u) (host) and the signature filter over the whole
 *      table, all query vertices in one pass: C(u) as a |V|-bit bitset;
 *   2. the matching order of Algorithm 2 (host, from |C(u)| and freq(l));
 *   3. M = C(u_first); then for each further query vertex u one join level
 *      (Algorithm 3 with Algorithm 4): locate N(v',l) through PCSR for every
 *      linking edge; each row scans its shortest located list (the list of
 *      Algorithm 4's first edge e0 on ties, or always with
 *      GSI_LEVEL_FIRST_EDGE or a given first_edge); prefix-sum the scanned
 *      lengths into F (|GBA|); keep x of row m_i's scanned list iff x is not
 *      in m_i, x is in C(u) and x is in every other linking list; prefix-sum
 *      survivors; link m_i with each survivor into M' (Prealloc-Combine, one
 *      join pass);
 *   4. the last level writes rows in query-vertex order (or only counts) and
 *      the order-independent digest.
 * A per-level level whose |GBA| exceeds twice the directed entries of its
 * first edge's label l0 (rows repeating hub vertices rescan the same lists)
 * first filters l0's lists by C(u) once for the level, in order, and its
 * rows scan the filtered lists (e0's for every row); the rows, count and
 * digest are unchanged, only |GBA| shrinks (GSI_NO_LIST_FILTER turns this
 * off).  With GSI_SINGLE_PASS the last per-level level runs in one launch:
 * each tile joins, finds the rows before it by a decoupled look-back over the
 * tiles started before it, and writes its rows at once (output sized at |GBA|
 * rows, then shrunk); by default it runs as separate join, scan and link
 * launches, which measure faster (a tile's rows wait on the slowest join
 * before it).
 * Up to 4096 roots one fused workgroup runs the levels while the tables stay
 * small (4096 rows and 16384 |GBA| slots per level, with F, the keep bits and
 * the survivor prefix sums in LDS); the per-level kernels run a level that
 * does not fit, and the workgroup takes the query back once the new table
 * fits and the next level's |GBA|, estimated at the current slots per row,
 * would fit too.  Above that, rows of M being
 * independent at every level, step 3 first runs on root chunks: small groups
 * of rows of M = C(u_first), each taken by one 256-thread workgroup of a
 * persistent launch that runs all levels of its chunk (1024 rows and 4096
 * slots per level).  The roots of chunks that do not fit continue with the
 * per-level kernels; the rows of both parts are concatenated (chunk rows
 * first, in root order).  Every route gives the same rows, count and digest.
 * q_vertex_labels[k]; q_src/q_dst/q_edge_labels[q_edges] (host).
 * Errors: GSI_E_INVALID for k == 0 or k > GSI_MAX_K, an endpoint >= k, a
 * self-loop, a repeated pair, a disconnected Q or a bad option; GSI_E_NOMEM
 * when the arena cannot hold a level.  An edge label absent from G is not an
 * error: the result has 0 rows.
 */
gsi_status gsi_query_run(gsi_graph *g, uint32_t k, const uint32_t *q_vertex_labels, uint32_t q_edges,
                         const uint32_t *q_src, const uint32_t *q_dst, const uint32_t *q_edge_labels,
                         const gsi_query_options *opts, gsi_result **out);

/*
 * Runs a multi-labelled query (Sec. VII-B): f is an embedding iff it is
 * injective, the label set of every query vertex u is contained in that of
 * f(u), and the labels of the query edges between every vertex pair are
 * among the labels of the data edges between their images.  Query vertex u
 * carries labels[label_offsets[u] .. label_offsets[u+1]) (label_offsets has
 * k + 1 entries, starting at 0; at most 256 labels in all); a query pair may
 * appear in several edges with distinct labels.  The path is gsi_query_run's
 * with the filter testing containment: the signature test, then each
 * candidate's label set checked exactly; the join then intersects the
 * partitions of every labelled edge to a placed vertex, so a pair with two
 * labels needs both.  On a single-label graph a vertex set of two or more
 * labels, or a pair with two labels, has no match (0 rows).  Options, result
 * and errors as gsi_query_run.
 */
gsi_status gsi_query_run_multi(gsi_graph *g, uint32_t k, const uint32_t *label_offsets, const uint32_t *labels,
                               uint32_t q_edges, const uint32_t *q_src, const uint32_t *q_dst,
                               const uint32_t *q_edge_labels, const gsi_query_options *opts, gsi_result **out);

/* Runs only the signature filter (step 1 above) and copies C(u) bitsets
 * (k x ceil(n/64) uint64, bit v%64 of word v/64 set iff v in C(u)) and
 * counts (k uint32) to host memory. */
gsi_status gsi_query_filter(gsi_graph *g, uint32_t k, const uint32_t *q_vertex_labels, uint32_t q_edges,
                            const uint32_t *q_src, const uint32_t *q_dst, const uint32_t *q_edge_labels,
                            uint64_t *host_bitsets, uint64_t capacity_words, uint32_t *host_counts);

/*
 * For callers that cannot allocate device memory during a call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * gsi_query_run without any device allocation.  Every scratch buffer of the
 * query comes from a fixed array of GSI_NOALLOC_SCRATCH_BYTES in the
 * library's own device memory (one per GPU, held until the process ends; its
 * address is taken when the first context on that GPU is created), and the
 * rows are copied into the caller's device buffer.  Results (rows as a set,
 * count, digest) are those of gsi_query_run with the same flags.
 *   flags           GSI_COUNT_ONLY and the other gsi_query_options flags
 *   dev_rows        device memory on the context's GPU, capacity_rows x k
 *                   uint32, row-major, column j = f(j) (ignored with
 *                   GSI_COUNT_ONLY); written on the context's stream, complete
 *                   when the call returns
 *   out_count, out_digest  the row count and the (sum, xor) digest
 * Single-label graphs only.  Every call on one GPU shares its scratch array
 * and finds it as the previous call left it; calls on one context are
 * serialised (GSI_E_BUSY), calls on two contexts of one GPU overlapping in
 * time race on the array and must be serialised by the caller.
 * Errors: as gsi_query_run; GSI_E_CAPACITY when the query needs more scratch
 * than the array holds (its candidate bitsets alone, k x |V|/8 bytes, may
 * take at most half of it) or when the rows exceed capacity_rows
 * (*out_count then holds the row count).
 */
#define GSI_NOALLOC_SCRATCH_BYTES (128ull << 20)
gsi_status gsi_query_run_noalloc(gsi_graph *g, uint32_t k, const uint32_t *q_vertex_labels, uint32_t q_edges,
                                 const uint32_t *q_src, const uint32_t *q_dst, const uint32_t *q_edge_labels,
                                 uint32_t flags, uint32_t *dev_rows, uint64_t capacity_rows, uint64_t *out_count,
                                 uint64_t out_digest[2]);

/* Number of embeddings (rows). */
gsi_status gsi_result_count(const gsi_result *r, uint64_t *rows);
/* Copies the rows (row-major, rows x k uint32, column j = f(j)) to host memory
 * of capacity_rows rows; GSI_E_CAPACITY if too small; GSI_E_INVALID for a
 * GSI_COUNT_ONLY result.  Row order is deterministic but unspecified. */
gsi_status gsi_result_rows(const gsi_result *r, uint32_t *host_dst, uint64_t capacity_rows);
/* Borrowed device pointer to the same rows; valid until gsi_result_free. */
gsi_status gsi_result_device_rows(const gsi_result *r, const uint32_t **dev_rows);
/* Order-independent digest: for each row t, h(t) = SplitMix64 finalizer of
 * FNV-1a-64 over t's k values taken as 32-bit symbols (h ^= t[j], h *= prime,
 * j = 0..k-1); out = {sum of h mod 2^64, xor of h}. */
gsi_status gsi_result_digest(const gsi_result *r, uint64_t out_sum_xor[2]);

typedef struct {
    uint32_t k;
    uint32_t levels;                 /* join levels run (k-1 unless stopped early) */
    uint32_t order[GSI_MAX_K];       /* matching order (query vertex ids) */
    uint32_t first_edge[GSI_MAX_K];  /* first_edge[j]: placed end of e0 at level j */
    uint32_t n_link[GSI_MAX_K];      /* |ES| at level j */
    uint32_t cand[GSI_MAX_K];        /* |C(u)| per query vertex id */
    uint64_t rows[GSI_MAX_K];        /* rows[j] = rows of M entering level j (rows[0] = |C(order[0])|) */
    uint64_t gba[GSI_MAX_K];         /* |GBA| at level j */
    uint64_t other_elems[GSI_MAX_K]; /* sum of non-first linking list lengths at level j
                                        (gathered in GSI_CTX_PROFILE contexts only, else 0) */
    uint64_t survivors[GSI_MAX_K];   /* rows of M' produced by level j */
    uint32_t chunks;                 /* root chunks run (0: none) */
    uint32_t chunks_left;            /* chunks finished by the per-level kernels */
    double filter_ms;                /* host wall time of the filter step */
    double join_ms;                  /* host wall time of the joins */
    double total_ms;                 /* host wall time of the whole call */
    uint32_t filtered_levels;        /* bit j: level j scanned filtered first-edge lists */
} gsi_stats;
gsi_status gsi_result_stats(const gsi_result *r, gsi_stats *out);
gsi_status gsi_result_free(gsi_result *r);

/* ------------------------------------------------------------ batches */
/* One query of a batch (host arrays, read during the call). */
typedef struct {
    uint32_t k;
    const uint32_t *vertex_labels;  /* k */
    uint32_t n_edges;
    const uint32_t *src, *dst, *edge_labels;  /* n_edges each */
} gsi_query_desc;

/* How a batch is scheduled.  Queries whose tables stay small run in a
 * persistent fused launch: every workgroup takes the next query from a
 * shared counter and runs all of its join levels (Algorithm 3 with
 * Algorithm 4) in LDS-staged form.  A first tier uses workgroups of
 * `threads` threads (64, 256 or 1024; tables of up to 4x`threads` rows and
 * 16x`threads` |GBA| slots per level); queries it cannot hold rerun in a
 * second tier of 1024-thread workgroups, and the rest run level-synchronously
 * together.  `grid_scale` (1..8) multiplies the number of
 * resident workgroups per compute unit that is launched, in eighths. */
typedef struct {
    uint32_t threads;     /* first-tier workgroup size: 64, 256 or 1024 */
    uint32_t grid_scale;  /* eighths of full occupancy launched, 1..8 */
    uint32_t engine_tiles;/* 256-slot tiles per workgroup of the level-
                             synchronous join and link: 1, 2, 4 or 8 (each
                             thread then takes that many slots); 0 = 4 */
} gsi_batch_schedule;

#define GSI_BATCH_LEVELS_ONLY 0x8u /* test only: no fused tiers; every query runs
                                      in the level-synchronous engine */
typedef struct {
    uint32_t flags;               /* GSI_COUNT_ONLY | GSI_BATCH_LEVELS_ONLY */
    gsi_batch_schedule schedule;  /* threads == 0: the graph's tuned schedule
                                     (gsi_batch_tune), else 256 / 8 eighths */
} gsi_batch_options;

typedef struct gsi_batch gsi_batch;

/* Runs `nq` queries over one resident graph (the batched path):
 *   1. one signature-filter pass per 32 query vertices of the whole batch
 *      (query vertices grouped by label), one readback of all |C(u)|;
 *   2. each query's matching order (Algorithm 2) on the host;
 *   3. all root tables C(u_first) compacted in one pass;
 *   4. the fused tiers; every query they cannot hold then runs in the
 *      level-synchronous engine: each step advances all of them by one join
 *      level in shared launches (one global row space, one global |GBA| slot
 *      space), with exact per-query table sizes read back once per step.
 * Every query's result is the one gsi_query_run returns (same rows, count
 * and digest; row order may differ).  Errors as gsi_query_run, for the first
 * invalid query (its index is in the message). */
gsi_status gsi_batch_run(gsi_graph *g, uint32_t nq, const gsi_query_desc *queries, const gsi_batch_options *opt,
                         gsi_batch **out);
gsi_status gsi_batch_count(const gsi_batch *b, uint32_t qi, uint64_t *rows);
gsi_status gsi_batch_digest(const gsi_batch *b, uint32_t qi, uint64_t out_sum_xor[2]);
/* Every query's count and digest at once: counts[nq], digests[2 nq] (sum,
 * xor of query qi at 2 qi, 2 qi + 1), host memory of the batch's nq. */
gsi_status gsi_batch_results(const gsi_batch *b, uint64_t *counts, uint64_t *digests);
/* Rows of query qi, row-major in query-vertex order; GSI_E_CAPACITY if
 * capacity_rows is too small, GSI_E_INVALID for a GSI_COUNT_ONLY batch. */
gsi_status gsi_batch_rows(const gsi_batch *b, uint32_t qi, uint32_t *host_dst, uint64_t capacity_rows);

typedef struct {
    uint32_t queries;
    uint32_t empty;        /* answered by the filter alone (0 rows) */
    uint32_t tier1;        /* finished in the first fused tier */
    uint32_t tier2;        /* finished in the 1024-thread tier */
    uint32_t per_level;    /* finished with the per-level kernels */
    gsi_batch_schedule schedule;
    double filter_ms, tier1_ms, tier2_ms, per_level_ms, total_ms;  /* host wall time */
} gsi_batch_info;
gsi_status gsi_batch_get_info(const gsi_batch *b, gsi_batch_info *out);
gsi_status gsi_batch_free(gsi_batch *b);

/* Autotuner: runs a sample of the batch (the first min(nq, sample) queries,
 * counts only) under candidate schedules and keeps the fastest as the
 * graph's tuned schedule (used when gsi_batch_options.schedule.threads is
 * 0): first the fused tiers — first-tier sizes 64, 256 and 1024 threads
 * (one, four or sixteen wavefronts per query) at full and half occupancy —
 * then, with the winner, the level-synchronous engine's tiles per workgroup
 * (1, 2, 4, 8: slots per thread).  The winner and its time per query are
 * returned. */
gsi_status gsi_batch_tune(gsi_graph *g, uint32_t nq, const gsi_query_desc *queries, uint32_t sample,
                          gsi_batch_schedule *out, double *out_ms_per_query);

/* ------------------------------------------------------------ serving */
/* A request loop over one resident graph (continuous batching).  Queries
 * are submitted at any time and wait in arrival order.  Each
 * gsi_server_step admits waiting queries, then advances every admitted
 * query by one join level:
 *   admission  up to max_admit waiting queries (first come, first served)
 *              are admitted while the in-flight count stays within
 *              max_inflight and the predicted intermediate-table bytes of
 *              all admitted queries stay within table_budget (a query
 *              admitted when nothing is in flight always fits).  The
 *              prediction follows the join of Algorithm 3: from |C(u)| (the
 *              vertices of u's label before the filter runs, the filtered
 *              count after), the number of PCSR vertices and edges per edge
 *              label (Sec. IV), it estimates every level's table and |GBA|
 *              and keeps the largest step; it is recomputed from the true
 *              table size after every step.  The admitted set then goes
 *              through one batched filter pass, plans (Algorithm 2) and the
 *              fused tiers, as in gsi_batch_run;
 *   levels     the queries the fused tiers cannot hold join the
 *              level-synchronous engine and advance one level per step in
 *              launches shared with every other query in flight, whatever
 *              level each is at.  When a step does not fit the arena it runs
 *              on fewer queries (a misprediction costs time, not a failure);
 *              a query whose level does not fit even alone after the others
 *              have drained finishes with status GSI_E_NOMEM.
 *   solo       at low load — nothing in flight and at most solo_queue
 *              requests waiting — the step instead answers the oldest request
 *              alone through gsi_query_run's path (fused workgroup, root
 *              chunks, per-level kernels), which has the lowest latency; once
 *              the queue grows past solo_queue, requests are admitted in
 *              batches as above (throughput).  GSI_SERVER_NO_SOLO turns this
 *              off.
 * PCSR, signatures, candidate bitsets and partial tables stay on the device.
 * Answers are the ones gsi_query_run gives for the same query alone (count,
 * digest, rows as a set).  Calls on one server must not overlap; the server
 * uses its graph's context (GSI_E_BUSY while another call runs on it). */
typedef struct gsi_server gsi_server;

#define GSI_SERVER_NO_SOLO 0x2u    /* server flag: never answer a request alone */
typedef struct {
    uint32_t flags;         /* GSI_COUNT_ONLY: answers hold count and digest;
                               GSI_SERVER_NO_SOLO */
    uint32_t max_inflight;  /* admitted queries not yet finished; 0: 1024 */
    uint32_t max_admit;     /* queries admitted per step; 0: 256 */
    uint32_t solo_queue;    /* longest queue still served one request at a
                               time when nothing is in flight; 0: 2 */
    uint64_t table_budget;  /* bytes; 0: half of the arena's largest free block
                               when the server is created */
    gsi_batch_schedule schedule;  /* fused tiers; threads == 0: the graph's
                                     tuned schedule, else 256 / 8 eighths */
} gsi_server_options;

/* Errors: GSI_E_INVALID for a bad option; GSI_E_NOMEM / GSI_E_DEVICE. */
gsi_status gsi_server_create(gsi_graph *g, const gsi_server_options *opt, gsi_server **out);
/* Copies and validates the query (errors as gsi_query_run) and queues it;
 * the ticket (> 0, increasing) names it in the calls below. */
gsi_status gsi_server_submit(gsi_server *s, const gsi_query_desc *query, uint64_t *ticket);
/* One admission and one level step; *finished = queries answered in it. */
gsi_status gsi_server_step(gsi_server *s, uint32_t *finished);
/* Moves up to `capacity` answered tickets (in the order they finished) to
 * `tickets`; *n = how many. */
gsi_status gsi_server_poll(gsi_server *s, uint64_t *tickets, uint32_t capacity, uint32_t *n);

#define GSI_PATH_EMPTY 0   /* answered by the filter (0 rows) */
#define GSI_PATH_TIER1 1   /* first fused tier */
#define GSI_PATH_TIER2 2   /* 1024-thread fused tier */
#define GSI_PATH_SINGLE 3  /* one-vertex query */
#define GSI_PATH_LEVELS 4  /* level-synchronous engine */
#define GSI_PATH_SOLO 5    /* alone, through gsi_query_run's path (low load) */
typedef struct {
    gsi_status status;         /* GSI_OK, or GSI_E_NOMEM (see above) */
    uint32_t k;
    uint64_t count;
    uint64_t digest[2];        /* (sum, xor) as gsi_result_digest */
    uint32_t path;             /* GSI_PATH_* */
    uint32_t levels;           /* level steps taken in the engine */
    uint64_t predicted_bytes;  /* prediction at submission */
    uint64_t peak_table_bytes; /* largest table held between steps */
    double submit_ms, admit_ms, done_ms;  /* host clock, since creation */
} gsi_server_answer;
/* Errors: GSI_E_INVALID for an unknown, released or unfinished ticket. */
gsi_status gsi_server_answer_get(const gsi_server *s, uint64_t ticket, gsi_server_answer *out);
/* Rows of an answered ticket, row-major in query-vertex order (sorted only
 * as the engine left them); GSI_E_CAPACITY if capacity_rows is too small,
 * GSI_E_INVALID for a GSI_COUNT_ONLY server. */
gsi_status gsi_server_rows(gsi_server *s, uint64_t ticket, uint32_t *host_dst, uint64_t capacity_rows);
/* Frees an answered ticket's rows and record. */
gsi_status gsi_server_release(gsi_server *s, uint64_t ticket);

typedef struct {
    uint64_t submitted, admitted, answered, released;
    uint32_t waiting, in_flight;      /* now */
    uint64_t steps, level_steps, admit_rounds;
    uint64_t predicted_in_flight;     /* bytes, now */
    uint64_t peak_predicted;          /* largest admitted prediction sum */
    uint64_t table_budget;
    double admit_ms, level_ms;        /* host wall time in the two phases */
    uint64_t solo;                    /* requests answered alone (low load) */
} gsi_server_info;
gsi_status gsi_server_get_info(const gsi_server *s, gsi_server_info *out);
/* Drops every query (waiting, in flight or answered) and the server. */
gsi_status gsi_server_free(gsi_server *s);

#ifdef __cplusplus
}
#endif
#endif /* GSI_H */
