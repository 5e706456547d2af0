/*
 * CPU ORACLE — test infrastructure only.
 *
 * A plain backtracking enumerator of every label-preserving injective
 * embedding of a connected query graph Q in a data graph G.  It follows the
 * problem definition (Sec. II-A, Definitions 1-3, with Q connected) read as
 * subgraph monomorphism: a map f from V(Q) to V(G) is an embedding iff
 *   (1) f is injective,
 *   (2) L_V(f(u)) = L_V(u) for every query vertex u,
 *   (3) every query edge (u1,u2) with label l has a data edge (f(u1),f(u2))
 *       whose label is l.
 * Non-edges of Q are not constrained (the join of Sec. V checks query edges
 * only).  The result is the set of all such maps, one row per map.
 *
 * Homomorphism mode (Sec. VII-A): condition (1) is dropped, so two query
 * vertices may share a data vertex (adjacent ones cannot, G having no
 * self-loops).  The degree pruning below is dropped with it, since query
 * neighbours may then share one data neighbour.
 *
 * The search is the textbook tree search with backtracking the paper contrasts
 * its method with (Sec. I).  The first query vertex is the one whose label is
 * rarest in G; each next one is an unplaced vertex with the most already-placed
 * neighbours (ties: rarer label, then smaller id), so cycles close early.  A
 * vertex is extended from the neighbour list of whichever already-placed
 * neighbour's image has the shortest list; the other placed neighbours are
 * checked by binary search in sorted adjacency lists.  Candidates are pruned
 * by label and degree only.  The order changes only the cost of the search,
 * never the set of maps found.  Nothing here shares code with the GPU library.
 *
 * Order-independent digest of a result set: for each tuple t (query-vertex
 * order) h(t) = SplitMix64-finalizer(FNV-1a-64 of t with its k 32-bit values
 * as the symbols); the digest is (sum of h mod 2^64, xor of h).  FNV-1a is
 * Fowler/Noll/Vo's published hash (offset basis 14695981039346656037, prime
 * 1099511628211: h ^= symbol, h *= prime, for each symbol); taken over 32-bit
 * symbols instead of octets it needs k steps per tuple instead of 4k, and
 * with symbols below 256 it is the octet form.  The finalizer is the output
 * mixing function of SplitMix64 (Steele et al., OOPSLA 2014).
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * this file.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_INVALID 1
#define OR_NOMEM 2
#define OR_LIMIT 3

/* ----------------------------------------------------------- hashing */
uint64_t oracle_fnv1a64(const uint8_t *p, uint64_t n) {
    uint64_t h = 14695981039346656037ULL;
    for (uint64_t i = 0; i < n; i++) { h ^= p[i]; h *= 1099511628211ULL; }
    return h;
}
uint64_t oracle_fnv1a64_words(const uint32_t *w, uint64_t n) {
    uint64_t h = 14695981039346656037ULL;
    for (uint64_t i = 0; i < n; i++) { h ^= w[i]; h *= 1099511628211ULL; }
    return h;
}
uint64_t oracle_sm64_finalize(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
uint64_t oracle_tuple_hash(const uint32_t *t, uint32_t k) {
    return oracle_sm64_finalize(oracle_fnv1a64_words(t, k));
}
/* digest of `rows` tuples laid out row-major (rows x k) */
void oracle_digest_rows(const uint32_t *rows, uint64_t nrows, uint32_t k, uint64_t out[2]) {
    uint64_t s = 0, x = 0;
    for (uint64_t r = 0; r < nrows; r++) {
        uint64_t h = oracle_tuple_hash(rows + r * k, k);
        s += h; x ^= h;
    }
    out[0] = s; out[1] = x;
}

/* ------------------------------------------------------------- graph */
typedef struct {
    uint32_t n;
    uint64_t m;
    uint32_t *vlabel;
    uint64_t *rp;     /* n+1 */
    uint32_t *adj;    /* neighbour ids, sorted within a row */
    uint32_t *adjl;   /* edge label of each adjacency entry */
    uint32_t *sorted_labels; /* vertex labels sorted, for label counts */
} og_graph;

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}
static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : x > y;
}

void oracle_graph_free(og_graph *g) {
    if (!g) return;
    free(g->vlabel); free(g->rp); free(g->adj); free(g->adjl); free(g->sorted_labels); free(g);
}

/* Builds sorted adjacency.  *status: OR_INVALID on an endpoint out of range, a
 * self-loop or a repeated vertex pair (Definition 1: one label per edge). */
og_graph *oracle_graph_build(uint32_t n, const uint32_t *vlabel, uint64_t m, const uint32_t *src,
                             const uint32_t *dst, const uint32_t *elabel, int *status) {
    *status = OR_OK;
    og_graph *g = (og_graph *)calloc(1, sizeof(og_graph));
    if (!g) { *status = OR_NOMEM; return NULL; }
    g->n = n; g->m = m;
    g->vlabel = (uint32_t *)malloc((size_t)n * 4 + 4);
    g->rp = (uint64_t *)calloc((size_t)n + 1, 8);
    g->adj = (uint32_t *)malloc(2 * m * 4 + 4);
    g->adjl = (uint32_t *)malloc(2 * m * 4 + 4);
    g->sorted_labels = (uint32_t *)malloc((size_t)n * 4 + 4);
    uint64_t *pk = (uint64_t *)malloc(2 * m * 8 + 8);
    uint64_t *cur = (uint64_t *)malloc((size_t)n * 8 + 8);
    if (!g->vlabel || !g->rp || !g->adj || !g->adjl || !g->sorted_labels || !pk || !cur) {
        free(pk); free(cur); oracle_graph_free(g); *status = OR_NOMEM; return NULL;
    }
    memcpy(g->vlabel, vlabel, (size_t)n * 4);
    memcpy(g->sorted_labels, vlabel, (size_t)n * 4);
    qsort(g->sorted_labels, n, 4, cmp_u32);
    for (uint64_t e = 0; e < m; e++) {
        if (src[e] >= n || dst[e] >= n || src[e] == dst[e]) { *status = OR_INVALID; break; }
        g->rp[src[e] + 1]++; g->rp[dst[e] + 1]++;
    }
    if (*status) { free(pk); free(cur); oracle_graph_free(g); return NULL; }
    for (uint32_t v = 0; v < n; v++) g->rp[v + 1] += g->rp[v];
    memcpy(cur, g->rp, (size_t)n * 8);
    for (uint64_t e = 0; e < m; e++) {
        pk[cur[src[e]]++] = ((uint64_t)dst[e] << 32) | elabel[e];
        pk[cur[dst[e]]++] = ((uint64_t)src[e] << 32) | elabel[e];
    }
    free(cur);
    for (uint32_t v = 0; v < n && !*status; v++) {
        uint64_t a = g->rp[v], b = g->rp[v + 1];
        if (b - a > 1) qsort(pk + a, b - a, 8, cmp_u64);
        for (uint64_t i = a; i < b; i++) {
            g->adj[i] = (uint32_t)(pk[i] >> 32);
            g->adjl[i] = (uint32_t)pk[i];
            if (i > a && g->adj[i] == g->adj[i - 1]) *status = OR_INVALID;
        }
    }
    free(pk);
    if (*status) { oracle_graph_free(g); return NULL; }
    return g;
}

static uint64_t label_count(const og_graph *g, uint32_t lab) {
    uint64_t lo = 0, hi = g->n;
    while (lo < hi) { uint64_t mid = (lo + hi) / 2; if (g->sorted_labels[mid] < lab) lo = mid + 1; else hi = mid; }
    uint64_t a = lo; hi = g->n;
    while (lo < hi) { uint64_t mid = (lo + hi) / 2; if (g->sorted_labels[mid] <= lab) lo = mid + 1; else hi = mid; }
    return lo - a;
}

/* label of data edge (a,b), or -1 if absent */
static int64_t edge_label(const og_graph *g, uint32_t a, uint32_t b) {
    uint64_t lo = g->rp[a], hi = g->rp[a + 1];
    while (lo < hi) { uint64_t mid = (lo + hi) / 2; if (g->adj[mid] < b) lo = mid + 1; else hi = mid; }
    if (lo < g->rp[a + 1] && g->adj[lo] == b) return g->adjl[lo];
    return -1;
}

/* ------------------------------------------------------------- search */
#define MAXK 64
typedef struct {
    uint32_t k;
    int homo;                  /* homomorphism mode */
    uint32_t qlabel[MAXK];
    uint32_t qdeg[MAXK];
    uint32_t order[MAXK];      /* order[d] = query vertex placed at depth d */
    uint32_t nlink[MAXK];      /* placed neighbours of order[d], d >= 1 */
    uint32_t link_u[MAXK][MAXK];
    uint32_t link_l[MAXK][MAXK];  /* label of edge (link_u, order[d]) */
} plan_t;

typedef struct {
    const og_graph *g;
    const plan_t *p;
    const uint32_t *roots;
    uint64_t nroots;
    uint32_t tid, nthreads;
    int want_tuples;
    uint64_t max_count, max_nodes; /* per thread share checked through shared flag */
    volatile int *stop;
    /* outputs */
    uint64_t count, dsum, dxor, nodes;
    uint32_t *tuples;
    uint64_t tcap;
    int status;
    uint32_t f[MAXK];
} worker_t;

static void emit(worker_t *w) {
    const plan_t *p = w->p;
    w->count++;
    uint64_t h = oracle_tuple_hash(w->f, p->k);
    w->dsum += h; w->dxor ^= h;
    if (w->want_tuples) {
        if (w->count > w->tcap) {
            uint64_t nc = w->tcap ? w->tcap * 2 : 1024;
            uint32_t *nt = (uint32_t *)realloc(w->tuples, nc * p->k * 4);
            if (!nt) { w->status = OR_NOMEM; *w->stop = 1; return; }
            w->tuples = nt; w->tcap = nc;
        }
        memcpy(w->tuples + (w->count - 1) * p->k, w->f, p->k * 4);
    }
}

static void dfs(worker_t *w, uint32_t d) {
    const plan_t *p = w->p;
    const og_graph *g = w->g;
    if (*w->stop) return;
    if (d == p->k) {
        emit(w);
        if (w->max_count && w->count > w->max_count) { w->status = OR_LIMIT; *w->stop = 1; }
        return;
    }
    uint32_t u = p->order[d];
    /* scan the shortest neighbour list among the placed neighbours' images */
    uint32_t src = 0;
    for (uint32_t c = 1; c < p->nlink[d]; c++) {
        uint32_t a = w->f[p->link_u[d][c]], b = w->f[p->link_u[d][src]];
        if (g->rp[a + 1] - g->rp[a] < g->rp[b + 1] - g->rp[b]) src = c;
    }
    uint32_t vp = w->f[p->link_u[d][src]];
    for (uint64_t i = g->rp[vp]; i < g->rp[vp + 1]; i++) {
        if (g->adjl[i] != p->link_l[d][src]) continue;
        uint32_t x = g->adj[i];
        w->nodes++;
        if (g->vlabel[x] != p->qlabel[u]) continue;
        if (!p->homo && g->rp[x + 1] - g->rp[x] < p->qdeg[u]) continue;
        int ok = 1;
        for (uint32_t e = 0; !p->homo && e < d; e++) if (w->f[p->order[e]] == x) { ok = 0; break; }
        for (uint32_t c = 0; ok && c < p->nlink[d]; c++)
            if (c != src && edge_label(g, w->f[p->link_u[d][c]], x) != (int64_t)p->link_l[d][c]) ok = 0;
        if (!ok) continue;
        w->f[u] = x;
        dfs(w, d + 1);
        if (*w->stop) return;
    }
    if (w->max_nodes && w->nodes > w->max_nodes) { w->status = OR_LIMIT; *w->stop = 1; }
}

static void *worker_main(void *arg) {
    worker_t *w = (worker_t *)arg;
    const plan_t *p = w->p;
    uint32_t u0 = p->order[0];
    for (uint64_t r = w->tid; r < w->nroots && !*w->stop; r += w->nthreads) {
        w->nodes++;
        w->f[u0] = w->roots[r];
        dfs(w, 1);
    }
    return NULL;
}

typedef struct {
    uint64_t count, dsum, dxor, nodes;
    uint32_t *tuples; /* row-major count x k, sorted lexicographically; free with oracle_free */
    int status;
} oracle_result;

void oracle_free(void *p) { free(p); }

static uint32_t g_sort_k;
static int cmp_tuple(const void *a, const void *b) {
    const uint32_t *x = (const uint32_t *)a, *y = (const uint32_t *)b;
    for (uint32_t i = 0; i < g_sort_k; i++) if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}
static pthread_mutex_t g_sort_lock = PTHREAD_MUTEX_INITIALIZER;

/* Validates Q (k >= 1, simple, connected, endpoints in range), builds the
 * plan, enumerates.  Limits: max_count / max_nodes = 0 means unlimited; when
 * a limit is exceeded status = OR_LIMIT and the partial outputs are
 * meaningless. */
int oracle_match(const og_graph *g, uint32_t k, const uint32_t *qlabel, uint32_t qm, const uint32_t *qsrc,
                 const uint32_t *qdst, const uint32_t *qelabel, uint32_t nthreads, int want_tuples,
                 uint64_t max_count, uint64_t max_nodes, int homomorphism, oracle_result *out) {
    memset(out, 0, sizeof(*out));
    if (k < 1 || k > MAXK || nthreads < 1) return out->status = OR_INVALID;
    plan_t *p = (plan_t *)calloc(1, sizeof(plan_t));
    if (!p) return out->status = OR_NOMEM;
    p->k = k;
    p->homo = homomorphism ? 1 : 0;
    uint8_t adjq[MAXK][MAXK];
    int32_t lq[MAXK][MAXK];
    memset(adjq, 0, sizeof(adjq));
    for (uint32_t i = 0; i < k; i++) p->qlabel[i] = qlabel[i];
    for (uint32_t e = 0; e < qm; e++) {
        uint32_t a = qsrc[e], b = qdst[e];
        if (a >= k || b >= k || a == b || adjq[a][b]) { free(p); return out->status = OR_INVALID; }
        adjq[a][b] = adjq[b][a] = 1;
        lq[a][b] = lq[b][a] = (int32_t)qelabel[e];
        p->qdeg[a]++; p->qdeg[b]++;
    }
    /* first vertex: rarest label in G, ties by smallest id */
    uint32_t first = 0;
    uint64_t best = UINT64_MAX;
    for (uint32_t u = 0; u < k; u++) {
        uint64_t c = label_count(g, qlabel[u]);
        if (c < best) { best = c; first = u; }
    }
    /* next vertex: most placed neighbours, then rarer label, then smaller id */
    uint32_t pos[MAXK];
    for (uint32_t u = 0; u < k; u++) pos[u] = UINT32_MAX;
    uint32_t nord = 0;
    p->order[nord] = first; pos[first] = nord++;
    while (nord < k) {
        uint32_t pick = UINT32_MAX, pick_links = 0;
        uint64_t pick_count = 0;
        for (uint32_t y = 0; y < k; y++) {
            if (pos[y] != UINT32_MAX) continue;
            uint32_t links = 0;
            for (uint32_t e = 0; e < nord; e++) links += adjq[y][p->order[e]];
            if (links == 0) continue;
            uint64_t c = label_count(g, qlabel[y]);
            if (pick == UINT32_MAX || links > pick_links || (links == pick_links && c < pick_count)) {
                pick = y; pick_links = links; pick_count = c;
            }
        }
        if (pick == UINT32_MAX) break;
        p->order[nord] = pick; pos[pick] = nord++;
    }
    if (nord != k) { free(p); return out->status = OR_INVALID; } /* disconnected */
    for (uint32_t d = 1; d < k; d++) {
        uint32_t u = p->order[d];
        for (uint32_t e = 0; e < d; e++) {
            uint32_t x = p->order[e];
            if (adjq[u][x]) {
                p->link_u[d][p->nlink[d]] = x;
                p->link_l[d][p->nlink[d]] = (uint32_t)lq[u][x];
                p->nlink[d]++;
            }
        }
    }
    /* root candidates: label and degree */
    uint32_t u0 = p->order[0];
    uint64_t nroots = 0;
    uint32_t *roots = (uint32_t *)malloc((size_t)g->n * 4 + 4);
    for (uint32_t v = 0; v < g->n; v++)
        if (g->vlabel[v] == qlabel[u0] && (p->homo || g->rp[v + 1] - g->rp[v] >= p->qdeg[u0])) roots[nroots++] = v;

    volatile int stop = 0;
    worker_t *ws = (worker_t *)calloc(nthreads, sizeof(worker_t));
    pthread_t *th = (pthread_t *)calloc(nthreads, sizeof(pthread_t));
    for (uint32_t t = 0; t < nthreads; t++) {
        ws[t].g = g; ws[t].p = p; ws[t].roots = roots; ws[t].nroots = nroots;
        ws[t].tid = t; ws[t].nthreads = nthreads; ws[t].want_tuples = want_tuples;
        ws[t].max_count = max_count ? max_count : 0;
        ws[t].max_nodes = max_nodes ? max_nodes / nthreads + 1 : 0;
        ws[t].stop = &stop;
    }
    if (k == 1) {
        /* no extension step: every root is an embedding */
        worker_t *w = &ws[0];
        for (uint64_t r = 0; r < nroots; r++) { w->f[u0] = roots[r]; w->nodes++; emit(w); }
    } else if (nthreads == 1) {
        worker_main(&ws[0]);
    } else {
        for (uint32_t t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, worker_main, &ws[t]);
        for (uint32_t t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    }
    int status = OR_OK;
    for (uint32_t t = 0; t < nthreads; t++) {
        out->count += ws[t].count; out->dsum += ws[t].dsum; out->dxor ^= ws[t].dxor; out->nodes += ws[t].nodes;
        if (ws[t].status) status = ws[t].status;
    }
    if (max_count && out->count > max_count) status = OR_LIMIT;
    if (!status && want_tuples) {
        uint32_t *all = (uint32_t *)malloc(out->count * k * 4 + 4);
        if (!all) status = OR_NOMEM;
        else {
            uint64_t o = 0;
            for (uint32_t t = 0; t < nthreads; t++) {
                memcpy(all + o * k, ws[t].tuples, ws[t].count * k * 4);
                o += ws[t].count;
            }
            pthread_mutex_lock(&g_sort_lock);
            g_sort_k = k;
            qsort(all, out->count, (size_t)k * 4, cmp_tuple);
            pthread_mutex_unlock(&g_sort_lock);
            out->tuples = all;
        }
    }
    for (uint32_t t = 0; t < nthreads; t++) free(ws[t].tuples);
    free(ws); free(th); free(roots); free(p);
    out->status = status;
    return status;
}
