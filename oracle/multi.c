/*
 * CPU ORACLE — test infrastructure only.
 *
 * Matching under multi-labels (Sec. VII-B): a vertex carries a set of labels
 * and a vertex pair may be joined by several edges, one per label (the
 * multigraph form of a multi-labelled edge).  A map f from V(Q) to V(G) is an
 * embedding iff
 *   (1) f is injective,
 *   (2) L_V(u) is a subset of L_V(f(u)) for every query vertex u,
 *   (3) for every query vertex pair (u1,u2), the set of labels of the query
 *       edges between them is a subset of the labels of the data edges
 *       between f(u1) and f(u2).
 * With one label per vertex and per pair this is exactly the single-label
 * definition (Definitions 1-3), which match.c implements separately.
 *
 * Plain backtracking: the first query vertex is the one with the fewest data
 * vertices whose label set contains its own (ties: smaller id); then breadth
 * first over Q (neighbours by ascending id).  A vertex is extended from the
 * distinct neighbours of its first placed neighbour's image; every condition
 * is checked directly (label sets by merging sorted lists, edge labels by
 * binary search over the sorted (neighbour, label) adjacency).  Root
 * candidates are dealt round-robin to the threads.
 *
 * Shares nothing with the GPU library.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_INVALID 1
#define OR_NOMEM 2
#define OR_LIMIT 3
#define MK 64

uint64_t oracle_tuple_hash(const uint32_t *t, uint32_t k); /* match.c */

typedef struct {
    uint32_t n;
    uint64_t *loff;   /* n+1: label set of v at lab[loff[v] .. loff[v+1]), ascending, distinct */
    uint32_t *lab;
    uint64_t *rp;     /* n+1 */
    uint64_t *pair;   /* (neighbour << 32 | label), ascending within a row */
    uint32_t *ndeg;   /* distinct neighbours */
} om_graph;

static int cmp64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}
static int cmp32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : x > y;
}

void oracle_mgraph_free(om_graph *g) {
    if (!g) return;
    free(g->loff); free(g->lab); free(g->rp); free(g->pair); free(g->ndeg); free(g);
}

/* sorts and deduplicates a label set in place; returns its new size */
static uint64_t set_norm(uint32_t *a, uint64_t n) {
    if (n > 1) qsort(a, n, 4, cmp32);
    uint64_t o = 0;
    for (uint64_t i = 0; i < n; i++) if (o == 0 || a[i] != a[o - 1]) a[o++] = a[i];
    return o;
}

/* a (na entries) is a subset of b (nb entries); both ascending */
static int subset(const uint32_t *a, uint64_t na, const uint32_t *b, uint64_t nb) {
    uint64_t j = 0;
    for (uint64_t i = 0; i < na; i++) {
        while (j < nb && b[j] < a[i]) j++;
        if (j == nb || b[j] != a[i]) return 0;
        j++;
    }
    return 1;
}

/* Label sets vlab[voff[v] .. voff[v+1]) (any order, repeats allowed); edges
 * (src[e], dst[e]) with label elabel[e], one entry per label of a pair.
 * *status: OR_INVALID on an endpoint out of range, a self-loop or the same
 * (pair, label) given twice. */
om_graph *oracle_mgraph_build(uint32_t n, const uint64_t *voff, const uint32_t *vlab, uint64_t m,
                              const uint32_t *src, const uint32_t *dst, const uint32_t *elabel, int *status) {
    *status = OR_OK;
    om_graph *g = (om_graph *)calloc(1, sizeof(om_graph));
    if (!g) { *status = OR_NOMEM; return NULL; }
    g->n = n;
    g->loff = (uint64_t *)calloc((size_t)n + 1, 8);
    g->lab = (uint32_t *)malloc(voff[n] * 4 + 4);
    g->rp = (uint64_t *)calloc((size_t)n + 1, 8);
    g->pair = (uint64_t *)malloc(2 * m * 8 + 8);
    g->ndeg = (uint32_t *)calloc((size_t)n + 1, 4);
    uint64_t *cur = (uint64_t *)malloc((size_t)n * 8 + 8);
    if (!g->loff || !g->lab || !g->rp || !g->pair || !g->ndeg || !cur) {
        free(cur); oracle_mgraph_free(g); *status = OR_NOMEM; return NULL;
    }
    for (uint32_t v = 0; v < n; v++) {
        uint64_t a = voff[v], c = voff[v + 1] - a;
        memcpy(g->lab + g->loff[v], vlab + a, c * 4);
        g->loff[v + 1] = g->loff[v] + set_norm(g->lab + g->loff[v], c);
    }
    for (uint64_t e = 0; e < m; e++) {
        if (src[e] >= n || dst[e] >= n || src[e] == dst[e]) { *status = OR_INVALID; break; }
        g->rp[src[e] + 1]++; g->rp[dst[e] + 1]++;
    }
    if (*status) { free(cur); oracle_mgraph_free(g); return NULL; }
    for (uint32_t v = 0; v < n; v++) g->rp[v + 1] += g->rp[v];
    memcpy(cur, g->rp, (size_t)n * 8);
    for (uint64_t e = 0; e < m; e++) {
        g->pair[cur[src[e]]++] = ((uint64_t)dst[e] << 32) | elabel[e];
        g->pair[cur[dst[e]]++] = ((uint64_t)src[e] << 32) | elabel[e];
    }
    free(cur);
    for (uint32_t v = 0; v < n && !*status; v++) {
        uint64_t a = g->rp[v], b = g->rp[v + 1];
        if (b - a > 1) qsort(g->pair + a, b - a, 8, cmp64);
        for (uint64_t i = a; i < b; i++) {
            if (i > a && g->pair[i] == g->pair[i - 1]) *status = OR_INVALID;
            if (i == a || (g->pair[i] >> 32) != (g->pair[i - 1] >> 32)) g->ndeg[v]++;
        }
    }
    if (*status) { oracle_mgraph_free(g); return NULL; }
    return g;
}

/* data edge (a, b) with label l present? */
static int has_edge(const om_graph *g, uint32_t a, uint32_t b, uint32_t l) {
    uint64_t key = ((uint64_t)b << 32) | l, lo = g->rp[a], hi = g->rp[a + 1];
    while (lo < hi) { uint64_t mid = (lo + hi) / 2; if (g->pair[mid] < key) lo = mid + 1; else hi = mid; }
    return lo < g->rp[a + 1] && g->pair[lo] == key;
}

typedef struct {
    uint32_t k;
    uint32_t order[MK], parent[MK];     /* parent[d]: first placed neighbour of order[d] */
    uint32_t ndeg[MK];                  /* distinct query neighbours */
    const uint32_t *ql[MK];             /* label set of each query vertex (ascending) */
    uint32_t nql[MK];
    uint32_t nlab[MK][MK];              /* labels between two query vertices */
    uint32_t lab[MK][MK][8];
} mplan_t;

typedef struct {
    const om_graph *g;
    const mplan_t *p;
    const uint32_t *roots;
    uint64_t nroots;
    uint32_t tid, nthreads;
    int want;
    uint64_t max_count;
    volatile int *stop;
    uint64_t count, dsum, dxor, cap;
    uint32_t *tuples;
    int status;
    uint32_t f[MK];
    uint8_t *used;
} mworker_t;

static void memit(mworker_t *w) {
    const mplan_t *p = w->p;
    w->count++;
    uint64_t h = oracle_tuple_hash(w->f, p->k);
    w->dsum += h; w->dxor ^= h;
    if (w->max_count && w->count > w->max_count) { w->status = OR_LIMIT; *w->stop = 1; return; }
    if (!w->want) return;
    if (w->count > w->cap) {
        uint64_t nc = w->cap ? 2 * w->cap : 1024;
        uint32_t *nt = (uint32_t *)realloc(w->tuples, nc * p->k * 4);
        if (!nt) { w->status = OR_NOMEM; *w->stop = 1; return; }
        w->tuples = nt; w->cap = nc;
    }
    memcpy(w->tuples + (w->count - 1) * p->k, w->f, p->k * 4);
}

/* v may be the image of query vertex u (labels, degree, not yet used) */
static int vertex_ok(const mworker_t *w, uint32_t u, uint32_t v) {
    const om_graph *g = w->g;
    const mplan_t *p = w->p;
    if (w->used[v]) return 0;
    if (g->ndeg[v] < p->ndeg[u]) return 0;
    return subset(p->ql[u], p->nql[u], g->lab + g->loff[v], g->loff[v + 1] - g->loff[v]);
}

static void mdfs(mworker_t *w, uint32_t d) {
    const mplan_t *p = w->p;
    const om_graph *g = w->g;
    if (*w->stop) return;
    if (d == p->k) { memit(w); return; }
    uint32_t u = p->order[d], vp = w->f[p->parent[d]];
    for (uint64_t i = g->rp[vp]; i < g->rp[vp + 1]; i++) {
        uint32_t x = (uint32_t)(g->pair[i] >> 32);
        if (i > g->rp[vp] && (uint32_t)(g->pair[i - 1] >> 32) == x) continue;  /* distinct neighbours */
        if (!vertex_ok(w, u, x)) continue;
        int ok = 1;
        for (uint32_t e = 0; ok && e < d; e++) {
            uint32_t y = p->order[e];
            for (uint32_t t = 0; ok && t < p->nlab[u][y]; t++) ok = has_edge(g, x, w->f[y], p->lab[u][y][t]);
        }
        if (!ok) continue;
        w->f[u] = x;
        w->used[x] = 1;
        mdfs(w, d + 1);
        w->used[x] = 0;
        if (*w->stop) return;
    }
}

static void *mworker_main(void *arg) {
    mworker_t *w = (mworker_t *)arg;
    uint32_t u0 = w->p->order[0];
    for (uint64_t r = w->tid; r < w->nroots && !*w->stop; r += w->nthreads) {
        w->f[u0] = w->roots[r];
        w->used[w->roots[r]] = 1;
        mdfs(w, 1);
        w->used[w->roots[r]] = 0;
    }
    return NULL;
}

typedef struct {
    uint64_t count, dsum, dxor, nodes;
    uint32_t *tuples;
    int status;
} oracle_mresult;

static uint32_t g_mk;
static int cmp_row(const void *a, const void *b) {
    const uint32_t *x = (const uint32_t *)a, *y = (const uint32_t *)b;
    for (uint32_t i = 0; i < g_mk; i++) if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}
static pthread_mutex_t g_mlock = PTHREAD_MUTEX_INITIALIZER;

/* Query: label sets qlab[qoff[u] .. qoff[u+1]); edges (qsrc, qdst, qel), one
 * per label of a pair (at most 8 labels per pair).  Q must be connected. */
int oracle_mmatch(const om_graph *g, uint32_t k, const uint32_t *qoff, const uint32_t *qlab, uint32_t qm,
                  const uint32_t *qsrc, const uint32_t *qdst, const uint32_t *qel, uint32_t nthreads, int want_tuples,
                  uint64_t max_count, oracle_mresult *out) {
    memset(out, 0, sizeof(*out));
    if (k < 1 || k > MK || nthreads < 1) return out->status = OR_INVALID;
    mplan_t *p = (mplan_t *)calloc(1, sizeof(mplan_t));
    uint32_t *qsets = (uint32_t *)malloc((qoff[k] + 1) * 4);
    if (!p || !qsets) { free(p); free(qsets); return out->status = OR_NOMEM; }
    p->k = k;
    for (uint32_t u = 0; u < k; u++) {
        uint32_t a = qoff[u], c = qoff[u + 1] - a;
        memcpy(qsets + a, qlab + a, c * 4);
        p->ql[u] = qsets + a;
        p->nql[u] = (uint32_t)set_norm(qsets + a, c);
    }
    for (uint32_t e = 0; e < qm; e++) {
        uint32_t a = qsrc[e], b = qdst[e];
        if (a >= k || b >= k || a == b) { free(p); free(qsets); return out->status = OR_INVALID; }
        for (uint32_t t = 0; t < p->nlab[a][b]; t++)
            if (p->lab[a][b][t] == qel[e]) { free(p); free(qsets); return out->status = OR_INVALID; }
        if (p->nlab[a][b] == 8) { free(p); free(qsets); return out->status = OR_INVALID; }
        if (p->nlab[a][b] == 0) { p->ndeg[a]++; p->ndeg[b]++; }
        p->lab[a][b][p->nlab[a][b]++] = qel[e];
        p->lab[b][a][p->nlab[b][a]++] = qel[e];
    }
    /* first vertex: fewest data vertices containing its labels */
    uint32_t first = 0;
    uint64_t best = UINT64_MAX;
    for (uint32_t u = 0; u < k; u++) {
        uint64_t c = 0;
        for (uint32_t v = 0; v < g->n; v++)
            c += subset(p->ql[u], p->nql[u], g->lab + g->loff[v], g->loff[v + 1] - g->loff[v]);
        if (c < best) { best = c; first = u; }
    }
    /* breadth first from it */
    uint32_t pos[MK], nord = 0, head = 0;
    for (uint32_t u = 0; u < k; u++) pos[u] = UINT32_MAX;
    p->order[nord] = first; pos[first] = nord++;
    while (head < nord) {
        uint32_t x = p->order[head++];
        for (uint32_t y = 0; y < k; y++)
            if (p->nlab[x][y] && pos[y] == UINT32_MAX) { p->order[nord] = y; pos[y] = nord++; p->parent[pos[y]] = x; }
    }
    if (nord != k) { free(p); free(qsets); return out->status = OR_INVALID; }
    /* root candidates */
    uint32_t u0 = p->order[0];
    uint32_t *roots = (uint32_t *)malloc((size_t)g->n * 4 + 4);
    uint64_t nroots = 0;
    for (uint32_t v = 0; v < g->n; v++)
        if (g->ndeg[v] >= p->ndeg[u0] &&
            subset(p->ql[u0], p->nql[u0], g->lab + g->loff[v], g->loff[v + 1] - g->loff[v]))
            roots[nroots++] = v;
    volatile int stop = 0;
    mworker_t *ws = (mworker_t *)calloc(nthreads, sizeof(mworker_t));
    pthread_t *th = (pthread_t *)calloc(nthreads, sizeof(pthread_t));
    int status = OR_OK;
    for (uint32_t t = 0; t < nthreads; t++) {
        ws[t].g = g; ws[t].p = p; ws[t].roots = roots; ws[t].nroots = nroots; ws[t].tid = t;
        ws[t].nthreads = nthreads; ws[t].want = want_tuples; ws[t].max_count = max_count; ws[t].stop = &stop;
        ws[t].used = (uint8_t *)calloc((size_t)g->n + 1, 1);
        if (!ws[t].used) status = OR_NOMEM;
    }
    if (!status) {
        if (k == 1) {
            for (uint64_t r = 0; r < nroots && !stop; r++) { ws[0].f[u0] = roots[r]; memit(&ws[0]); }
        } else if (nthreads == 1) {
            mworker_main(&ws[0]);
        } else {
            for (uint32_t t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, mworker_main, &ws[t]);
            for (uint32_t t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
        }
    }
    for (uint32_t t = 0; t < nthreads; t++) {
        out->count += ws[t].count; out->dsum += ws[t].dsum; out->dxor ^= ws[t].dxor;
        if (ws[t].status) status = ws[t].status;
    }
    if (!status && want_tuples) {
        uint32_t *all = (uint32_t *)malloc(out->count * k * 4 + 4);
        if (!all) status = OR_NOMEM;
        else {
            uint64_t o = 0;
            for (uint32_t t = 0; t < nthreads; t++) { memcpy(all + o * k, ws[t].tuples, ws[t].count * k * 4); o += ws[t].count; }
            pthread_mutex_lock(&g_mlock);
            g_mk = k;
            qsort(all, out->count, (size_t)k * 4, cmp_row);
            pthread_mutex_unlock(&g_mlock);
            out->tuples = all;
        }
    }
    for (uint32_t t = 0; t < nthreads; t++) { free(ws[t].tuples); free(ws[t].used); }
    free(ws); free(th); free(roots); free(p); free(qsets);
    out->status = status;
    return status;
}
