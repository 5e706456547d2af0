/*
 * Seeded synthetic input generators for labelled data graphs and query graphs.
 *
 * This file holds graph *generation* only: random graph models, label
 * assignment and random-walk query extraction.  It contains none of the
 * matching method's arithmetic (no signatures, no hashed adjacency, no joins)
 * and is the one module whose outputs feed both the CPU oracle and the GPU
 * library.
 *
 * Pseudo-random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), written from its published
 * definition.  Bounded integers use Lemire's multiply-shift reduction
 * ("Fast random integer generation in an interval", 2019) without the
 * rejection step (bias < n / 2^64, irrelevant for workload synthesis).
 *
 * Models:
 *   - Erdos-Renyi G(n, m): m distinct unordered pairs, uniform, no self-loops.
 *   - Barabasi-Albert via the Batagelj-Brandes edge-list method ("Efficient
 *     generation of large random networks", Phys. Rev. E 71, 2005): a seed
 *     clique K_{d+1}, then each new vertex attaches d distinct targets drawn
 *     proportionally to degree (uniform position in the endpoint list).
 *   - R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004) with quadrant
 *     probabilities (a, b, c, 1-a-b-c), canonical (min,max) pairs, self-loops
 *     and duplicates dropped until exactly m edges remain.
 * Vertex ids of BA and R-MAT graphs are shuffled by Fisher-Yates.
 *
 * Queries follow the paper's recipe (Sec. VIII-A): a random walk from a
 * random vertex until k distinct vertices are visited; visited vertices and
 * edges, with their labels, form the query.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ---------------------------------------------------------------- PRNG */
static inline uint64_t sm64(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline uint64_t below(uint64_t *s, uint64_t n) {
    return (uint64_t)(((unsigned __int128)sm64(s) * n) >> 64);
}
static inline double unit(uint64_t *s) { return (double)(sm64(s) >> 11) * (1.0 / 9007199254740992.0); }

/* ---------------------------------------------------------- hash set u64 */
typedef struct { uint64_t *slot; uint64_t mask; } pairset;
#define EMPTY_KEY 0xFFFFFFFFFFFFFFFFULL
static int ps_init(pairset *p, uint64_t expected) {
    uint64_t cap = 16;
    while (cap < expected * 2) cap <<= 1;
    p->slot = (uint64_t *)malloc(cap * sizeof(uint64_t));
    if (!p->slot) return -1;
    memset(p->slot, 0xFF, cap * sizeof(uint64_t));
    p->mask = cap - 1;
    return 0;
}
static inline uint64_t mix(uint64_t x) {
    x ^= x >> 33; x *= 0xFF51AFD7ED558CCDULL; x ^= x >> 33;
    x *= 0xC4CEB9FE1A85EC53ULL; x ^= x >> 33; return x;
}
/* returns 1 if inserted, 0 if present */
static inline int ps_insert(pairset *p, uint64_t key) {
    uint64_t h = mix(key) & p->mask;
    for (;;) {
        uint64_t k = p->slot[h];
        if (k == EMPTY_KEY) { p->slot[h] = key; return 1; }
        if (k == key) return 0;
        h = (h + 1) & p->mask;
    }
}
static void ps_free(pairset *p) { free(p->slot); p->slot = NULL; }

static void shuffle_ids(uint32_t n, uint64_t m, uint32_t *src, uint32_t *dst, uint64_t *st) {
    uint32_t *perm = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    for (uint32_t i = 0; i < n; i++) perm[i] = i;
    for (uint32_t i = n; i > 1; i--) {
        uint32_t j = (uint32_t)below(st, i);
        uint32_t t = perm[i - 1]; perm[i - 1] = perm[j]; perm[j] = t;
    }
    for (uint64_t e = 0; e < m; e++) { src[e] = perm[src[e]]; dst[e] = perm[dst[e]]; }
    free(perm);
}

/* ------------------------------------------------------------- models */
int gen_er(uint32_t n, uint64_t m, uint64_t seed, uint32_t *src, uint32_t *dst) {
    if (n < 2 || m > (uint64_t)n * (n - 1) / 2) return -1;
    uint64_t st = seed;
    pairset ps;
    if (ps_init(&ps, m)) return -2;
    uint64_t e = 0;
    while (e < m) {
        uint32_t a = (uint32_t)below(&st, n), b = (uint32_t)below(&st, n);
        if (a == b) continue;
        uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
        if (!ps_insert(&ps, ((uint64_t)lo << 32) | hi)) continue;
        src[e] = lo; dst[e] = hi; e++;
    }
    ps_free(&ps);
    return 0;
}

uint64_t gen_ba_edge_count(uint32_t n, uint32_t d) {
    if (n < d + 1) return 0;
    return (uint64_t)(d + 1) * d / 2 + (uint64_t)d * (n - d - 1);
}

int gen_ba(uint32_t n, uint32_t d, uint64_t seed, uint32_t *src, uint32_t *dst) {
    if (d < 1 || n < d + 1) return -1;
    uint64_t st = seed;
    uint64_t total = gen_ba_edge_count(n, d);
    uint32_t *ep = (uint32_t *)malloc(total * 2 * sizeof(uint32_t));
    if (!ep) return -2;
    uint64_t e = 0;
    for (uint32_t a = 0; a <= d; a++)
        for (uint32_t b = a + 1; b <= d; b++) {
            src[e] = a; dst[e] = b; ep[2 * e] = a; ep[2 * e + 1] = b; e++;
        }
    uint32_t *pick = (uint32_t *)malloc(d * sizeof(uint32_t));
    for (uint32_t v = d + 1; v < n; v++) {
        uint64_t pool = 2 * e; /* endpoints present before v attaches */
        uint32_t got = 0;
        while (got < d) {
            uint32_t t = ep[below(&st, pool)];
            int dup = 0;
            for (uint32_t q = 0; q < got; q++) if (pick[q] == t) { dup = 1; break; }
            if (!dup) pick[got++] = t;
        }
        for (uint32_t q = 0; q < d; q++) {
            src[e] = v; dst[e] = pick[q]; ep[2 * e] = v; ep[2 * e + 1] = pick[q]; e++;
        }
    }
    free(pick);
    free(ep);
    shuffle_ids(n, total, src, dst, &st);
    return 0;
}

int gen_rmat(uint32_t scale, uint64_t m, double a, double b, double c, uint64_t seed,
             uint32_t *src, uint32_t *dst) {
    if (scale < 1 || scale > 31) return -1;
    uint64_t n = 1ULL << scale;
    if (m > n * (n - 1) / 2) return -1;
    uint64_t st = seed;
    pairset ps;
    if (ps_init(&ps, m)) return -2;
    double ab = a + b, abc = a + b + c;
    uint64_t e = 0;
    while (e < m) {
        uint32_t r = 0, q = 0;
        for (uint32_t lev = 0; lev < scale; lev++) {
            double x = unit(&st);
            uint32_t bit = 1u << (scale - 1 - lev);
            if (x < a) { }
            else if (x < ab) q |= bit;
            else if (x < abc) r |= bit;
            else { r |= bit; q |= bit; }
        }
        if (r == q) continue;
        uint32_t lo = r < q ? r : q, hi = r < q ? q : r;
        if (!ps_insert(&ps, ((uint64_t)lo << 32) | hi)) continue;
        src[e] = lo; dst[e] = hi; e++;
    }
    ps_free(&ps);
    shuffle_ids((uint32_t)n, m, src, dst, &st);
    return 0;
}

/* ------------------------------------------------------------- labels */
void gen_labels_uniform(uint64_t n, uint32_t nl, uint64_t seed, uint32_t *out) {
    uint64_t st = seed;
    for (uint64_t i = 0; i < n; i++) out[i] = (uint32_t)below(&st, nl);
}

/* P(label = i) proportional to (i+1)^-s, sampled by inverse CDF. */
void gen_labels_zipf(uint64_t n, uint32_t nl, double s, uint64_t seed, uint32_t *out) {
    uint64_t st = seed;
    double *cdf = (double *)malloc(nl * sizeof(double));
    double acc = 0.0;
    for (uint32_t i = 0; i < nl; i++) {
        double w = pow((double)(i + 1), -s);
        acc += w;
        cdf[i] = acc;
    }
    for (uint32_t i = 0; i < nl; i++) cdf[i] /= acc;
    cdf[nl - 1] = 1.0;
    for (uint64_t i = 0; i < n; i++) {
        double x = unit(&st);
        uint32_t lo = 0, hi = nl - 1;
        while (lo < hi) { uint32_t mid = (lo + hi) / 2; if (cdf[mid] > x) hi = mid; else lo = mid + 1; }
        out[i] = lo;
    }
    free(cdf);
}

/* ------------------------------------------------------------ queries */
typedef struct {
    uint32_t n;
    uint64_t *rp;      /* n+1 */
    uint32_t *nb;      /* sorted neighbour ids per row */
    uint32_t *nl;      /* edge label, parallel to nb */
    const uint32_t *vlabel;
    uint32_t *nonisolated;
    uint32_t n_noniso;
} qctx;

static int cmp_pair(const void *x, const void *y) {
    const uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
    return a < b ? -1 : a > b;
}

void *gen_qctx_create(uint32_t n, const uint32_t *vlabel, uint64_t m, const uint32_t *src,
                      const uint32_t *dst, const uint32_t *elabel) {
    qctx *q = (qctx *)calloc(1, sizeof(qctx));
    q->n = n;
    q->vlabel = vlabel;
    q->rp = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    for (uint64_t e = 0; e < m; e++) { q->rp[src[e] + 1]++; q->rp[dst[e] + 1]++; }
    for (uint32_t v = 0; v < n; v++) q->rp[v + 1] += q->rp[v];
    uint64_t *cur = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    memcpy(cur, q->rp, (size_t)n * sizeof(uint64_t));
    /* pack (neighbour << 32 | label) so one sort orders by neighbour id */
    uint64_t *pk = (uint64_t *)malloc(2 * m * sizeof(uint64_t));
    for (uint64_t e = 0; e < m; e++) {
        pk[cur[src[e]]++] = ((uint64_t)dst[e] << 32) | elabel[e];
        pk[cur[dst[e]]++] = ((uint64_t)src[e] << 32) | elabel[e];
    }
    free(cur);
    q->nb = (uint32_t *)malloc(2 * m * sizeof(uint32_t) + 4);
    q->nl = (uint32_t *)malloc(2 * m * sizeof(uint32_t) + 4);
    uint32_t cnt = 0;
    q->nonisolated = (uint32_t *)malloc((size_t)n * sizeof(uint32_t) + 4);
    for (uint32_t v = 0; v < n; v++) {
        uint64_t a = q->rp[v], b = q->rp[v + 1];
        if (b > a + 1) qsort(pk + a, b - a, sizeof(uint64_t), cmp_pair);
        for (uint64_t i = a; i < b; i++) { q->nb[i] = (uint32_t)(pk[i] >> 32); q->nl[i] = (uint32_t)pk[i]; }
        if (b > a) q->nonisolated[cnt++] = v;
    }
    q->n_noniso = cnt;
    free(pk);
    return q;
}

void gen_qctx_free(void *p) {
    qctx *q = (qctx *)p;
    if (!q) return;
    free(q->rp); free(q->nb); free(q->nl); free(q->nonisolated); free(q);
}

/* label of edge (a,b) or -1 */
static int64_t edge_label(const qctx *q, uint32_t a, uint32_t b) {
    uint64_t lo = q->rp[a], hi = q->rp[a + 1];
    while (lo < hi) {
        uint64_t mid = (lo + hi) / 2;
        if (q->nb[mid] < b) lo = mid + 1; else hi = mid;
    }
    if (lo < q->rp[a + 1] && q->nb[lo] == b) return q->nl[lo];
    return -1;
}

/*
 * mode 0 = walk (all traversed edges), 1 = tree (first-visit edges only),
 * 2 = dense (every data edge among the visited vertices),
 * 3 = walk with cycle: the traversed edges plus the first data edge among the
 *     visited vertices that the walk did not traverse (pairs in first-visit
 *     order), so the query holds a cycle; redrawn if there is no such edge.
 * Outputs: qlabel[k], edges (qsrc,qdst,qel) with capacity k*(k-1)/2,
 * source[k] = the data vertices visited (an embedding of the query).
 * Returns the number of query edges, or -1 if no walk reached k vertices.
 */
int64_t gen_query(void *p, uint32_t k, int mode, uint64_t seed, uint32_t *qlabel, uint32_t *qsrc,
                  uint32_t *qdst, uint32_t *qel, uint32_t *source) {
    qctx *q = (qctx *)p;
    uint64_t st = seed;
    if (k < 1 || q->n_noniso == 0) return -1;
    uint32_t *vis = source;
    uint8_t *adj = (uint8_t *)calloc((size_t)k * k, 1);
    for (int attempt = 0; attempt < 1000; attempt++) {
        memset(adj, 0, (size_t)k * k);
        uint32_t nv = 1;
        uint32_t cur = q->nonisolated[below(&st, q->n_noniso)];
        vis[0] = cur;
        uint32_t curq = 0;
        uint64_t steps = 0, limit = 100ULL * k;
        while (nv < k && steps < limit) {
            uint64_t a = q->rp[cur], deg = q->rp[cur + 1] - a;
            uint64_t pick = a + below(&st, deg);
            uint32_t nxt = q->nb[pick];
            steps++;
            uint32_t nq = nv;
            for (uint32_t i = 0; i < nv; i++) if (vis[i] == nxt) { nq = i; break; }
            int first = (nq == nv);
            if (first) { vis[nv] = nxt; nv++; }
            if (mode != 1 || first) { adj[curq * k + nq] = 1; adj[nq * k + curq] = 1; }
            cur = nxt; curq = nq;
        }
        if (nv < k) continue;
        if (mode == 2) {
            for (uint32_t i = 0; i < k; i++)
                for (uint32_t j = i + 1; j < k; j++)
                    if (edge_label(q, vis[i], vis[j]) >= 0) { adj[i * k + j] = 1; adj[j * k + i] = 1; }
        }
        if (mode == 3) {
            int added = 0;
            for (uint32_t i = 0; i < k && !added; i++)
                for (uint32_t j = i + 1; j < k && !added; j++)
                    if (!adj[i * k + j] && edge_label(q, vis[i], vis[j]) >= 0) {
                        adj[i * k + j] = 1; adj[j * k + i] = 1; added = 1;
                    }
            if (!added) continue;
        }
        uint32_t ne = 0;
        for (uint32_t i = 0; i < k; i++)
            for (uint32_t j = i + 1; j < k; j++)
                if (adj[i * k + j]) {
                    qsrc[ne] = i; qdst[ne] = j; qel[ne] = (uint32_t)edge_label(q, vis[i], vis[j]); ne++;
                }
        for (uint32_t i = 0; i < k; i++) qlabel[i] = q->vlabel[vis[i]];
        free(adj);
        return ne;
    }
    free(adj);
    return -1;
}
