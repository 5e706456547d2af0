// One query: signature filter (Sec. III-A), matching order (Algorithm 2) and
// the vertex-at-a-time Prealloc-Combine join (Sec. V, Algorithms 3-4).
//
// Intermediate tables are column-major (column c of M at M + c*R): the link
// step then writes every column of M' with fully coalesced stores and the
// join reads one column of a row without touching the others.  The last
// level writes rows in query-vertex order.
//
// Join level j, for the next query vertex u with linking edges ES:
//   k_locate  one thread per row i: locate N(v,l) in PCSR for every e in ES
//             (home group, probe the 15 keys of its 128-byte group, follow GID);
//             bound_i = |N(v'_i, l0)| for the first edge e0 (Algorithm 4)
//   scan      F = exclusive prefix sum of bound; |GBA| = F[R]
//   k_join    the element index space [0, |GBA|) is cut into tiles of 256
//             (one element per lane): the element at p belongs to the row i
//             with F[i] <= p < F[i+1] and is x = N(v'_i, l0)[p - F[i]]; it is
//             kept iff x is not in m_i (set subtraction), x is in C(u) (one
//             bitset probe) and x is in every other linking list (binary
//             search in the sorted list).  The tile's keep flags are written
//             as one 64-bit ballot word per wave: GBA holds one bit per
//             pre-allocated slot instead of a vertex id, so the join writes
//             |GBA|/8 bytes, coalesced.
//   scan      tile survivor counts -> tile offsets; |M'| = total
//   k_link    every kept slot re-reads its x and writes (m_i, x) at its
//             position in M' (order: parent row, then ascending x).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>

#include "gsi_internal.h"
#include "fused.h"
#include "join_device.h"
#include "level.h"
#include "scan_device.h"

namespace gsi {

constexpr uint32_t QT = 256;  // threads per workgroup (4 waves)

static uint32_t nblocks(uint64_t n, uint64_t per = QT) {
    uint64_t b = (n + per - 1) / per;
    if (b == 0) b = 1;
    if (b > 0x7FFFFFFFull) fail(GSI_E_CAPACITY, "grid of %llu workgroups exceeds the launch limit",
                                (unsigned long long)b);
    return (uint32_t)b;
}

// ------------------------------------------------------------ validation
HostQuery validate_query(uint32_t k, const uint32_t *vl, uint32_t qm, const uint32_t *s, const uint32_t *d,
                         const uint32_t *l) {
    if (k < 1 || k > GSI_MAX_K) fail(GSI_E_INVALID, "query must have 1..%d vertices", GSI_MAX_K);
    if (!vl) fail(GSI_E_INVALID, "null query labels");
    if (qm && (!s || !d || !l)) fail(GSI_E_INVALID, "null query edge array");
    if (qm > (uint32_t)k * (k - 1) / 2) fail(GSI_E_INVALID, "too many query edges for a simple graph");
    HostQuery q;
    q.k = k;
    q.vl.assign(vl, vl + k);
    q.adj.assign(k, {});
    std::vector<uint8_t> seen((size_t)k * k, 0);
    for (uint32_t e = 0; e < qm; e++) {
        uint32_t a = s[e], b = d[e];
        if (a >= k || b >= k) fail(GSI_E_INVALID, "query edge %u has an endpoint >= k", e);
        if (a == b) fail(GSI_E_INVALID, "query edge %u is a self-loop", e);
        if (seen[(size_t)a * k + b]) fail(GSI_E_INVALID, "query edge %u repeats a vertex pair", e);
        seen[(size_t)a * k + b] = seen[(size_t)b * k + a] = 1;
        q.src.push_back(a);
        q.dst.push_back(b);
        q.el.push_back(l[e]);
        q.adj[a].push_back({b, l[e]});
        q.adj[b].push_back({a, l[e]});
    }
    std::vector<uint8_t> vis(k, 0);
    std::vector<uint32_t> st{0};
    vis[0] = 1;
    uint32_t reached = 1;
    while (!st.empty()) {
        uint32_t x = st.back();
        st.pop_back();
        for (auto &p : q.adj[x])
            if (!vis[p.first]) {
                vis[p.first] = 1;
                reached++;
                st.push_back(p.first);
            }
    }
    if (reached != k) fail(GSI_E_INVALID, "query graph is not connected");
    return q;
}

// Multi-label query (Sec. VII-B): label sets per vertex; a vertex pair may
// carry several edges, one per label (the same pair and label twice is
// rejected); Q connected.
HostQuery validate_query_multi(uint32_t k, const uint32_t *off, const uint32_t *lab, uint32_t qm, const uint32_t *s,
                               const uint32_t *d, const uint32_t *l) {
    if (k == 0 || k > GSI_MAX_K) fail(GSI_E_INVALID, "k must be in [1, %u]", (unsigned)GSI_MAX_K);
    if (!off || !lab) fail(GSI_E_INVALID, "null query label sets");
    if (qm && (!s || !d || !l)) fail(GSI_E_INVALID, "null query edge array");
    if (off[0] != 0 || off[k] > MULTI_MAX_QUERY_LABELS)
        fail(GSI_E_INVALID, "label offsets must start at 0 and hold at most %u labels", MULTI_MAX_QUERY_LABELS);
    if (qm > 8u * k * (k - 1) / 2) fail(GSI_E_INVALID, "more than 8 labelled edges per query vertex pair");
    HostQuery q;
    q.k = k;
    q.multi = true;
    q.vl.assign(k, 0);
    q.vls.assign(k, {});
    for (uint32_t u = 0; u < k; u++) {
        if (off[u + 1] < off[u]) fail(GSI_E_INVALID, "label offsets must not decrease");
        std::vector<uint32_t> ls(lab + off[u], lab + off[u + 1]);
        std::sort(ls.begin(), ls.end());
        ls.erase(std::unique(ls.begin(), ls.end()), ls.end());
        q.vls[u] = ls;
        q.vl[u] = ls.empty() ? 0u : ls[0];
    }
    q.adj.assign(k, {});
    std::vector<uint8_t> linked((size_t)k * k, 0);
    for (uint32_t e = 0; e < qm; e++) {
        uint32_t a = s[e], b = d[e];
        if (a >= k || b >= k) fail(GSI_E_INVALID, "query edge %u has an endpoint >= k", e);
        if (a == b) fail(GSI_E_INVALID, "query edge %u is a self-loop", e);
        for (auto &p : q.adj[a])
            if (p.first == b && p.second == l[e]) fail(GSI_E_INVALID, "query edge %u repeats a labelled edge", e);
        q.src.push_back(a);
        q.dst.push_back(b);
        q.el.push_back(l[e]);
        q.adj[a].push_back({b, l[e]});
        q.adj[b].push_back({a, l[e]});
        linked[(size_t)a * k + b] = linked[(size_t)b * k + a] = 1;
    }
    std::vector<uint8_t> vis(k, 0);
    std::vector<uint32_t> st{0};
    vis[0] = 1;
    uint32_t reached = 1;
    while (!st.empty()) {
        uint32_t x = st.back();
        st.pop_back();
        for (uint32_t y = 0; y < k; y++)
            if (linked[(size_t)x * k + y] && !vis[y]) {
                vis[y] = 1;
                reached++;
                st.push_back(y);
            }
    }
    if (reached != k) fail(GSI_E_INVALID, "query graph is not connected");
    return q;
}

void make_multi(HostQuery &q) {
    if (q.multi) return;
    q.multi = true;
    q.vls.assign(q.k, {});
    for (uint32_t u = 0; u < q.k; u++) q.vls[u] = {q.vl[u]};
}

// ------------------------------------------------------------------ filter
struct FilterArgs {
    uint32_t k;
    uint32_t label_only;
    uint32_t subset0;              // word 0: containment (multi-label) instead of equality
    uint32_t word_mask;            // bit i set when some query vertex has bits in word i
    uint32_t dst[GSI_MAX_K];       // bitset row / count slot of query vertex u
    uint32_t q[GSI_MAX_K][GSI_SIG_WORDS];
};

// Query signatures with the same encoding as the data table (Sec. III-A).
// Under homomorphism two query neighbours with one (edge label, vertex
// label) key may map to one data neighbour, so a group asks for one
// neighbour at most (code 01): the "two or more" code would not be sound.
static void query_signatures(const HostQuery &q, FilterArgs &fa, bool homo = false) {
    memset(&fa, 0, sizeof(fa));
    fa.k = q.k;
    for (uint32_t u = 0; u < q.k; u++) {
        fa.dst[u] = u;
        uint32_t cnt[SIG_GROUPS] = {0};
        if (q.multi) {
            // every label of u in word 0; a neighbour contributes the pair
            // (edge label, x) for each of its labels x
            fa.subset0 = 1;
            for (uint32_t x : q.vls[u]) fa.q[u][0] |= label_bit(x);
            for (auto &p : q.adj[u])
                for (uint32_t x : q.vls[p.first]) cnt[sig_group(p.second, x)]++;
        } else {
            fa.q[u][0] = q.vl[u];
            for (auto &p : q.adj[u]) cnt[sig_group(p.second, q.vl[p.first])]++;
        }
        for (uint32_t g = 0; g < SIG_GROUPS; g++)
            if (cnt[g]) fa.q[u][1 + g / 16] |= (cnt[g] == 1 || homo ? 1u : 3u) << (2 * (g % 16));
        for (int i = 1; i < GSI_SIG_WORDS; i++)
            if (fa.q[u][i]) fa.word_mask |= 1u << i;
    }
}

// The filter for one query.  A workgroup takes FILTER_TILES tiles of 256
// data vertices; a lane owns one data vertex of each and reads their labels
// and every signature word some query vertex uses, all in one batch of
// loads (a wave reads word i of 64 consecutive vertices in one 256-byte
// access; since 32 vertices share a 128-byte line, skipping the words of
// vertices whose label matches no query vertex would save no traffic, only
// add a second round trip).  The words are kept complemented, so the bits
// of query word q that the vertex lacks are (~w & q), one and-or per word.
// The wave's ballot of "v in C(u)" is the bitset word of its 64 vertices;
// lane u stores the word of query vertex u, so one store instruction
// writes them all.  One tile per workgroup: on an 8.4M-vertex table with
// every word in use the launch takes 118 us (4.6 TB/s), 133 us with four
// tiles (fewer workgroups in flight, more registers each).
constexpr uint32_t FILTER_TILES = 1;

__global__ __launch_bounds__(QT) void k_filter(const uint32_t *sig, uint32_t n, uint64_t nwords, FilterArgs fa,
                                              uint64_t *bits) {
    const uint32_t need = fa.label_only ? 0u : fa.word_mask;
    const uint32_t K = fa.k;
    const uint32_t lane = lane_id();
    uint32_t w0[FILTER_TILES], nw[FILTER_TILES][GSI_SIG_WORDS];
    // Every load is issued unconditionally (a word no query vertex uses, or
    // a lane past n, re-reads a valid word-0 address, a cache hit) and only
    // then masked: branching around a load makes it wait for the one before.
#pragma unroll
    for (uint32_t r = 0; r < FILTER_TILES; r++) {
        const uint64_t v = ((uint64_t)blockIdx.x * FILTER_TILES + r) * QT + threadIdx.x;
        const uint64_t vv = v < n ? v : (uint64_t)n - 1;
        w0[r] = sig[vv];
#pragma unroll
        for (int i = 1; i < GSI_SIG_WORDS; i++) nw[r][i] = sig[((need >> i) & 1u) ? (uint64_t)i * n + vv : vv];
    }
#pragma unroll
    for (uint32_t r = 0; r < FILTER_TILES; r++) {
        const bool valid = ((uint64_t)blockIdx.x * FILTER_TILES + r) * QT + threadIdx.x < n;
        if (!valid) w0[r] = NONE32;
#pragma unroll
        for (int i = 1; i < GSI_SIG_WORDS; i++) nw[r][i] = (((need >> i) & 1u) && valid) ? ~nw[r][i] : 0u;
    }
#pragma unroll
    for (uint32_t r = 0; r < FILTER_TILES; r++) {
        const uint64_t tile = (uint64_t)blockIdx.x * FILTER_TILES + r;
        const bool valid = tile * QT + threadIdx.x < n;
        uint32_t ok = 0;
        for (uint32_t u = 0; u < K; u++) {
            const bool lab_ok = valid && (fa.subset0 ? (~w0[r] & fa.q[u][0]) == 0 : w0[r] == fa.q[u][0]);
            // the word tests are most of the kernel's vector work: a wave
            // none of whose vertices has u's label skips them (uniform)
            if (__ballot(lab_ok) == 0) continue;
            uint32_t miss = 0;
#pragma unroll
            for (int i = 1; i < GSI_SIG_WORDS; i++) miss |= nw[r][i] & fa.q[u][i];
            ok |= (lab_ok && miss == 0) ? (1u << u) : 0u;
        }
        uint64_t mine = 0;
        for (uint32_t u = 0; u < K; u++) {
            const uint64_t m = __ballot((ok >> u) & 1u);
            if (lane == u) mine = m;
        }
        const uint64_t wave_first = tile * QT + (threadIdx.x & ~63u);
        if (lane < K && wave_first < n) bits[(uint64_t)fa.dst[lane] * nwords + (wave_first >> 6)] = mine;
    }
}

// counts[r] = set bits of bitset row r (one 1024-thread workgroup per row);
// wave w counts run w of the row's words (BITS_RUNS runs of equal length)
// and, with `runs`, writes that count to runs[r * BITS_RUNS + w]
__global__ __launch_bounds__(1024) void k_bit_counts(const uint64_t *bits, uint64_t nwords, uint32_t *counts,
                                                    uint32_t *runs) {
    static_assert(BITS_RUNS == 1024 / 64, "one run per wave");
    __shared__ uint32_t s_w[16];
    const uint64_t *row = bits + (uint64_t)blockIdx.x * nwords;
    const uint32_t wv = threadIdx.x >> 6;
    const uint64_t per = (nwords + BITS_RUNS - 1) / BITS_RUNS;
    const uint64_t ws = per * wv < nwords ? per * wv : nwords;
    const uint64_t we = ws + per < nwords ? ws + per : nwords;
    uint32_t sum = 0;
    uint64_t q = ws + lane_id();
    for (; q + 192 < we; q += 256)
        sum += (uint32_t)(__popcll(row[q]) + __popcll(row[q + 64]) + __popcll(row[q + 128]) + __popcll(row[q + 192]));
    for (; q < we; q += 64) sum += (uint32_t)__popcll(row[q]);
    sum = wave_sum(sum);
    if (lane_id() == 0 && runs) runs[(uint64_t)blockIdx.x * BITS_RUNS + wv] = sum;
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < 16; w++) t += s_w[w];
        counts[blockIdx.x] = t;
    }
}

// Multi-labelled graphs (Sec. VII-B): the signature test lets through the
// vertices whose hashed label bits contain u's; each candidate v of C(u)
// then stays only if its label set contains u's (both ascending).  One
// thread per (query vertex, bitset word).
struct RefineArgs {
    uint32_t k;
    uint32_t dst[GSI_MAX_K];
    uint32_t off[GSI_MAX_K + 1];
    uint32_t lab[MULTI_MAX_QUERY_LABELS];
};

__global__ __launch_bounds__(QT) void k_label_refine(uint64_t *bits, uint64_t nwords, const uint32_t *voff,
                                                    const uint32_t *vlab, RefineArgs ra) {
    const uint64_t w = (uint64_t)blockIdx.x * QT + threadIdx.x;
    const uint32_t u = blockIdx.y;
    if (w >= nwords) return;
    uint64_t *word = bits + (uint64_t)ra.dst[u] * nwords + w;
    uint64_t b = *word, keep = b;
    while (b) {
        const uint32_t t = (uint32_t)__ffsll((unsigned long long)b) - 1;
        b &= b - 1;
        const uint32_t v = (uint32_t)(w * 64 + t);
        uint32_t j = voff[v];
        const uint32_t je = voff[v + 1];
        bool ok = true;
        for (uint32_t i = ra.off[u]; ok && i < ra.off[u + 1]; i++) {
            while (j < je && vlab[j] < ra.lab[i]) j++;
            ok = j < je && vlab[j] == ra.lab[i];
        }
        if (!ok) keep &= ~(1ull << t);
    }
    if (keep != *word) *word = keep;
}

static void launch_filter(gsi_ctx *c, gsi_graph *g, const FilterArgs &fa, uint64_t *bits, uint32_t *counts,
                          uint32_t *runs, const HostQuery *mq = nullptr) {
    const uint64_t nwords = ((uint64_t)g->n + 63) / 64;
    const uint32_t nb = nblocks(g->n);
    const uint32_t need = fa.label_only ? 0u : fa.word_mask;
    double bytes = 4.0 * g->n * (1 + __builtin_popcount(need)) + (double)fa.k * nwords * 8;
    const uint32_t nfb = (nb + FILTER_TILES - 1) / FILTER_TILES;
    launch(c, "k_filter", bytes, k_filter, nfb, QT, (const uint32_t *)g->sig, g->n, nwords, fa, bits);
    if (g->multi && mq) {
        RefineArgs ra;
        memset(&ra, 0, sizeof(ra));
        ra.k = fa.k;
        uint32_t o = 0;
        for (uint32_t u = 0; u < fa.k; u++) {
            ra.dst[u] = fa.dst[u];
            ra.off[u] = o;
            for (uint32_t x : mq->vls[u]) ra.lab[o++] = x;
        }
        ra.off[fa.k] = o;
        launch(c, "k_label_refine", 16.0 * fa.k * nwords, k_label_refine, dim3(nblocks(nwords), fa.k), QT, bits,
               nwords, (const uint32_t *)g->vl_off, (const uint32_t *)g->vl_lab, ra);
    }
    launch(c, "k_filter_counts", 8.0 * fa.k * nwords, k_bit_counts, fa.k, 1024, (const uint64_t *)bits, nwords,
           counts, runs);
}

// Batched filter: the query vertices of many queries, 32 per pass, all
// passes in one launch (blockIdx.y = pass; workgroups stride over rounds of
// FM_TILE data vertices).  A pass takes query vertices sorted by label, so
// its vertices form a few groups of one label each.  A round first finds,
// per data vertex, the group of its label (most vertices have none), and
// compacts the vertices that have one into a list in LDS; the signature
// test then runs on that list in dense waves, each thread testing its
// vertex against the query vertices of its group only (testing in place,
// a wave would run the test of every query vertex its lanes match for the
// few lanes that match).  Passing pairs set bits of the round's bitset
// words in LDS, which are then written out one 128-byte line per query
// vertex.  Each workgroup keeps per query vertex counts in LDS and writes
// them to part[(pass * 32 + u) * gridDim.x + workgroup].
constexpr uint32_t FM_TILE = 1024;

__global__ __launch_bounds__(QT) void k_filter_multi(const uint32_t *sig, uint32_t n, uint64_t nwords,
                                                    const FilterArgs *__restrict__ passes, uint64_t *bits,
                                                    uint32_t *part) {
    constexpr uint32_t TW = FM_TILE / 64;  // bitset words per round
    const FilterArgs &fa = passes[blockIdx.y];
    __shared__ uint32_t s_q[GSI_MAX_K][GSI_SIG_WORDS];
    __shared__ uint32_t s_dst[GSI_MAX_K];
    __shared__ uint32_t s_cnt[GSI_MAX_K];
    __shared__ uint32_t s_glab[GSI_MAX_K];      // label of group g
    __shared__ uint32_t s_gbeg[GSI_MAX_K + 1];  // its query vertices: s_gbeg[g] .. s_gbeg[g+1]-1
    __shared__ uint32_t s_ng, s_n;
    __shared__ uint64_t s_res[GSI_MAX_K][TW];   // the round's bitset words
    __shared__ uint16_t s_v[FM_TILE];           // vertices with a group (offset in the round)
    __shared__ uint8_t s_g[FM_TILE];            // and their groups
    const uint32_t K = fa.k;
    const uint32_t need = fa.word_mask;
    for (uint32_t t = threadIdx.x; t < K * GSI_SIG_WORDS; t += QT)
        s_q[t / GSI_SIG_WORDS][t % GSI_SIG_WORDS] = fa.q[t / GSI_SIG_WORDS][t % GSI_SIG_WORDS];
    for (uint32_t t = threadIdx.x; t < GSI_MAX_K * TW; t += QT) s_res[t / TW][t % TW] = 0;
    if (threadIdx.x < GSI_MAX_K) {
        s_cnt[threadIdx.x] = 0;
        s_dst[threadIdx.x] = threadIdx.x < K ? fa.dst[threadIdx.x] : 0u;
    }
    if (threadIdx.x == 0) {
        uint32_t ng = 0;
        for (uint32_t u = 0; u < K; u++) {
            if (u == 0 || fa.q[u][0] != fa.q[u - 1][0]) {
                s_glab[ng] = fa.q[u][0];
                s_gbeg[ng] = u;
                ng++;
            }
        }
        s_gbeg[ng] = K;
        s_ng = ng;
        s_n = 0;
    }
    __syncthreads();
    const uint32_t ng = __builtin_amdgcn_readfirstlane(s_ng);
    const uint32_t lane = lane_id();
    const uint64_t nrounds = ((uint64_t)n + FM_TILE - 1) / FM_TILE;
    for (uint64_t round = blockIdx.x; round < nrounds; round += gridDim.x) {
        const uint64_t v0 = round * FM_TILE;
        // labels of the round's vertices (all loads first), their groups
        uint32_t w0[FM_TILE / QT];
#pragma unroll
        for (uint32_t r = 0; r < FM_TILE / QT; r++) {
            const uint64_t v = v0 + r * QT + threadIdx.x;
            w0[r] = sig[v < n ? v : (uint64_t)n - 1];
            if (v >= n) w0[r] = NONE32;
        }
#pragma unroll
        for (uint32_t r = 0; r < FM_TILE / QT; r++) {
            // (groups are runs of equal labels: the host sorts by label)
            uint32_t gi = NONE32;
            for (uint32_t g = 0; g < ng; g++)
                if (w0[r] == s_glab[g]) gi = g;
            const bool has = gi != NONE32 && v0 + r * QT + threadIdx.x < n;
            const uint64_t mask = __ballot(has);
            if (mask) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(&s_n, (uint32_t)__popcll(mask));
                base = __shfl(base, 0, 64);
                if (has) {
                    const uint32_t idx = base + rank_below(mask);
                    s_v[idx] = (uint16_t)(r * QT + threadIdx.x);
                    s_g[idx] = (uint8_t)gi;
                }
            }
        }
        __syncthreads();
        // signature test of the listed vertices against their groups
        const uint32_t nm = __builtin_amdgcn_readfirstlane(s_n);
        for (uint32_t e = threadIdx.x; e < nm; e += QT) {
            const uint32_t off = s_v[e], gi = s_g[e];
            const uint64_t v = v0 + off;
            // complemented words: a query word's bits missing from the
            // vertex's are then (~w & q), one and-or per word, with no
            // per-word branch or mask arithmetic; words no query vertex of
            // the pass uses are zero in every query signature
            // (every load issued unconditionally, an unused word re-reading
            // word 0 of the vertex, then masked: a load behind a branch
            // waits for the one before)
            uint32_t nw[GSI_SIG_WORDS];
#pragma unroll
            for (int i = 1; i < GSI_SIG_WORDS; i++) nw[i] = sig[((need >> i) & 1u) ? (uint64_t)i * n + v : v];
#pragma unroll
            for (int i = 1; i < GSI_SIG_WORDS; i++) nw[i] = ((need >> i) & 1u) ? ~nw[i] : 0u;
            const uint32_t ue = s_gbeg[gi + 1];
            for (uint32_t u = s_gbeg[gi]; u < ue; u++) {
                uint32_t miss = 0;
#pragma unroll
                for (int i = 1; i < GSI_SIG_WORDS; i++) miss |= nw[i] & s_q[u][i];
                if (miss == 0) atomicOr(&s_res[u][off >> 6], 1ull << (off & 63));
            }
        }
        __syncthreads();
        // the round's words of every query vertex of the pass, then cleared
        const uint64_t wbase = round * TW;
        for (uint32_t t = threadIdx.x; t < K * TW; t += QT) {
            const uint32_t u = t / TW, q = t % TW;
            const uint64_t word = s_res[u][q];
            if (wbase + q < nwords) bits[(uint64_t)s_dst[u] * nwords + wbase + q] = word;
            if (word) atomicAdd(&s_cnt[u], (uint32_t)__popcll(word));
            s_res[u][q] = 0;
        }
        if (threadIdx.x == 0) s_n = 0;
        __syncthreads();
    }
    if (threadIdx.x < GSI_MAX_K)
        part[((uint64_t)blockIdx.y * GSI_MAX_K + threadIdx.x) * gridDim.x + blockIdx.x] = s_cnt[threadIdx.x];
}

// counts of every pass: workgroup (u, pass) sums u's partial counts
__global__ __launch_bounds__(QT) void k_filter_counts_multi(const uint32_t *part, uint32_t nb,
                                                           const FilterArgs *passes, uint32_t *counts) {
    __shared__ uint32_t s_w[QT / 64];
    const uint32_t u = blockIdx.x, pass = blockIdx.y;
    const FilterArgs &fa = passes[pass];
    if (u >= fa.k) return;
    const uint32_t *row = part + ((uint64_t)pass * GSI_MAX_K + u) * nb;
    uint32_t sum = 0;
    for (uint32_t b = threadIdx.x; b < nb; b += QT) sum += row[b];
    sum = wave_sum(sum);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int q = 0; q < QT / 64; q++) t += s_w[q];
        counts[fa.dst[u]] = t;
    }
}

void run_filter_many(gsi_graph *g, const std::vector<const HostQuery *> &qs, const std::vector<uint32_t> &qbase,
                     uint64_t *bits, uint32_t *counts) {
    gsi_ctx *c = g->ctx;
    struct QV {
        uint32_t label, q, u;
    };
    std::vector<QV> all;
    for (size_t i = 0; i < qs.size(); i++)
        for (uint32_t u = 0; u < qs[i]->k; u++) all.push_back({qs[i]->vl[u], (uint32_t)i, u});
    if (all.empty()) return;
    std::stable_sort(all.begin(), all.end(), [](const QV &a, const QV &b) { return a.label < b.label; });
    std::vector<FilterArgs> one(qs.size());
    for (size_t i = 0; i < qs.size(); i++) query_signatures(*qs[i], one[i]);
    const uint32_t npass = (uint32_t)((all.size() + GSI_MAX_K - 1) / GSI_MAX_K);
    if (npass > 65535) fail(GSI_E_CAPACITY, "too many query vertices in one batch (%zu)", all.size());
    std::vector<FilterArgs> passes(npass);
    uint32_t words = 0;
    for (uint32_t p = 0; p < npass; p++) {
        FilterArgs &fa = passes[p];
        memset(&fa, 0, sizeof(fa));
        const size_t base = (size_t)p * GSI_MAX_K;
        const uint32_t k = (uint32_t)std::min<size_t>(GSI_MAX_K, all.size() - base);
        fa.k = k;
        for (uint32_t t = 0; t < k; t++) {
            const QV &x = all[base + t];
            fa.dst[t] = qbase[x.q] + x.u;
            memcpy(fa.q[t], one[x.q].q[x.u], sizeof(fa.q[t]));
            for (int i = 1; i < GSI_SIG_WORDS; i++)
                if (fa.q[t][i]) fa.word_mask |= 1u << i;
        }
        words += 1 + __builtin_popcount(fa.word_mask);
    }
    Scratch s(c);
    const uint64_t nwords = ((uint64_t)g->n + 63) / 64;
    // workgroups per pass: enough to fill the chip when passes are few
    const uint32_t nrounds = (uint32_t)(((uint64_t)g->n + FM_TILE - 1) / FM_TILE);
    const uint32_t nb = std::max<uint32_t>(1, std::min<uint32_t>(nrounds, std::max<uint32_t>(32, 8192 / npass)));
    FilterArgs *dp = reinterpret_cast<FilterArgs *>(s.get<uint32_t>((uint64_t)npass * sizeof(FilterArgs) / 4,
                                                                    "filter passes"));
    uint32_t *part = s.get<uint32_t>((uint64_t)npass * GSI_MAX_K * nb, "filter partial counts");
    GSI_HIP(hipMemcpyAsync(dp, passes.data(), sizeof(FilterArgs) * npass, hipMemcpyHostToDevice, c->stream));
    const double bytes = 4.0 * g->n * words + (double)all.size() * nwords * 8;
    launch(c, "k_filter", bytes, k_filter_multi, dim3(nb, npass), QT, (const uint32_t *)g->sig, g->n, nwords,
           (const FilterArgs *)dp, bits, part);
    launch(c, "k_filter_counts", 4.0 * nb * all.size(), k_filter_counts_multi, dim3(GSI_MAX_K, npass), QT,
           (const uint32_t *)part, nb, (const FilterArgs *)dp, counts);
    sync(c);  // `passes` is read by the copy above
}

// The single-query filter through the grouped kernel (k_filter_multi, one
// pass): a round's vertices whose label some query vertex has are listed in
// LDS and tested against the query vertices of that label only.  Counts and
// per-run counts come from the bitsets (k_bit_counts), as in launch_filter.
constexpr bool GROUPED_SINGLE_FILTER = true;
constexpr size_t PINNED_FILTER_ARGS = 5120;  // staging offset in c->pinned (status region, past the chunk summary)
static void launch_filter_grouped(gsi_ctx *c, gsi_graph *g, const FilterArgs &f, uint64_t *bits, uint32_t *counts,
                                  uint32_t *runs) {
    static_assert(PINNED_FILTER_ARGS >= 4096 + sizeof(FChunkSummary) &&
                      PINNED_FILTER_ARGS + sizeof(FilterArgs) <= 8192,
                  "filter arguments between the chunk summary and the plans");
    FilterArgs *fa = reinterpret_cast<FilterArgs *>(reinterpret_cast<char *>(c->pinned) + PINNED_FILTER_ARGS);
    uint32_t idx[GSI_MAX_K];
    for (uint32_t u = 0; u < f.k; u++) idx[u] = u;
    std::stable_sort(idx, idx + f.k, [&](uint32_t x, uint32_t y) { return f.q[x][0] < f.q[y][0]; });
    memset(fa, 0, sizeof(*fa));
    fa->k = f.k;
    fa->word_mask = f.word_mask;
    for (uint32_t t = 0; t < f.k; t++) {
        fa->dst[t] = f.dst[idx[t]];
        memcpy(fa->q[t], f.q[idx[t]], sizeof(fa->q[t]));
    }
    Scratch s(c);
    const uint64_t nwords = ((uint64_t)g->n + 63) / 64;
    const uint32_t nrounds = (uint32_t)(((uint64_t)g->n + FM_TILE - 1) / FM_TILE);
    const uint32_t nb = std::max<uint32_t>(1, std::min<uint32_t>(nrounds, 8192));
    FilterArgs *dp = reinterpret_cast<FilterArgs *>(s.get<uint32_t>(sizeof(FilterArgs) / 4, "filter pass"));
    uint32_t *part = s.get<uint32_t>((uint64_t)GSI_MAX_K * nb, "filter partial counts");
    GSI_HIP(hipMemcpyAsync(dp, fa, sizeof(FilterArgs), hipMemcpyHostToDevice, c->stream));
    const double bytes = 4.0 * g->n * (1 + __builtin_popcount(f.word_mask)) + (double)f.k * nwords * 8;
    launch(c, "k_filter", bytes, k_filter_multi, dim3(nb, 1), QT, (const uint32_t *)g->sig, g->n, nwords,
           (const FilterArgs *)dp, bits, part);
    launch(c, "k_filter_counts", 8.0 * f.k * nwords, k_bit_counts, f.k, 1024, (const uint64_t *)bits, nwords, counts,
           runs);
}

static void filter_impl(gsi_graph *g, const HostQuery &q, bool label_only, uint64_t *bits, uint32_t *counts,
                        bool homo = false, uint32_t *runs = nullptr) {
    gsi_ctx *c = g->ctx;
    FilterArgs fa;
    query_signatures(q, fa, homo);
    fa.label_only = label_only ? 1u : 0u;
    if (GROUPED_SINGLE_FILTER && !label_only && !q.multi && !g->multi) {
        launch_filter_grouped(c, g, fa, bits, counts, runs);
        return;
    }
    launch_filter(c, g, fa, bits, counts, runs, q.multi ? &q : nullptr);
}

void run_filter(gsi_graph *g, const HostQuery &q, uint64_t *bits, uint32_t *counts) {
    filter_impl(g, q, false, bits, counts);
}

// ----------------------------------------------------- M0 from a bitset
__global__ void k_word_popc(const uint64_t *bits, uint64_t nwords, uint32_t *cnt) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nwords) cnt[i] = (uint32_t)__popcll(bits[i]);
}
__global__ void k_word_emit(const uint64_t *bits, uint64_t nwords, const uint64_t *off, uint32_t *out) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nwords) return;
    uint64_t b = bits[i];
    uint64_t o = off[i];
    while (b) {
        uint32_t t = (uint32_t)__ffsll((unsigned long long)b) - 1;
        out[o++] = (uint32_t)(i * 64 + t);
        b &= b - 1;
    }
}

// ------------------------------------------------------------ join level
// The list a row scans (its slots of GBA): the first edge e0 of Algorithm 4,
// or, with `pick`, whichever linking list of the row is shortest (e0 on
// ties).  The row's survivors are the same either way (they lie in every
// linking list), and, the lists being sorted, so is their order.
__global__ __launch_bounds__(QT) void k_locate(LevelArgs a) {
    const uint64_t i = (uint64_t)blockIdx.x * QT + threadIdx.x;
    const bool valid = i < a.R;
    uint64_t other = 0;
    if (valid) {
        uint32_t s0 = 0, l0 = 0, ob = NONE32, os = 0, ol = 0xFFFFFFFFu;
        uint64_t all = 0;
        for (uint32_t e = 0; e < a.ne; e++) {
            const EdgeRef &er = a.e[e];
            uint32_t v = a.M[(uint64_t)er.col * a.ldm + i];
            uint2 r = a.abl_cr ? cr_find(er, v) : pcsr_find(er.gl, er.G, er.H, v);
            reinterpret_cast<uint2 *>(a.loc)[(uint64_t)e * a.R + i] = r;
            all += r.y;
            if (e == a.e0) {
                s0 = r.x;
                l0 = r.y;
            } else if (r.y < ol) {
                ob = e;
                os = r.x;
                ol = r.y;
            }
        }
        uint32_t be = a.e0, bs = s0, bl = l0;
        if (a.pick && ob != NONE32 && ol < l0) {
            be = ob;
            bs = os;
            bl = ol;
        }
        a.bound[i] = bl;
        a.loc[(uint64_t)(2 * a.ne) * a.R + i] = a.e[be].ci_off + bs;
        if (a.ne > 1) a.loc[(uint64_t)(2 * a.ne + 1) * a.R + i] = be;
        // elements of the other linking lists the join must read at least:
        // testing at most bl candidates against a list of L entries touches
        // at least min(L, bl) of them (one per candidate, or the whole list)
        if (a.part) {
            (void)all;
            for (uint32_t e = 0; e < a.ne; e++) {
                if (e == be) continue;
                const uint64_t L = loc_pair(a, e, i).y;
                other += L < (uint64_t)bl ? L : (uint64_t)bl;
            }
        }
    }
    if (a.part) {  // list-length totals are gathered for profiling only
        __shared__ uint64_t s_o[QT / 64];
        other = wave_sum(other);
        if (lane_id() == 0) s_o[threadIdx.x >> 6] = other;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t t = 0;
#pragma unroll
            for (int q = 0; q < QT / 64; q++) t += s_o[q];
            a.part[2 * (uint64_t)blockIdx.x] = t;
            a.part[2 * (uint64_t)blockIdx.x + 1] = 0;
        }
    }
    if (a.scan_total) {  // the only workgroup: F = exclusive sums of the bounds
        __shared__ uint64_t s_b[QT / 64];
        const uint64_t b = valid ? a.bound[i] : 0u;
        const uint64_t inc = wave_inclusive_sum(b);
        if (lane_id() == 63) s_b[threadIdx.x >> 6] = inc;
        __syncthreads();
        uint64_t pre = 0, tot = 0;
#pragma unroll
        for (uint32_t q = 0; q < QT / 64; q++) {
            pre += q < (threadIdx.x >> 6) ? s_b[q] : 0ull;
            tot += s_b[q];
        }
        uint64_t *F = const_cast<uint64_t *>(a.F);
        if (valid) F[i] = pre + inc - b;
        if (threadIdx.x == 0) {
            F[a.R] = tot;
            *a.scan_total = tot;
            post_seq(a.seq_slot, a.seq_value);
        }
    }
}

// tile_row[t] = the row whose slice of GBA holds element ts*t
__global__ __launch_bounds__(QT) void k_tile_rows(const uint64_t *F, uint64_t R, uint64_t ntiles, uint32_t ts,
                                                 uint64_t *tile_row) {
    const uint64_t i = (uint64_t)blockIdx.x * QT + threadIdx.x;
    if (i >= R) return;
    const uint64_t lo = F[i], hi = F[i + 1];
    for (uint64_t t = (lo + ts - 1) / ts; t * ts < hi; t++) tile_row[t] = i;
    if (i == R - 1) tile_row[ntiles] = R - 1;
}

void tile_rows(gsi_ctx *c, const uint64_t *F, uint64_t R, uint64_t ntiles, uint64_t *tile_row) {
    launch(c, "k_tile_rows", 8.0 * (R + 1) + 8.0 * (ntiles + 1), k_tile_rows, nblocks(R), QT, F, R, ntiles, (uint32_t)QT,
           tile_row);
}

// Level-wide filtering of the first-edge lists.  When the rows of a level
// scan far more list elements than label l0 holds (rows repeat hub
// vertices: Sec. VI-B's duplicate reads, level-wide), the C(u) test is run
// once per element of l0's lists instead of once per slot: keep bits over
// l0's ci, their per-word prefix counts, and the kept elements compacted in
// order (every list stays contiguous and ascending, so list [s, s+len)
// becomes [rank(s), rank(s+len)) of the compacted array).  Each row then
// scans its list's members of C(u) only; the survivors, and their order,
// are unchanged.
// Each thread takes FN_TILES elements (one per 256-element tile of its
// workgroup) and issues their loads, then their C(u) word loads, together.
constexpr uint32_t FN_TILES = 4;

__global__ __launch_bounds__(QT) void k_fn_bits(const uint32_t *ci, uint64_t n, const uint64_t *Cu, uint64_t *bits,
                                               uint32_t *wcnt) {
    uint32_t x[FN_TILES];
    uint64_t cw[FN_TILES];
#pragma unroll
    for (uint32_t r = 0; r < FN_TILES; r++) {
        const uint64_t p = ((uint64_t)blockIdx.x * FN_TILES + r) * QT + threadIdx.x;
        x[r] = ci[p < n ? p : n - 1];
    }
#pragma unroll
    for (uint32_t r = 0; r < FN_TILES; r++) cw[r] = Cu[x[r] >> 6];
#pragma unroll
    for (uint32_t r = 0; r < FN_TILES; r++) {
        const uint64_t p = ((uint64_t)blockIdx.x * FN_TILES + r) * QT + threadIdx.x;
        const bool keep = p < n && ((cw[r] >> (x[r] & 63)) & 1ull);
        const uint64_t m = __ballot(keep);
        if (lane_id() == 0 && p < n) {
            bits[p >> 6] = m;
            wcnt[p >> 6] = (uint32_t)__popcll(m);
        }
    }
}

__global__ __launch_bounds__(QT) void k_fn_compact(const uint32_t *ci, uint64_t n, const uint64_t *bits,
                                                  const uint64_t *wpre, uint32_t *fn) {
    const uint64_t p = (uint64_t)blockIdx.x * QT + threadIdx.x;
    if (p >= n) return;
    const uint64_t m = bits[p >> 6];
    if ((m >> (p & 63)) & 1ull) fn[wpre[p >> 6] + (uint64_t)__popcll(m & ((1ull << (p & 63)) - 1))] = ci[p];
}

// kept elements of l0's lists before position p
__device__ __forceinline__ uint64_t fn_rank(const uint64_t *bits, const uint64_t *wpre, uint64_t p) {
    const uint64_t w = p >> 6;
    const uint32_t b = (uint32_t)(p & 63);
    return b ? wpre[w] + (uint64_t)__popcll(bits[w] & ((1ull << b) - 1)) : wpre[w];
}

// every row scans its e0 list, filtered: its slots are that list's members
// of C(u)
__global__ __launch_bounds__(QT) void k_fn_relocate(LevelArgs a, const uint64_t *bits, const uint64_t *wpre) {
    const uint64_t i = (uint64_t)blockIdx.x * QT + threadIdx.x;
    if (i >= a.R) return;
    const uint2 sl = loc_pair(a, a.e0, i);
    const uint32_t s = sl.x, len = sl.y;
    const uint64_t fs = len ? fn_rank(bits, wpre, s) : 0;
    const uint64_t fe = len ? fn_rank(bits, wpre, (uint64_t)s + len) : 0;
    a.bound[i] = (uint32_t)(fe - fs);
    a.loc[(uint64_t)(2 * a.ne) * a.R + i] = (uint32_t)fs;
    if (a.ne > 1) a.loc[(uint64_t)(2 * a.ne + 1) * a.R + i] = a.e0;
}

// |GBA| over the label's directed entries from which the level filters its
// first-edge lists once for the whole level
constexpr double FN_FACTOR = 2.0;
// The fused workgroup builds M0 from root bitsets of at most this many
// words (2^20 vertices); a larger bitset is emitted grid-wide first
// (popcounts, scan, emit), since one CU reading it all costs more: on
// 8.4M vertices the fused launches went from 6.2 to 4.1 ms per 50 queries
// for 0.8 ms of added launches.
constexpr uint64_t M0_FUSED_MAX_WORDS = 16384;

// The per-level join and link work on tiles of SPT x 256 |GBA| slots.  On
// large levels (SPT = 4) a 256-thread workgroup takes four consecutive
// 256-slot rounds, issuing the loads of its four slots together, so the
// tile's set-up (its rows staged in LDS) is paid once per 1024 slots and
// each thread has four independent gathers in flight; small levels keep
// one slot per thread (SPT = 1) and four times as many workgroups.
constexpr uint64_t WIDE_TILE_SLOTS = 1ull << 20;  // |GBA| from which SPT = 4
// Candidates a join thread tests at once (keep_many).  The join is bound by
// its gathers (their issue and their latency), so waves in flight matter
// more than loads per thread: two candidates per thread fit in 64 VGPRs,
// the most that still lets a SIMD hold 8 waves (the join and the record
// link are built for 8, their spare scalar registers going to VGPR lanes);
// four took 95 VGPRs (5 waves) and were 19 % slower on an R-MAT graph of
// 8.4M vertices and 100M edges.
constexpr uint32_t JU = 2;
// rows of the last level are staged in LDS and written out as one
// contiguous block per round (coalesced stores) when k is at most this
constexpr uint32_t LINK_STAGE_K = 16;

// The rows r_lo..r_hi a tile touches.  When they are at most the tile's slot
// count they are staged in LDS; tiles spanning more rows (long runs of rows
// with no first-edge neighbours) search F in global memory instead.  The
// link stages F[i] and the start of N(v'_i, l0) in ci and finds the row of
// each survivor by a binary search in LDS (stage_rows, find_row): its
// survivors are often few.  The join, which needs the row of every slot,
// builds a map from slot to row once per tile (stage_slot_rows).
struct TileRows {
    uint64_t r_lo, r_hi;
    bool staged;
};

template <uint32_t SPT>
__device__ __forceinline__ TileRows stage_rows(const LevelArgs &a, uint64_t tile, uint64_t *s_F, uint32_t *s_st) {
    TileRows t;
    t.r_lo = a.tile_row[tile];
    t.r_hi = a.tile_row[tile + 1];
    const uint64_t nr = t.r_hi - t.r_lo + 1;
    t.staged = nr <= SPT * QT;
    if (t.staged) {
        for (uint32_t r = threadIdx.x; r < nr; r += QT) {
            s_F[r] = a.F[t.r_lo + r];
            s_st[r] = a.loc[(uint64_t)(2 * a.ne) * a.R + t.r_lo + r];
        }
        __syncthreads();
    }
    return t;
}

// row i holding slot p, with F[i] and the start (in ci_all) of its scanned list
__device__ __forceinline__ void find_row(const LevelArgs &a, const TileRows &t, const uint64_t *s_F,
                                         const uint32_t *s_st, uint64_t p, uint64_t *i, uint64_t *Fi, uint32_t *st) {
    if (t.staged) {
        uint32_t lo = 0, hi = (uint32_t)(t.r_hi - t.r_lo);
        while (lo < hi) {
            uint32_t mid = (lo + hi + 1) >> 1;
            if (s_F[mid] <= p) lo = mid;
            else hi = mid - 1;
        }
        *i = t.r_lo + lo;
        *Fi = s_F[lo];
        *st = s_st[lo];
    } else {
        *i = row_of(a.F, t.r_lo, t.r_hi, p);
        *Fi = a.F[*i];
        *st = a.loc[(uint64_t)(2 * a.ne) * a.R + *i];
    }
}

// The join's view of a tile's rows.  When they fit (staged), every slot's
// row is found once for the whole tile instead of by a binary search per
// slot: each row after the first marks the slot where its slice of GBA
// starts (the largest row wins where empty rows share a start), and a
// max-scan over the tile's slots carries each mark forward, so s_row[s] is
// the largest row whose slice starts at or before slot s.  s_base[r] is the
// position in ci_all of the tile's slot 0 as seen from row r (mod 2^32), so
// slot s reads ci_all[s_base[s_row[s]] + s].  s_row must be zero on entry,
// published by a barrier.
template <uint32_t SPT>
__device__ __forceinline__ TileRows stage_slot_rows(const LevelArgs &a, uint64_t tile, uint32_t *s_row,
                                                    uint32_t *s_base, uint32_t *s_w) {
    constexpr uint32_t TS = SPT * QT;
    TileRows t;
    if (a.rows_in_join) {
        // at most 256 rows: wave 0 counts the row starts at or before the
        // tile's first slot and the next tile's (four per lane), which gives
        // the rows holding them; the link reads tile_row[tile] later
        __shared__ uint32_t s_rr[2];
        if (threadIdx.x < 64) {
            const uint64_t p0 = tile * TS, p1 = p0 + TS;
            uint32_t c0 = 0, c1 = 0;
#pragma unroll
            for (uint32_t k = 0; k < 4; k++) {
                const uint64_t r = 4ull * threadIdx.x + k;
                const uint64_t f = a.F[r < a.R ? r : 0];
                c0 += (r < a.R && f <= p0) ? 1u : 0u;
                c1 += (r < a.R && f <= p1) ? 1u : 0u;
            }
            c0 = wave_sum(c0);
            c1 = wave_sum(c1);
            if (threadIdx.x == 0) {
                s_rr[0] = c0 - 1;
                s_rr[1] = p1 < a.gba ? c1 - 1 : (uint32_t)(a.R - 1);
                const_cast<uint64_t *>(a.tile_row)[tile] = c0 - 1;
                if (tile + 1 == gridDim.x) const_cast<uint64_t *>(a.tile_row)[tile + 1] = a.R - 1;
            }
        }
        __syncthreads();
        t.r_lo = s_rr[0];
        t.r_hi = s_rr[1];
    } else {
        t.r_lo = a.tile_row[tile];
        t.r_hi = a.tile_row[tile + 1];
    }
    const uint64_t nr = t.r_hi - t.r_lo + 1;
    t.staged = nr <= TS;
    if (t.staged) {
        const uint64_t p0 = tile * TS;
        for (uint32_t r = threadIdx.x; r < nr; r += QT) {
            const uint64_t F = a.F[t.r_lo + r];
            s_base[r] = a.loc[(uint64_t)(2 * a.ne) * a.R + t.r_lo + r] + (uint32_t)(p0 - F);
            // rows after the first start past p0 (the first holds slot 0)
            if (r > 0 && F - p0 < TS) atomicMax(&s_row[F - p0], r);
        }
        __syncthreads();
        block_max_scan<QT, SPT>(s_row, s_w);
    }
    return t;
}

// row i of the tile's slot s and the position of its element in ci_all
__device__ __forceinline__ void slot_row(const LevelArgs &a, const TileRows &t, const uint32_t *s_row,
                                         const uint32_t *s_base, uint64_t p0, uint32_t s, uint64_t *i,
                                         uint32_t *pos) {
    if (t.staged) {
        const uint32_t r = s_row[s];
        *i = t.r_lo + r;
        *pos = s_base[r] + s;
    } else {
        const uint64_t p = p0 + s;
        *i = row_of(a.F, t.r_lo, t.r_hi, p);
        *pos = a.loc[(uint64_t)(2 * a.ne) * a.R + *i] + (uint32_t)(p - a.F[*i]);
    }
}

template <uint32_t SPT>
__global__ __launch_bounds__(QT) __attribute__((amdgpu_waves_per_eu(8))) void k_join(LevelArgs a) {
    constexpr uint32_t TS = SPT * QT;
    __shared__ uint32_t s_row[TS];    // row of each slot of the tile (staged tiles)
    __shared__ uint32_t s_base[TS];   // per row: ci_all position of slot 0
    __shared__ uint32_t s_x[TS];      // elements that passed the C(u) test, compacted
    __shared__ uint32_t s_ri[TS];     // and their rows (from r_lo)
    __shared__ uint16_t s_slot[TS];   // and their slots in the tile
    __shared__ uint64_t s_keep[TS / 64];
    __shared__ uint32_t s_w[QT / 64];
    __shared__ uint32_t s_n;
    if (threadIdx.x == 0) s_n = 0;
    if (threadIdx.x < TS / 64) s_keep[threadIdx.x] = 0;
#pragma unroll
    for (uint32_t k = 0; k < SPT; k++) s_row[threadIdx.x * SPT + k] = 0;
    __syncthreads();
    const uint64_t p0 = (uint64_t)blockIdx.x * TS;
    const TileRows tr = stage_slot_rows<SPT>(a, blockIdx.x, s_row, s_base, s_w);
    const uint32_t *ci0 = a.ci_all;
    const uint32_t lane = lane_id();
    uint32_t xs[SPT];
    uint64_t is[SPT];
    bool kp[SPT];
    // x = N(v'_i, l0)[p - F[i]] for the thread's slots
#pragma unroll
    for (uint32_t r = 0; r < SPT; r++) {
        const uint32_t sl = r * QT + threadIdx.x;
        kp[r] = p0 + sl < a.gba;
        xs[r] = 0;
        is[r] = 0;
        if (kp[r]) {
            uint32_t pos;
            slot_row(a, tr, s_row, s_base, p0, sl, &is[r], &pos);
            xs[r] = ci0[pos];
        }
    }
    // x in C(u); the slots that pass are compacted (in no particular order)
    // so that the remaining tests, the costly ones, run in dense waves
    if (!a.prefiltered) {
        // every slot's C(u) word is loaded before any is tested (an invalid
        // slot has x = 0, a valid word)
        uint64_t cw[SPT];
#pragma unroll
        for (uint32_t r = 0; r < SPT; r++) cw[r] = a.Cu[xs[r] >> 6];
#pragma unroll
        for (uint32_t r = 0; r < SPT; r++) kp[r] = kp[r] && ((cw[r] >> (xs[r] & 63)) & 1ull);
    }
#pragma unroll
    for (uint32_t r = 0; r < SPT; r++) {
        const uint64_t mask = __ballot(kp[r]);
        if (mask) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(&s_n, (uint32_t)__popcll(mask));
            base = __shfl(base, 0, 64);
            if (kp[r]) {
                const uint32_t idx = base + rank_below(mask);
                s_slot[idx] = (uint16_t)(r * QT + threadIdx.x);
                s_x[idx] = xs[r];
                s_ri[idx] = (uint32_t)(is[r] - tr.r_lo);
            }
        }
    }
    __syncthreads();
    // x not in m_i (the row's values are loaded four at a time, not one
    // dependent load per column), x in every other linking list
    const uint32_t n = __builtin_amdgcn_readfirstlane(s_n);
    // JU candidates per thread at a time, their loads issued together
    for (uint32_t e0 = 0; e0 < n; e0 += JU * QT) {
        uint32_t xs[JU], sl[JU];
        uint64_t is[JU];
        bool kp[JU];
#pragma unroll
        for (uint32_t u = 0; u < JU; u++) {
            const uint32_t e = e0 + u * QT + threadIdx.x;
            kp[u] = e < n;
            const uint32_t c = kp[u] ? e : 0u;  // a past-the-end thread reads candidate 0
            sl[u] = s_slot[c];
            xs[u] = s_x[c];
            is[u] = tr.r_lo + s_ri[c];
        }
        keep_many<JU>(a, xs, is, kp);
#pragma unroll
        for (uint32_t u = 0; u < JU; u++)
            if (kp[u]) atomicOr(&s_keep[sl[u] >> 6], 1ull << (sl[u] & 63));
    }
    __syncthreads();
    if (a.rec_x) {
        // the tile's survivors as records in slot order (element, row from
        // r_lo), so that the link reads them instead of searching rows and
        // re-gathering elements
        __shared__ uint32_t s_pre[TS / 64 + 1];
        if (threadIdx.x < 64) {
            const uint32_t c = threadIdx.x < TS / 64 ? (uint32_t)__popcll(s_keep[threadIdx.x]) : 0u;
            const uint32_t inc = wave_inclusive_sum(c);
            if (threadIdx.x < TS / 64) s_pre[threadIdx.x] = inc - c;
            if (threadIdx.x == 63) {
                s_pre[TS / 64] = inc;
                a.tile_cnt[blockIdx.x] = inc;
            }
        }
        __syncthreads();
        // every kept slot was a candidate: its element and row are in the
        // compacted lists (read from LDS, not held in registers across the
        // tests); its record goes to its rank among the tile's kept slots
        const uint64_t rb = (uint64_t)blockIdx.x * TS;
        for (uint32_t e = threadIdx.x; e < n; e += QT) {
            const uint32_t sl = s_slot[e];
            const uint64_t word = s_keep[sl >> 6];
            if ((word >> (sl & 63)) & 1ull) {
                const uint32_t q = s_pre[sl >> 6] + (uint32_t)__popcll(word & ((1ull << (sl & 63)) - 1));
                a.rec_x[rb + q] = s_x[e];
                a.rec_r[rb + q] = s_ri[e];
            }
        }
    } else if (threadIdx.x < 64) {
        // the tile's keep bits (one word per 64 slots) and their count
        const uint64_t word = threadIdx.x < TS / 64 ? s_keep[threadIdx.x] : 0ull;
        if (threadIdx.x < TS / 64 && !a.abl_two_step) a.bitmap[(uint64_t)blockIdx.x * (TS / 64) + threadIdx.x] = word;
        const uint32_t t = wave_sum((uint32_t)__popcll(word));
        if (threadIdx.x == 0) a.tile_cnt[blockIdx.x] = t;
    }
}

// The link over survivor records (k_join wrote each tile's kept slots in
// slot order as (element, row) records): survivor q of tile t is row
// tile_off[t] + q of M', extended from row tile_row[t] + rec_r of M by
// rec_x.  No row search and no second gather of the element.
// W > 0: the row has at most 4W values to gather (j columns on an inner
// level, k values on the last), so all 4W loads are issued in one
// straight-line batch (entries past the row re-read a valid column); W = 0
// takes any width, eight columns per batch.
template <uint32_t SPT, uint32_t W>
__global__ __launch_bounds__(QT) __attribute__((amdgpu_waves_per_eu(8))) void k_link_rec(LevelArgs a) {
    constexpr uint32_t TS = SPT * QT;
    __shared__ uint64_t s_d[2][QT / 64];
    __shared__ uint32_t s_rows[QT * LINK_STAGE_K];
    __shared__ uint32_t s_qc[GSI_MAX_K];  // query vertex -> column (last level)
    const uint64_t tile = blockIdx.x;
    const uint64_t tbase = a.tile_off[tile];
    const uint32_t n = (uint32_t)(a.tile_off[tile + 1] - tbase);
    if (n == 0) {  // uniform
        if (a.final_level && threadIdx.x == 0) {
            a.dig_part[2 * tile] = 0;
            a.dig_part[2 * tile + 1] = 0;
        }
        return;
    }
    if (threadIdx.x < GSI_MAX_K) s_qc[threadIdx.x] = a.qcol[threadIdx.x];
    __syncthreads();
    const uint32_t w = threadIdx.x >> 6, lane = lane_id();
    const uint64_t r_lo = a.tile_row[tile];
    const uint64_t rb = tile * TS;
    const bool stage = a.final_level && !a.count_only && a.k <= LINK_STAGE_K;
    uint64_t hs = 0, hx = 0;
    for (uint32_t q0 = 0; q0 < n; q0 += QT) {
        const uint32_t q = q0 + threadIdx.x;
        const uint64_t pos = tbase + q;
        const bool mine = q < n && pos < a.S;
        const uint32_t qq = mine ? q : 0u;  // a past-the-end thread reads record 0
        const uint32_t x = a.rec_x[rb + qq];
        const uint64_t i = r_lo + a.rec_r[rb + qq];
        if (!a.final_level) {
            if (mine) {
                if (W) {
                    uint32_t m[4 * (W ? W : 1)];
#pragma unroll
                    for (uint32_t c = 0; c < 4 * W; c++) m[c] = a.M[(uint64_t)(c < a.j ? c : a.j - 1) * a.ldm + i];
#pragma unroll
                    for (uint32_t c = 0; c < 4 * W; c++)
                        if (c < a.j) a.Mn[(uint64_t)c * a.S + pos] = m[c];
                } else {
                    copy_row(a, i, a.Mn, a.S, pos);
                }
                a.Mn[(uint64_t)a.j * a.S + pos] = x;
            }
        } else if (mine && W) {
            uint64_t f = 14695981039346656037ull;
            uint32_t val[4 * (W ? W : 1)];
#pragma unroll
            for (uint32_t u = 0; u < 4 * W; u++) {
                const uint32_t c = u < a.k ? s_qc[u] : a.j;
                const uint32_t mv = a.M[(uint64_t)(c < a.j ? c : 0u) * a.ldm + i];
                val[u] = c < a.j ? mv : x;
            }
#pragma unroll
            for (uint32_t u = 0; u < 4 * W; u++) {
                if (u >= a.k) break;
                if (stage) s_rows[threadIdx.x * a.k + u] = val[u];
                else if (!a.count_only) a.out[pos * a.k + u] = val[u];
                f = fnv_word(f, val[u]);
            }
            const uint64_t h = mix64(f);
            hs += h;
            hx ^= h;
        } else if (mine) {
            uint64_t f = 14695981039346656037ull;
            for (uint32_t u0 = 0; u0 < a.k; u0 += 8) {
                uint32_t val[8];
                // every load issued before any is used (no branch between them)
#pragma unroll
                for (uint32_t k4 = 0; k4 < 8; k4++) {
                    const uint32_t c = u0 + k4 < a.k ? s_qc[u0 + k4] : a.j;
                    const uint32_t mv = a.M[(uint64_t)(c < a.j ? c : 0u) * a.ldm + i];
                    val[k4] = c < a.j ? mv : x;
                }
#pragma unroll
                for (uint32_t k4 = 0; k4 < 8; k4++) {
                    const uint32_t u = u0 + k4;
                    if (u >= a.k) break;
                    if (stage) s_rows[threadIdx.x * a.k + u] = val[k4];
                    else if (!a.count_only) a.out[pos * a.k + u] = val[k4];
                    f = fnv_word(f, val[k4]);
                }
            }
            const uint64_t h = mix64(f);
            hs += h;
            hx ^= h;
        }
        if (stage) {
            // the round's rows are one contiguous block of the output
            __syncthreads();
            const uint64_t first = tbase + q0;
            uint64_t end = tbase + (q0 + QT < n ? q0 + QT : n);
            if (end > a.S) end = a.S;
            const uint32_t nw = first < end ? (uint32_t)(end - first) * a.k : 0u;
            uint32_t *dst = a.out + first * a.k;
            for (uint32_t t = threadIdx.x; t < nw; t += QT) dst[t] = s_rows[t];
            __syncthreads();
        }
    }
    if (a.final_level) {
        const uint64_t sum = wave_sum(hs), xr = wave_xor(hx);
        if (lane == 0) {
            s_d[0][w] = sum;
            s_d[1][w] = xr;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t ts = 0, tx = 0;
#pragma unroll
            for (int q = 0; q < QT / 64; q++) {
                ts += s_d[0][q];
                tx ^= s_d[1][q];
            }
            a.dig_part[2 * tile] = ts;
            a.dig_part[2 * tile + 1] = tx;
        }
    }
}


// k_link_rec for tiles of spt x 256 slots and rows of at most 4 * wg
// values (wg = 0: any)
template <uint32_t SPT>
static void launch_link_rec_w(gsi_ctx *c, double lb, uint32_t wg, uint32_t ntiles, const LevelArgs &a) {
    switch (wg) {
        case 1: launch(c, "k_link", lb, k_link_rec<SPT, 1>, ntiles, QT, a); break;
        case 2: launch(c, "k_link", lb, k_link_rec<SPT, 2>, ntiles, QT, a); break;
        case 3: launch(c, "k_link", lb, k_link_rec<SPT, 3>, ntiles, QT, a); break;
        case 4: launch(c, "k_link", lb, k_link_rec<SPT, 4>, ntiles, QT, a); break;
        default: launch(c, "k_link", lb, k_link_rec<SPT, 0>, ntiles, QT, a); break;
    }
}
static void launch_link_rec(gsi_ctx *c, double lb, uint32_t spt, uint32_t wg, uint32_t ntiles, const LevelArgs &a) {
    if (spt == 4) launch_link_rec_w<4>(c, lb, wg, ntiles, a);
    else launch_link_rec_w<1>(c, lb, wg, ntiles, a);
}

template <uint32_t SPT>
__global__ __launch_bounds__(QT) void k_link(LevelArgs a) {
    constexpr uint32_t TS = SPT * QT;
    __shared__ uint64_t s_d[2][QT / 64];
    __shared__ uint64_t s_F[TS];
    __shared__ uint32_t s_st[TS];
    __shared__ uint32_t s_rows[QT * LINK_STAGE_K];
    __shared__ uint32_t s_pre[TS / 64 + 1];  // kept slots before each bitmap word of the tile
    __shared__ uint64_t s_w[TS / 64];        // the tile's keep bits (two-step ablation)
    __shared__ uint16_t s_list[TS];          // the tile's kept slots, compacted
    __shared__ uint32_t s_qc[GSI_MAX_K];     // query vertex -> column (last level)
    const uint64_t tile = blockIdx.x;
    // the column map is read from LDS in the row loop: from the argument
    // segment each column would be a scalar load waited on in turn
    if (threadIdx.x < GSI_MAX_K) s_qc[threadIdx.x] = a.qcol[threadIdx.x];
    if (a.tile_off[tile + 1] == a.tile_off[tile]) {  // whole tile empty (uniform)
        if (a.final_level && threadIdx.x == 0) {
            a.dig_part[2 * tile] = 0;
            a.dig_part[2 * tile + 1] = 0;
        }
        return;
    }
    const uint64_t p0 = tile * TS;
    const uint64_t *words = a.bitmap + tile * (TS / 64);
    if (threadIdx.x == 0 && !a.abl_two_step) {
        uint32_t run = 0;
        for (uint32_t q = 0; q < TS / 64; q++) {
            s_pre[q] = run;
            run += (uint32_t)__popcll(words[q]);
        }
        s_pre[TS / 64] = run;
    }
    const TileRows tr = stage_rows<SPT>(a, tile, s_F, s_st);  // (its barrier also publishes s_pre)
    if (!tr.staged) __syncthreads();
    const uint32_t w = threadIdx.x >> 6, lane = lane_id();
    if (a.abl_two_step) {
        // two-step output: the join only counted; find the survivors again
        for (uint32_t r = 0; r < SPT; r++) {
            const uint64_t p = p0 + r * QT + threadIdx.x;
            bool keep = false;
            if (p < a.gba) {
                uint64_t i, Fi;
                uint32_t st0;
                find_row(a, tr, s_F, s_st, p, &i, &Fi, &st0);
                keep = slot_keep(a, i, a.ci_all[st0 + (uint32_t)(p - Fi)]);
            }
            const uint64_t mask = __ballot(keep);
            if (lane == 0) s_w[r * (QT / 64) + w] = mask;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t run = 0;
            for (uint32_t q = 0; q < TS / 64; q++) {
                s_pre[q] = run;
                run += (uint32_t)__popcll(s_w[q]);
            }
            s_pre[TS / 64] = run;
        }
        __syncthreads();
        words = s_w;
    }
    const uint64_t tbase = a.tile_off[tile];
    const bool stage = a.final_level && !a.count_only && a.k <= LINK_STAGE_K && !a.abl_no_stage;
    const uint32_t *ci0 = a.ci_all;
    uint64_t hs = 0, hx = 0;
    // The tile's kept slots, compacted in slot order into s_list, so that
    // the waves that gather, write and hash are dense: in a sparse last level
    // nearly every wave holds some kept slot, and would run the whole
    // survivor path for a few lanes.  Survivor q of the tile (its q-th kept
    // slot) is row tbase + q of M'.
#pragma unroll
    for (uint32_t r = 0; r < SPT; r++) {
        const uint32_t wi = r * (QT / 64) + w;
        const uint64_t word = words[wi];
        if ((word >> lane) & 1ull) s_list[s_pre[wi] + rank_below(word)] = (uint16_t)(r * QT + threadIdx.x);
    }
    __syncthreads();
    // the same count in every lane (the loop holds barriers)
    const uint32_t n = __builtin_amdgcn_readfirstlane(s_pre[TS / 64]);
    for (uint32_t q0 = 0; q0 < n; q0 += QT) {
        const uint32_t q = q0 + threadIdx.x;
        const uint64_t pos = tbase + q;
        if (q < n && pos < a.S) {
            const uint64_t p = p0 + s_list[q];
            uint64_t i, Fi;
            uint32_t st0;
            find_row(a, tr, s_F, s_st, p, &i, &Fi, &st0);
            const uint32_t x = ci0[st0 + (uint32_t)(p - Fi)];
            // the row's values are loaded four at a time (independent
            // loads), not one dependent round trip per column
            if (!a.final_level) {
                copy_row(a, i, a.Mn, a.S, pos);
                a.Mn[(uint64_t)a.j * a.S + pos] = x;
            } else {
                const uint32_t local = threadIdx.x;  // row within this round's block
                uint64_t f = 14695981039346656037ull;
                for (uint32_t u0 = 0; u0 < a.k; u0 += 8) {
                    uint32_t val[8];
                    // every load issued before any is used (no branch between them)
#pragma unroll
                    for (uint32_t k4 = 0; k4 < 8; k4++) {
                        const uint32_t c = u0 + k4 < a.k ? s_qc[u0 + k4] : a.j;
                        const uint32_t mv = a.M[(uint64_t)(c < a.j ? c : 0u) * a.ldm + i];
                        val[k4] = c < a.j ? mv : x;
                    }
#pragma unroll
                    for (uint32_t k4 = 0; k4 < 8; k4++) {
                        const uint32_t u = u0 + k4;
                        if (u >= a.k) break;
                        if (stage) s_rows[local * a.k + u] = val[k4];
                        else if (!a.count_only) a.out[pos * a.k + u] = val[k4];
                        f = fnv_word(f, val[k4]);
                    }
                }
                const uint64_t h = mix64(f);
                hs += h;
                hx ^= h;
            }
        }
        if (stage) {
            // the round's rows are one contiguous block of the output
            __syncthreads();
            const uint64_t first = tbase + q0;
            uint64_t end = tbase + (q0 + QT < n ? q0 + QT : n);
            if (end > a.S) end = a.S;
            const uint32_t nw = first < end ? (uint32_t)(end - first) * a.k : 0u;
            uint32_t *dst = a.out + first * a.k;
            for (uint32_t t = threadIdx.x; t < nw; t += QT) dst[t] = s_rows[t];
            __syncthreads();
        }
    }
    if (a.final_level) {
        // per-tile partial digest; reduced by one small kernel afterwards
        uint64_t sum = wave_sum(hs), xr = wave_xor(hx);
        if (lane == 0) {
            s_d[0][w] = sum;
            s_d[1][w] = xr;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t ts = 0, tx = 0;
#pragma unroll
            for (int q = 0; q < QT / 64; q++) {
                ts += s_d[0][q];
                tx ^= s_d[1][q];
            }
            a.dig_part[2 * tile] = ts;
            a.dig_part[2 * tile + 1] = tx;
        }
    }
}

// ------------------------------------------ single-pass last level
// The last join level in one launch: each workgroup joins its tile (as
// k_join), learns where its survivors start in the output from the tiles
// before it by a decoupled look-back (Merrill and Garland, "Single-pass
// Parallel Prefix Scan with Decoupled Look-back", 2016), and writes its rows
// there at once (as k_link), so the keep bitmap, the tile-count scan, the
// link's second gather of x and its row search all go away.  Tiles are
// numbered in the order workgroups start (an atomic counter), so a tile
// only ever waits for tiles that are already running; each publishes its
// own count before it waits.  A status word holds the value in bits 0..61
// and a flag in bits 62..63: 1 = the tile's count, 2 = the count of every
// row up to and including the tile.
constexpr uint64_t LB_AGG = 1ull << 62, LB_PRE = 2ull << 62, LB_VAL = (1ull << 62) - 1;
constexpr uint32_t LB_SPIN_MAX = 1u << 22;  // re-reads of an unpublished predecessor before giving up

// wave 0 of the workgroup: rows before this tile (uniform in the wave)
__device__ __forceinline__ uint64_t lookback(unsigned long long *st, uint64_t tile, uint64_t count, uint32_t *err) {
    const uint32_t lane = lane_id();
    if (tile == 0) {
        if (lane == 0) __hip_atomic_store(st, LB_PRE | count, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        return 0;
    }
    if (lane == 0) __hip_atomic_store(st + tile, LB_AGG | count, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    int64_t t = (int64_t)tile - 1;  // nearest predecessor not yet added
    uint32_t spins = 0;
    for (;;) {
        const int64_t idx = t - (int64_t)lane;
        const uint64_t v = idx >= 0 ? __hip_atomic_load(st + idx, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)
                                    : LB_PRE;  // before tile 0: a prefix of 0
        const uint32_t flag = (uint32_t)(v >> 62);
        const uint64_t val = v & LB_VAL;
        const uint64_t isP = __ballot(flag == 2), isZ = __ballot(flag == 0);
        const uint32_t p = isP ? (uint32_t)__ffsll((unsigned long long)isP) - 1 : 64u;
        const uint64_t before = p == 64 ? ~0ull : ((1ull << p) - 1);
        const uint64_t zb = isZ & before;
        if (zb) {
            // add the published counts up to the first unpublished tile
            const uint32_t z = (uint32_t)__ffsll((unsigned long long)zb) - 1;
            excl += wave_sum(lane < z ? val : 0ull);
            t -= z;
            if (++spins > LB_SPIN_MAX) {
                if (lane == 0) atomicOr(err, 1u);
                break;
            }
            continue;
        }
        excl += wave_sum(lane <= p ? val : 0ull);
        if (p < 64) break;
        t -= 64;
    }
    if (lane == 0) __hip_atomic_store(st + tile, LB_PRE | (excl + count), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

// FINAL: rows in query-vertex order to a.out (row-major) and the digest;
// else the next table to a.Mn, column-major with column stride a.out_cap.
template <uint32_t SPT, bool FINAL>
__global__ __launch_bounds__(QT) void k_join_pass(LevelArgs a) {
    constexpr uint32_t TS = SPT * QT;
    // The join's arrays and the write's share one LDS block (the join's are
    // dead once the keep bits are summed), so that more workgroups fit a CU.
    constexpr uint32_t JOIN_WORDS = 3 * TS + TS / 2, WRITE_WORDS = (FINAL ? QT * LINK_STAGE_K : 0) + TS / 2;
    __shared__ uint32_t s_u[JOIN_WORDS > WRITE_WORDS ? JOIN_WORDS : WRITE_WORDS];
    __shared__ uint32_t s_row[TS];    // row of each slot (staged tiles)
    __shared__ uint32_t s_xv[TS];     // element of each slot
    uint32_t *s_base = s_u;           // join: per row, ci_all position of slot 0
    uint32_t *s_x = s_u + TS;         // join: elements that passed C(u), compacted
    uint32_t *s_ri = s_u + 2 * TS;    // join: and their rows
    uint16_t *s_slot = reinterpret_cast<uint16_t *>(s_u + 3 * TS);  // join: and their slots
    uint32_t *s_rows = s_u;           // write: the round's rows, staged
    uint16_t *s_list = reinterpret_cast<uint16_t *>(s_u + (FINAL ? QT * LINK_STAGE_K : 0));  // write: kept slots
    __shared__ uint64_t s_keep[TS / 64];
    __shared__ uint32_t s_pre[TS / 64 + 1];
    __shared__ uint32_t s_w[QT / 64];
    __shared__ uint64_t s_d[2][QT / 64];
    __shared__ uint32_t s_qc[GSI_MAX_K];  // query vertex -> column (read from LDS in the row loop)
    __shared__ uint32_t s_n;
    __shared__ uint64_t s_tile, s_off;
    if (threadIdx.x == 0) {
        s_n = 0;
        s_tile = atomicAdd(a.tctr, 1u);
    }
    if (FINAL && threadIdx.x < GSI_MAX_K) s_qc[threadIdx.x] = a.qcol[threadIdx.x];
    if (threadIdx.x < TS / 64) s_keep[threadIdx.x] = 0;
#pragma unroll
    for (uint32_t k = 0; k < SPT; k++) s_row[threadIdx.x * SPT + k] = 0;
    __syncthreads();
    const uint64_t tile = s_tile;
    const uint64_t p0 = tile * TS;
    const TileRows tr = stage_slot_rows<SPT>(a, tile, s_row, s_base, s_w);
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t xs[SPT];
    uint64_t is[SPT];
    bool kp[SPT];
#pragma unroll
    for (uint32_t r = 0; r < SPT; r++) {
        const uint32_t sl = r * QT + threadIdx.x;
        kp[r] = p0 + sl < a.gba;
        xs[r] = 0;
        is[r] = 0;
        if (kp[r]) {
            uint32_t pos;
            slot_row(a, tr, s_row, s_base, p0, sl, &is[r], &pos);
            xs[r] = a.ci_all[pos];
        }
        s_xv[sl] = xs[r];
    }
    if (!a.prefiltered) {
        // every slot's C(u) word is loaded before any is tested (an invalid
        // slot has x = 0, a valid word)
        uint64_t cw[SPT];
#pragma unroll
        for (uint32_t r = 0; r < SPT; r++) cw[r] = a.Cu[xs[r] >> 6];
#pragma unroll
        for (uint32_t r = 0; r < SPT; r++) kp[r] = kp[r] && ((cw[r] >> (xs[r] & 63)) & 1ull);
    }
#pragma unroll
    for (uint32_t r = 0; r < SPT; r++) {
        const uint64_t mask = __ballot(kp[r]);
        if (mask) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(&s_n, (uint32_t)__popcll(mask));
            base = __shfl(base, 0, 64);
            if (kp[r]) {
                const uint32_t idx = base + rank_below(mask);
                s_slot[idx] = (uint16_t)(r * QT + threadIdx.x);
                s_x[idx] = xs[r];
                s_ri[idx] = (uint32_t)(is[r] - tr.r_lo);
            }
        }
    }
    __syncthreads();
    const uint32_t nc = __builtin_amdgcn_readfirstlane(s_n);
    // JU candidates per thread at a time, their loads issued together
    for (uint32_t e0 = 0; e0 < nc; e0 += JU * QT) {
        uint32_t xs[JU], sl[JU];
        uint64_t is[JU];
        bool kp[JU];
#pragma unroll
        for (uint32_t u = 0; u < JU; u++) {
            const uint32_t e = e0 + u * QT + threadIdx.x;
            kp[u] = e < nc;
            const uint32_t c = kp[u] ? e : 0u;  // a past-the-end thread reads candidate 0
            sl[u] = s_slot[c];
            xs[u] = s_x[c];
            is[u] = tr.r_lo + s_ri[c];
        }
        keep_many<JU>(a, xs, is, kp);
#pragma unroll
        for (uint32_t u = 0; u < JU; u++)
            if (kp[u]) atomicOr(&s_keep[sl[u] >> 6], 1ull << (sl[u] & 63));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t q = 0; q < TS / 64; q++) {
            s_pre[q] = run;
            run += (uint32_t)__popcll(s_keep[q]);
        }
        s_pre[TS / 64] = run;
    }
    __syncthreads();
    const uint32_t n = __builtin_amdgcn_readfirstlane(s_pre[TS / 64]);
    if (w == 0) {
        const uint64_t off = lookback(a.tstat, tile, n, a.tctr + 1);
        if (lane == 0) {
            s_off = off;
            if (tile + 1 == (a.gba + TS - 1) / TS) *a.total = off + n;
        }
    }
#pragma unroll
    for (uint32_t r = 0; r < SPT; r++) {
        const uint32_t wi = r * (QT / 64) + w;
        const uint64_t word = s_keep[wi];
        if ((word >> lane) & 1ull) s_list[s_pre[wi] + rank_below(word)] = (uint16_t)(r * QT + threadIdx.x);
    }
    __syncthreads();
    const uint64_t tbase = s_off;
    if (!FINAL) {
        // the next table: survivor q of the tile is row tbase + q of M'
        for (uint32_t q = threadIdx.x; q < n; q += QT) {
            const uint64_t pos = tbase + q;
            if (pos >= a.out_cap) break;
            const uint32_t slot = s_list[q];
            const uint64_t i = tr.staged ? tr.r_lo + s_row[slot] : row_of(a.F, tr.r_lo, tr.r_hi, p0 + slot);
            copy_row(a, i, a.Mn, a.out_cap, pos);
            a.Mn[(uint64_t)a.j * a.out_cap + pos] = s_xv[slot];
        }
        return;
    }
    const bool stage = !a.count_only && a.k <= LINK_STAGE_K;
    uint64_t hs = 0, hx = 0;
    for (uint32_t q0 = 0; q0 < n; q0 += QT) {
        const uint32_t q = q0 + threadIdx.x;
        const uint64_t pos = tbase + q;
        const bool mine = q < n && (a.count_only || pos < a.out_cap);
        if (mine) {
            const uint32_t slot = s_list[q];
            uint64_t i;
            if (tr.staged) {
                i = tr.r_lo + s_row[slot];
            } else {
                i = row_of(a.F, tr.r_lo, tr.r_hi, p0 + slot);
            }
            const uint32_t x = s_xv[slot];
            uint64_t f = 14695981039346656037ull;
            for (uint32_t u0 = 0; u0 < a.k; u0 += 8) {
                uint32_t val[8];
                // every load issued before any is used (no branch between them)
#pragma unroll
                for (uint32_t k4 = 0; k4 < 8; k4++) {
                    const uint32_t c = u0 + k4 < a.k ? s_qc[u0 + k4] : a.j;
                    const uint32_t mv = a.M[(uint64_t)(c < a.j ? c : 0u) * a.ldm + i];
                    val[k4] = c < a.j ? mv : x;
                }
#pragma unroll
                for (uint32_t k4 = 0; k4 < 8; k4++) {
                    const uint32_t u = u0 + k4;
                    if (u >= a.k) break;
                    if (stage) s_rows[threadIdx.x * a.k + u] = val[k4];
                    else if (!a.count_only) a.out[pos * a.k + u] = val[k4];
                    f = fnv_word(f, val[k4]);
                }
            }
            const uint64_t h = mix64(f);
            hs += h;
            hx ^= h;
        }
        if (stage) {
            __syncthreads();
            const uint64_t first = tbase + q0;
            uint64_t end = tbase + (q0 + QT < n ? q0 + QT : n);
            if (end > a.out_cap) end = a.out_cap;
            const uint32_t nw = first < end ? (uint32_t)(end - first) * a.k : 0u;
            uint32_t *dst = a.out + first * a.k;
            for (uint32_t t = threadIdx.x; t < nw; t += QT) dst[t] = s_rows[t];
            __syncthreads();
        }
    }
    const uint64_t sum = wave_sum(hs), xr = wave_xor(hx);
    if (lane == 0) {
        s_d[0][w] = sum;
        s_d[1][w] = xr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t ts = 0, tx = 0;
#pragma unroll
        for (int q = 0; q < QT / 64; q++) {
            ts += s_d[0][q];
            tx ^= s_d[1][q];
        }
        a.dig_part[2 * tile] = ts;
        a.dig_part[2 * tile + 1] = tx;
    }
}

// (sum, xor) over n pairs part[2i], part[2i+1]: one workgroup
__global__ __launch_bounds__(1024) void k_reduce_pairs(const uint64_t *part, uint64_t n, uint64_t *out, uint64_t *seqp,
                                                      uint64_t seqv) {
    __shared__ uint64_t s_s[16], s_x[16];
    uint64_t sm = 0, xr = 0;
    for (uint64_t i = threadIdx.x; i < n; i += 1024) {
        sm += part[2 * i];
        xr ^= part[2 * i + 1];
    }
    sm = wave_sum(sm);
    xr = wave_xor(xr);
    if (lane_id() == 0) {
        s_s[threadIdx.x >> 6] = sm;
        s_x[threadIdx.x >> 6] = xr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t ts = 0, tx = 0;
        for (int q = 0; q < 16; q++) {
            ts += s_s[q];
            tx ^= s_x[q];
        }
        out[0] = ts;
        out[1] = tx;
        post_seq(seqp, seqv);
    }
}

// rows of a one-column table (k = 1): copy out, per-workgroup partial digest
__global__ __launch_bounds__(QT) void k_emit_single(const uint32_t *M, uint64_t R, uint32_t *out, uint32_t count_only,
                                                   uint64_t *dig_part) {
    __shared__ uint64_t s_d[2][QT / 64];
    const uint64_t i = (uint64_t)blockIdx.x * QT + threadIdx.x;
    uint64_t h = 0;
    if (i < R) {
        uint32_t v = M[i];
        if (!count_only) out[i] = v;
        h = mix64(fnv_word(14695981039346656037ull, v));
    }
    uint64_t sum = wave_sum(h), xr = wave_xor(h);
    if (lane_id() == 0) {
        s_d[0][threadIdx.x >> 6] = sum;
        s_d[1][threadIdx.x >> 6] = xr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t ts = 0, tx = 0;
#pragma unroll
        for (int q = 0; q < QT / 64; q++) {
            ts += s_d[0][q];
            tx ^= s_d[1][q];
        }
        dig_part[2 * (uint64_t)blockIdx.x] = ts;
        dig_part[2 * (uint64_t)blockIdx.x + 1] = tx;
    }
}

static void reduce_pairs(gsi_ctx *c, const uint64_t *part, uint64_t n, uint64_t *out) {
    uint64_t seqv = 0;
    uint64_t *seqp = seq_slot(c, out, &seqv);
    launch(c, "k_reduce_pairs", 16.0 * n + 16.0, k_reduce_pairs, 1, 1024, part, n, out, seqp, seqv);
    c->seq_armed = seqp != nullptr;
}

// ---------------------------------------------------------------- planner
// Algorithm 2: the first vertex minimises |C(u)|/deg(u); afterwards the
// unplaced vertex adjacent to the placed ones with the least score, where
// every placement multiplies the scores of its neighbours by freq(l) =
// |E_l|/|E|.  Ties go to the smaller query vertex id.  First edge e0
// (Algorithm 4): the linking edge of least freq(l), ties to the placed end
// that was placed first.
void make_plan(const gsi_graph *g, const HostQuery &q, const std::vector<uint32_t> &cand,
               std::vector<uint32_t> &order, std::vector<uint32_t> &e0src) {
    const uint32_t k = q.k;
    order.clear();
    e0src.assign(k, NONE32);
    auto freq = [&](uint32_t l) -> double {
        if (l >= g->nlab || g->m == 0) return 0.0;
        return (double)g->edges[l] / (double)g->m;
    };
    if (k == 1) {
        order.push_back(0);
        return;
    }
    std::vector<double> score(k);
    for (uint32_t u = 0; u < k; u++) score[u] = (double)cand[u] / (double)q.adj[u].size();
    std::vector<uint8_t> placed(k, 0);
    std::vector<uint32_t> pos(k, NONE32);
    auto place = [&](uint32_t u) {
        pos[u] = (uint32_t)order.size();
        order.push_back(u);
        placed[u] = 1;
        for (auto &p : q.adj[u]) score[p.first] *= freq(p.second);
    };
    uint32_t first = 0;
    for (uint32_t u = 1; u < k; u++)
        if (score[u] < score[first]) first = u;
    place(first);
    while (order.size() < k) {
        uint32_t best = NONE32;
        for (uint32_t u = 0; u < k; u++) {
            if (placed[u]) continue;
            bool linked = false;
            for (auto &p : q.adj[u]) linked |= placed[p.first] != 0;
            if (!linked) continue;
            if (best == NONE32 || score[u] < score[best]) best = u;
        }
        uint32_t e0 = NONE32;
        double fbest = 0;
        for (auto &p : q.adj[best]) {
            if (!placed[p.first]) continue;
            double f = freq(p.second);
            if (e0 == NONE32 || f < fbest || (f == fbest && pos[p.first] < pos[e0])) {
                e0 = p.first;
                fbest = f;
            }
        }
        e0src[order.size()] = e0;
        place(best);
    }
}

// ---------------------------------------------------------------- driver
namespace {
struct Block {
    gsi_ctx *c;
    void *p = nullptr;
    explicit Block(gsi_ctx *cc) : c(cc) {}
    ~Block() { reset(); }
    void reset() {
        if (p) c->arena.release(p);
        p = nullptr;
    }
    template <typename T>
    T *get(uint64_t count, const char *what) {
        reset();
        uint64_t bytes = count * sizeof(T);
        p = c->arena.alloc(bytes ? bytes : 256, false);
        if (!p)
            fail(GSI_E_NOMEM, "arena exhausted allocating %llu bytes for %s (largest free block %llu)",
                 (unsigned long long)bytes, what, (unsigned long long)c->arena.largest_free());
        return static_cast<T *>(p);
    }
};
double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}
}  // namespace

gsi_result *run_query(gsi_graph *g, const HostQuery &q, const gsi_query_options *opt) {
    gsi_ctx *c = g->ctx;
    auto t0 = std::chrono::steady_clock::now();
    const uint32_t k = q.k;
    // join-step ablations (each replaces k_join by a variant with the same output)
    constexpr uint32_t JOIN_ABL = GSI_ABL_NAIVE_SETOPS | GSI_ABL_ROW_PER_WAVE | GSI_ABL_FOUR_LAYER;
    constexpr uint32_t ABL = GSI_ABL_CR | GSI_ABL_TWO_STEP | GSI_ABL_NO_STAGING | JOIN_ABL | GSI_ABL_DUP_REMOVAL;
    const uint32_t flags = (opt ? opt->flags : 0u) | ((opt && (opt->flags & ABL)) ? GSI_NO_FUSED : 0u);
    if (opt && (opt->flags & ~(GSI_COUNT_ONLY | GSI_FILTER_LABEL_ONLY | GSI_NO_FUSED | GSI_NO_CHUNKS |
                               GSI_LEVEL_FIRST_EDGE | GSI_HOMOMORPHISM | GSI_NO_LIST_FILTER | GSI_SINGLE_PASS |
                               ABL)))
        fail(GSI_E_INVALID, "unknown query flag");
    if (__builtin_popcount(flags & JOIN_ABL) > 1 || ((flags & JOIN_ABL) && (flags & GSI_ABL_TWO_STEP)))
        fail(GSI_E_INVALID, "at most one join ablation, and not with GSI_ABL_TWO_STEP");
    if ((flags & GSI_ABL_DUP_REMOVAL) && !(flags & (GSI_ABL_ROW_PER_WAVE | GSI_ABL_FOUR_LAYER)))
        fail(GSI_E_INVALID, "GSI_ABL_DUP_REMOVAL needs GSI_ABL_ROW_PER_WAVE or GSI_ABL_FOUR_LAYER");
    if ((flags & GSI_ABL_CR) && !g->cr_vid) fail(GSI_E_INVALID, "GSI_ABL_CR needs a graph loaded with GSI_GRAPH_KEEP_CR");
    const bool count_only = (flags & GSI_COUNT_ONLY) != 0;
    const bool homo = (flags & GSI_HOMOMORPHISM) != 0;
    // each row scans its shortest linking list unless the first edge is fixed
    const bool per_row = !(flags & GSI_LEVEL_FIRST_EDGE) && !(opt && opt->first_edge);
    // level-wide filtered first-edge lists; off for the paper's ablations
    const bool level_filter = !(flags & (GSI_NO_LIST_FILTER | ABL));
    const uint64_t max_rows = opt ? opt->max_rows : 0;

    std::vector<uint32_t> order, e0src;
    if (opt && opt->order) {
        order.assign(opt->order, opt->order + k);
        std::vector<uint8_t> seen(k, 0);
        for (uint32_t j = 0; j < k; j++) {
            if (order[j] >= k || seen[order[j]]) fail(GSI_E_INVALID, "order is not a permutation of 0..k-1");
            seen[order[j]] = 1;
            if (j == 0) continue;
            bool linked = false;
            for (auto &p : q.adj[order[j]])
                for (uint32_t i = 0; i < j; i++) linked |= p.first == order[i];
            if (!linked) fail(GSI_E_INVALID, "order[%u] has no edge to an earlier vertex", j);
        }
        if (opt->first_edge) {
            e0src.assign(opt->first_edge, opt->first_edge + k);
            for (uint32_t j = 1; j < k; j++) {
                bool ok = false;
                for (auto &p : q.adj[order[j]])
                    for (uint32_t i = 0; i < j; i++) ok |= (p.first == order[i] && p.first == e0src[j]);
                if (!ok) fail(GSI_E_INVALID, "first_edge[%u] is not a placed neighbour of order[%u]", j, j);
            }
        }
    } else if (opt && opt->first_edge) {
        fail(GSI_E_INVALID, "first_edge needs order");
    }

    // a result that never reaches the caller gives its rows back to the arena
    struct ResultGuard {
        gsi_result *r;
        ~ResultGuard() {
            if (r) {
                r->ctx->arena.release(r->rows);
                delete r;
            }
        }
        gsi_result *operator->() { return r; }
        gsi_result *release() {
            gsi_result *t = r;
            r = nullptr;
            return t;
        }
    } res{new gsi_result()};
    res->ctx = c;
    res->k = k;
    res->count_only = count_only;
    gsi_stats &st = res->stats;
    st.k = k;
    for (uint32_t j = 0; j < GSI_MAX_K; j++) st.order[j] = st.first_edge[j] = NONE32;

    auto finish = [&]() -> gsi_result * {
        st.total_ms = ms_since(t0);
        return res.release();
    };

    // a query edge whose label G lacks has no match
    for (uint32_t e = 0; e < q.el.size(); e++) {
        uint32_t l = q.el[e];
        if (l >= g->nlab || g->edges[l] == 0) return finish();
    }

    Scratch s(c);
    const uint64_t nwords = ((uint64_t)g->n + 63) / 64;
    uint64_t *bits = s.get<uint64_t>(nwords * k, "candidate bitsets");
    static_assert(MBOX_STATUS + sizeof(FStatus) / 8 <= MAILBOX_WORDS, "mailbox holds the fused status");
    // counts and level scalars go straight to the host mailbox
    uint32_t *dcnt = reinterpret_cast<uint32_t *>(c->mbox_dev + MBOX_COUNTS);
    uint64_t *dscal = c->mbox_dev + MBOX_SCALARS;
    auto tf = std::chrono::steady_clock::now();
    uint32_t *druns = s.get<uint32_t>((uint64_t)k * BITS_RUNS, "candidate run counts");
    filter_impl(g, q, (flags & GSI_FILTER_LABEL_ONLY) != 0, bits, dcnt, homo, druns);
    std::vector<uint32_t> cand(k);
    {
        uint64_t tmp[GSI_MAX_K / 2 + 1];
        read_scalars(c, reinterpret_cast<const uint64_t *>(dcnt), tmp, (int)((k + 1) / 2));
        memcpy(cand.data(), tmp, 4ull * k);
    }
    st.filter_ms = ms_since(tf);
    for (uint32_t u = 0; u < k; u++) st.cand[u] = cand[u];
    for (uint32_t u = 0; u < k; u++)
        if (cand[u] == 0) return finish();

    if (order.empty()) make_plan(g, q, cand, order, e0src);
    if (e0src.empty()) {
        // order given without first edges: least freq(l), earliest placed end
        e0src.assign(k, NONE32);
        for (uint32_t j = 1; j < k; j++) {
            double fb = 0;
            for (uint32_t i = 0; i < j; i++)
                for (auto &p : q.adj[order[j]])
                    if (p.first == order[i]) {
                        double f = (double)g->edges[p.second] / (double)g->m;
                        if (e0src[j] == NONE32 || f < fb) {
                            e0src[j] = order[i];
                            fb = f;
                        }
                    }
        }
    }
    for (uint32_t j = 0; j < k; j++) {
        st.order[j] = order[j];
        st.first_edge[j] = e0src[j];
    }
    std::vector<uint32_t> col(k, NONE32);
    for (uint32_t j = 0; j < k; j++) col[order[j]] = j;

    auto tj = std::chrono::steady_clock::now();

    // M0 = C(order[0]), ascending.  When the single fused workgroup will run
    // the levels, it writes M0 itself (saving three launches).
    uint64_t R = cand[order[0]];
    if (max_rows && R > max_rows) fail(GSI_E_CAPACITY, "rows exceed max_rows");
    Block Mb(c);
    uint32_t *M = Mb.get<uint32_t>(R, "first table");
    const uint64_t *b0 = bits + (uint64_t)order[0] * nwords;
    uint32_t fcap_rows = FUSED_MAX_ROWS, fcap_slots = FUSED_MAX_SLOTS;
    if (opt && opt->fused_max_rows) fcap_rows = std::min(fcap_rows, opt->fused_max_rows);
    if (opt && opt->fused_max_slots) fcap_slots = std::min(fcap_slots, opt->fused_max_slots);
    const uint32_t chunk_min = (opt && opt->chunk_min_rows) ? opt->chunk_min_rows : CHUNK_MIN_ROWS;
    const bool try_chunks = !(flags & GSI_NO_FUSED) && !(flags & GSI_NO_CHUNKS) && R >= chunk_min;
    const bool m0_in_fused = k >= 2 && !try_chunks && !(flags & GSI_NO_FUSED) && R <= fcap_rows &&
                             fcap_slots >= 64 && nwords <= M0_FUSED_MAX_WORDS;
    if (!m0_in_fused) {
        Scratch s0(c);
        uint32_t *wc = s0.get<uint32_t>(nwords, "word counts");
        uint64_t *wo = s0.get<uint64_t>(nwords + 1, "word offsets");
        launch(c, "k_word_popc", 8.0 * nwords, k_word_popc, nblocks(nwords), QT, b0, nwords, wc);
        exclusive_scan(c, wc, nwords, wo, s0);
        launch(c, "k_word_emit", 16.0 * nwords + 4.0 * R, k_word_emit, nblocks(nwords), QT, b0, nwords, (const uint64_t *)wo, M);
    }
    st.rows[0] = R;

    if (k == 1) {
        uint32_t *out = count_only ? nullptr : persist<uint32_t>(c, R, "result rows");
        res->rows = out;
        uint64_t nb = nblocks(R);
        uint64_t *dpart = s.get<uint64_t>(2 * nb, "digest partials");
        launch(c, "k_emit_single", 8.0 * R, k_emit_single, (uint32_t)nb, QT, M, R, out, count_only ? 1u : 0u, dpart);
        reduce_pairs(c, dpart, nb, dscal);
        uint64_t dg[2];
        read_scalars(c, dscal, dg, 2);
        res->rows = out;
        res->count = R;
        res->digest[0] = dg[0];
        res->digest[1] = dg[1];
        st.join_ms = ms_since(tj);
        return finish();
    }

    // Fused plan (device copy of the levels' linking edges) for the fused
    // kernels, written into the pinned staging buffer and uploaded.
    Scratch fs(c);
    // With `inl`, a plan of at most FPLAN_ARG_EDGES edges is copied there (it
    // travels as a kernel argument) and nullptr is returned instead of a
    // device copy.
    auto fused_plan = [&](uint32_t cap_rows, uint32_t cap_slots, FPlan **host, FPlanArg *inl = nullptr) -> FPlan * {
        uint32_t n_edges = 0;
        for (uint32_t j = 1; j < k; j++)
            for (uint32_t i = 0; i < j; i++)
                for (auto &p : q.adj[order[j]]) n_edges += p.first == order[i];
        const size_t pb = fplan_bytes(n_edges);
        if (pb > 56 * 1024) fail(GSI_E_INTERNAL, "query plan too large for the staging buffer");
        FPlan *hp = reinterpret_cast<FPlan *>(reinterpret_cast<char *>(c->pinned) + 8192);
        memset(hp, 0, pb);
        hp->k = k;
        hp->count_only = count_only ? 1u : 0u;
        hp->cap_rows = cap_rows;
        hp->cap_slots = cap_slots;
        hp->pick = per_row ? 1u : 0u;
        hp->homo = homo ? 1u : 0u;
        hp->ci_all = g->ci;
        for (uint32_t v = 0; v < k; v++) hp->qcol[v] = col[v];
        uint32_t ei = 0;
        for (uint32_t j = 1; j < k; j++) {
            hp->lv_first[j] = ei;
            hp->Cu[j] = bits + (uint64_t)order[j] * nwords;
            uint32_t ne = 0;
            for (uint32_t i = 0; i < j; i++)
                for (auto &p : q.adj[order[j]])
                    if (p.first == order[i]) {
                        const uint32_t l = p.second;
                        FEdge &fe = hp->edges[ei + ne];
                        fe.gl = g->gl + g->group_base[l] * GROUP_WORDS;
                        fe.ci = g->ci + g->ci_base[l];
                        fe.G = g->G[l];
                        fe.H = g->H[l];
                        fe.col = i;
                        fe.ci_off = (uint32_t)g->ci_base[l];
                        if (order[i] == e0src[j]) hp->lv_e0[j] = ne;
                        ne++;
                    }
            hp->lv_ne[j] = ne;
            hp->lv_mmask[j] = 0;
            for (uint32_t c = 0; c < j; c++)
                if (q.multi || q.vl[order[c]] == q.vl[order[j]]) hp->lv_mmask[j] |= 1u << c;
            st.n_link[j] = ne;
            ei += ne;
        }
        *host = hp;
        if (inl && n_edges <= FPLAN_ARG_EDGES) {
            memcpy(inl, hp, pb);
            return nullptr;
        }
        FPlan *dplan = reinterpret_cast<FPlan *>(fs.get<uint8_t>(pb, "fused plan"));
        GSI_HIP(hipMemcpyAsync(dplan, hp, pb, hipMemcpyHostToDevice, c->stream));
        return dplan;
    };
    // algorithmic bytes of a fused launch, from the per-level sizes it met
    auto fused_bytes = [&](const FPlan *hp, uint32_t last, const uint64_t *rows, const uint64_t *gbas,
                           const uint64_t *survs) {
        double b = 0;
        for (uint32_t j = 1; j <= last && j < k; j++) {
            double Rj = (double)rows[j], Gj = (double)gbas[j], Sj = (double)survs[j];
            double ne = hp->lv_ne[j];
            b += Rj * (4.0 * ne + 128.0 * ne + 8.0 * ne + 4.0 * j) + 4.0 * Gj + Sj * (4.0 + 4.0 * j + 4.0 * (j + 1));
        }
        return b;
    };

    // Root chunks: a persistent launch runs all levels of small groups of
    // root rows, one chunk per workgroup at a time, over the whole chip.
    // Chunks that do not fit are finished by the per-level kernels below on
    // their roots only; both parts are merged at the end.
    struct ChunkPart {
        bool active = false, merged = false;
        uint32_t n = 0;
        uint64_t count = 0, digest[2] = {0, 0};
        const FStatus *sts = nullptr;
        const uint64_t *offs = nullptr;
        const uint32_t *staging = nullptr;
        uint64_t rows[GSI_MAX_K] = {0}, gba[GSI_MAX_K] = {0}, surv[GSI_MAX_K] = {0};
        uint32_t levels = 0;
    } cp;
    Scratch cs(c);
    // adds the chunk part to the result; `front` (if any) already has room
    // for the chunk rows before the per-level rows
    auto merge_chunks = [&](uint32_t *front) {
        if (!cp.active || cp.merged) return;
        cp.merged = true;
        if (!count_only && cp.count) {
            if (!front) {
                front = persist<uint32_t>(c, cp.count * k, "result rows");
                res->rows = front;
            }
            launch_chunk_gather(c, cp.n, cp.sts, cp.offs, cp.staging, k, front, cp.count * k);
        }
        res->count += cp.count;
        res->digest[0] += cp.digest[0];
        res->digest[1] ^= cp.digest[1];
        for (uint32_t j = 1; j < k; j++) {
            st.rows[j] += cp.rows[j];
            st.gba[j] += cp.gba[j];
            st.survivors[j] += cp.surv[j];
        }
        st.levels = std::max(st.levels, cp.levels);
        sync(c);
    };
    auto done = [&]() -> gsi_result * {
        merge_chunks(nullptr);
        return finish();
    };

    // Runs the chunks from level j0 on M (R rows, j0 columns, column stride
    // R).  Returns 0 when they could not be set up (M unchanged), 1 when
    // every chunk finished (the result is complete), 2 when some did not:
    // M and R then hold those chunks' rows, for the per-level kernels.
    auto run_chunks = [&](uint32_t j0) -> int {
        const FTier t = fused_tier(256);
        const uint64_t slot_words = 2ull * t.cap_rows * k + fused_loc_words(k, t.cap_rows);
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || ncu < 1)
            ncu = 1;
        const uint64_t room = c->arena.largest_free() / 4;
        uint64_t grid = std::min<uint64_t>((uint64_t)t.blocks_per_cu * ncu, room / (slot_words * 4));
        uint64_t target = std::min<uint64_t>(std::max<uint64_t>(4 * grid, 1), CHUNK_MAX);
        if (opt && opt->chunk_rows) target = (R + opt->chunk_rows - 1) / opt->chunk_rows;
        // a chunk's first table must fit the workgroup's row capacity
        const uint32_t chunk_rows =
            (uint32_t)std::min<uint64_t>(t.cap_rows, std::max<uint64_t>(1, (R + target - 1) / target));
        const uint32_t nchunks = (uint32_t)((R + chunk_rows - 1) / chunk_rows);
        grid = std::min<uint64_t>(grid, nchunks);
        const uint64_t ocap = count_only ? 0
                                         : std::min<uint64_t>((uint64_t)nchunks * t.cap_slots * k,
                                                              c->arena.largest_free() / 32);
        if (!(grid >= 1 && nchunks <= CHUNK_MAX && (count_only || ocap >= 1024))) return 0;
        FPlan *hp;
        FPlan *dplan = fused_plan(0xFFFFFFFFu, 0xFFFFFFFFu, &hp);
        uint32_t *slots = cs.get<uint32_t>(slot_words * grid, "chunk tables");
        FStatus *sts = reinterpret_cast<FStatus *>(cs.get<uint64_t>((uint64_t)nchunks * sizeof(FStatus) / 8,
                                                                    "chunk status"));
        uint64_t *offs = cs.get<uint64_t>((uint64_t)nchunks + 1, "chunk offsets");
        uint32_t *dflags = cs.get<uint32_t>(nchunks, "chunk done flags");
        // one zeroed block: counters (next chunk, abort, failures), the
        // output counter and the summary
        const uint64_t zwords = 3 + sizeof(FChunkSummary) / 8;
        uint64_t *zb = cs.get<uint64_t>(zwords, "chunk counters");
        uint32_t *ctr = reinterpret_cast<uint32_t *>(zb);
        unsigned long long *ocount = reinterpret_cast<unsigned long long *>(zb + 2);
        FChunkSummary *dsum = reinterpret_cast<FChunkSummary *>(zb + 3);
        uint32_t *staging = count_only ? nullptr : cs.get<uint32_t>(ocap, "chunk rows");
        fill_u64(c, reinterpret_cast<uint64_t *>(sts), 0, (uint64_t)nchunks * sizeof(FStatus) / 8);
        fill_u64(c, zb, 0, zwords);
        const uint32_t max_fail = std::max<uint32_t>(16, nchunks / 8);
        const size_t ri = c->recs.size();
        launch_fused_chunks(c, t, (uint32_t)grid, dplan, j0, M, (uint32_t)R, chunk_rows, nchunks, slots, slot_words,
                            k, staging, ocap, ocount, ctr + 1, max_fail, sts, ctr, offs, dflags, dsum);
        FChunkSummary *hsum = reinterpret_cast<FChunkSummary *>(reinterpret_cast<char *>(c->pinned) + 4096);
        GSI_HIP(hipMemcpyAsync(hsum, dsum, sizeof(FChunkSummary), hipMemcpyDeviceToHost, c->stream));
        sync(c);
        if ((c->flags & GSI_CTX_PROFILE) && ri < c->recs.size())
            c->recs[ri].bytes = fused_bytes(hp, (uint32_t)hsum->levels, hsum->lv_rows, hsum->lv_gba,
                                            hsum->lv_surv);
        cp.active = true;
        cp.n = nchunks;
        cp.count = hsum->count;
        cp.digest[0] = hsum->digest[0];
        cp.digest[1] = hsum->digest[1];
        cp.sts = sts;
        cp.offs = offs;
        cp.staging = staging;
        cp.levels = (uint32_t)hsum->levels;
        for (uint32_t j = 1; j < k; j++) {
            cp.rows[j] = hsum->lv_rows[j];
            cp.gba[j] = hsum->lv_gba[j];
            cp.surv[j] = hsum->lv_surv[j];
        }
        st.chunks = nchunks;
        if (hsum->all_done) {
            if (!count_only && cp.count) {
                uint32_t *out = persist<uint32_t>(c, cp.count * k, "result rows");
                res->rows = out;
                merge_chunks(out);
            } else {
                merge_chunks(nullptr);
            }
            st.join_ms = ms_since(tj);
            return 1;
        }
        // the rows of the chunks left undone continue level by level
        std::vector<uint32_t> fl(nchunks);
        GSI_HIP(hipMemcpyAsync(fl.data(), dflags, 4ull * nchunks, hipMemcpyDeviceToHost, c->stream));
        sync(c);
        std::vector<uint32_t> list;
        uint64_t left = 0;
        for (uint32_t ch = 0; ch < nchunks; ch++) {
            if (fl[ch]) continue;
            list.push_back(ch);
            list.push_back((uint32_t)left);
            left += std::min<uint64_t>(chunk_rows, R - (uint64_t)ch * chunk_rows);
        }
        st.chunks_left = (uint32_t)(list.size() / 2);
        uint32_t *dl = cs.get<uint32_t>(list.size(), "chunks left");
        GSI_HIP(hipMemcpyAsync(dl, list.data(), 4 * list.size(), hipMemcpyHostToDevice, c->stream));
        Block Mr(c);
        uint32_t *Mleft = Mr.get<uint32_t>(left * j0, "rows left");
        launch_take_rows(c, (uint32_t)(list.size() / 2), M, (uint32_t)R, j0, chunk_rows, dl, Mleft, left);
        sync(c);  // `list` is read by the copy above
        Mb.reset();
        Mb.p = Mr.p;
        Mr.p = nullptr;
        M = Mleft;
        R = left;
        return 2;
    };

    uint32_t jstart = 1;
    if (try_chunks && run_chunks(1) == 1) return finish();

    // One workgroup runs levels j0.. of M (R rows, j0 columns) while they
    // fit.  Returns true when it finished the query (the result is
    // complete); otherwise M and R hold the input of the level it stopped
    // at, returned in `stop`.
    const uint32_t cap_rows = fcap_rows, cap_slots = fcap_slots;
    FPlan *fhp = nullptr, *fdplan = nullptr;
    std::unique_ptr<FPlanArg> finl;  // the plan as a kernel argument, when it fits
    uint32_t *fbuf0 = nullptr, *fbuf1 = nullptr, *floc = nullptr;
    FStatus *fdst = nullptr;
    auto run_fused = [&](uint32_t j0, const uint64_t *root_bits, uint32_t &stop) -> bool {
        if (!fhp) {
            finl.reset(new FPlanArg());
            fdplan = fused_plan(cap_rows, cap_slots, &fhp, finl.get());
            fbuf0 = fs.get<uint32_t>((uint64_t)cap_rows * k, "fused table 0");
            fbuf1 = fs.get<uint32_t>((uint64_t)cap_rows * k, "fused table 1");
            floc = fs.get<uint32_t>(fused_loc_words(k, cap_rows), "fused lookups");
            fdst = reinterpret_cast<FStatus *>(c->mbox_dev + MBOX_STATUS);
        }
        uint32_t *out = count_only ? nullptr : persist<uint32_t>(c, (uint64_t)cap_slots * k, "result rows");
        res->rows = out;
        launch_fused(c, fdplan, *finl, j0, M, (uint32_t)R, druns + (uint64_t)order[0] * BITS_RUNS, root_bits, nwords,
                     fbuf0, fbuf1, floc, out, fdst, 0.0);
        const size_t frec = c->recs.size();  // the fused launch's record (the wait may add one)
        FStatus *hs = reinterpret_cast<FStatus *>(c->mbox_host + MBOX_STATUS);
        wait_mailbox(c);
        const uint32_t last = hs->done ? (uint32_t)hs->levels : (uint32_t)hs->level;
        if ((c->flags & GSI_CTX_PROFILE) && frec > 0 && frec <= c->recs.size())
            // plus, when it builds M0 itself, the root's candidate bitset it
            // scans and the rows it writes
            c->recs[frec - 1].bytes = fused_bytes(fhp, last, hs->lv_rows, hs->lv_gba, hs->lv_surv) +
                                      (root_bits ? 8.0 * (double)nwords + 4.0 * (double)R : 0.0);
        for (uint32_t j = j0; j <= last && j < k; j++) {
            st.rows[j] = hs->lv_rows[j];
            st.gba[j] = hs->lv_gba[j];
            st.survivors[j] = hs->lv_surv[j];
        }
        if (hs->done) {
            st.levels = (uint32_t)hs->levels;
            res->count = hs->count;
            res->digest[0] = hs->digest[0];
            res->digest[1] = hs->digest[1];
            if (out && hs->count == 0) {
                c->arena.release(out);
                res->rows = nullptr;
            } else if (out) {
                c->arena.shrink(out, hs->count * k * 4);
            }
            st.join_ms = ms_since(tj);
            return true;
        }
        if (out) c->arena.release(out);
        res->rows = nullptr;
        stop = (uint32_t)hs->level;
        R = hs->rows;
        if (hs->mloc == 0) M = fbuf0;
        else if (hs->mloc == 1) M = fbuf1;
        return false;
    };
    const bool fused_ok = !(flags & GSI_NO_FUSED) && cap_slots >= 64;

    // Small root sets: the workgroup starts; the per-level kernels continue
    // from where it stopped, and hand the query back to it once the table
    // fits again.
    if (!cp.active && fused_ok && R <= cap_rows) {
        if (run_fused(1, m0_in_fused ? b0 : nullptr, jstart)) return finish();
    }
    uint32_t fused_stuck = NONE32;  // level at which the workgroup last stopped without progress
    // column stride of M when a one-pass level wrote it at its capacity (0: R)
    uint64_t Mld = 0;

    for (uint32_t j = jstart; j < k; j++) {
        const uint32_t u = order[j];
        const bool final_level = (j == k - 1);
        st.rows[j] = R;
        LevelArgs a;
        memset(&a, 0, sizeof(a));
        a.M = M;
        a.R = R;
        a.ldm = Mld ? Mld : R;
        a.j = j;
        a.k = k;
        a.Cu = bits + (uint64_t)u * nwords;
        uint32_t ne = 0;
        uint32_t elab[GSI_MAX_K] = {0};  // label of each linking edge
        for (uint32_t i = 0; i < j; i++)
            for (auto &p : q.adj[u])
                if (p.first == order[i]) {
                    uint32_t l = p.second;
                    EdgeRef &er = a.e[ne];
                    er.gl = g->gl + g->group_base[l] * GROUP_WORDS;
                    er.ci = g->ci + g->ci_base[l];
                    er.G = g->G[l];
                    er.H = g->H[l];
                    er.col = i;
                    er.ci_off = (uint32_t)g->ci_base[l];
                    if (g->cr_vid) {
                        er.cr_vid = g->cr_vid + g->group_base[l];
                        er.cr_start = g->cr_start + g->group_base[l];
                        er.cr_off = g->cr_off + g->group_base[l];
                    }
                    er.cr_end = (uint32_t)(g->ci_base[l] + 2 * g->edges[l]);
                    elab[ne] = l;
                    if (order[i] == e0src[j]) a.e0 = ne;
                    ne++;
                }
        a.ne = ne;
        st.n_link[j] = ne;
        {
            uint32_t ord[GSI_MAX_K];
            for (uint32_t e = 0; e < ne; e++) ord[e] = e;
            std::stable_sort(ord, ord + ne, [&](uint32_t x, uint32_t y) { return g->edges[elab[x]] < g->edges[elab[y]]; });
            for (uint32_t e = 0; e < ne; e++) a.eorder[e] = ord[e];
        }
        for (uint32_t v = 0; v < k; v++) a.qcol[v] = col[v];
        // columns of m_i the subtraction has to look at
        for (uint32_t c = 0; c < j; c++)
            if (q.multi || q.vl[order[c]] == q.vl[u]) a.mcol[a.nmc++] = c;
        a.final_level = final_level ? 1u : 0u;
        a.count_only = count_only ? 1u : 0u;

        Scratch ls(c);
        a.ci_all = g->ci;
        a.pick = per_row ? 1u : 0u;
        a.homo = homo ? 1u : 0u;
        a.abl_cr = (flags & GSI_ABL_CR) ? 1u : 0u;
        a.abl_two_step = (flags & GSI_ABL_TWO_STEP) ? 1u : 0u;
        a.abl_no_stage = (flags & GSI_ABL_NO_STAGING) ? 1u : 0u;
        a.loc = ls.get<uint32_t>((2ull * ne + 2) * R, "located lists");
        a.bound = ls.get<uint32_t>(R, "row bounds");
        uint64_t *F = ls.get<uint64_t>(R + 1, "offsets F");
        a.F = F;
        const uint64_t nbr = nblocks(R);
        const bool prof = (c->flags & GSI_CTX_PROFILE) != 0;
        a.part = prof ? ls.get<uint64_t>(2 * nbr, "locate partials") : nullptr;
        // the streamed bytes: row values read, located lists, bound and F
        // written.  The 128 B PCSR groups are not counted: rows repeat few
        // distinct vertices, so all but the first read of a group hit L2
        // (counting every read, or every group of the label, gives rates
        // above what HBM can deliver).
        const double lbytes = (double)R * (4.0 * ne + 4.0 * (2.0 * ne + 2.0) + 4.0 + 8.0);
        // one workgroup's worth of rows: k_locate scans F itself
        const bool one_wg = nbr == 1;
        if (one_wg) {
            a.scan_total = dscal + 3;
            a.seq_slot = seq_slot(c, a.scan_total, &a.seq_value);
        }
        launch(c, "k_locate", lbytes, k_locate, (uint32_t)nbr, QT, a);
        if (one_wg) c->seq_armed = a.seq_slot != nullptr;
        a.scan_total = a.seq_slot = nullptr;
        // |GBA| lands in dscal[3]; the profiling sums go to dscal[4..5]
        if (prof) reduce_pairs(c, a.part, nbr, dscal + 4);
        if (!one_wg) exclusive_scan(c, a.bound, R, F, ls, dscal + 3);
        uint64_t sc[2];
        read_scalars(c, dscal + 3, sc, 2);
        uint64_t gba = sc[0];
        sc[0] = prof ? sc[1] : 0;
        // a level whose rows rescan l0's lists many times over: filter those
        // lists by C(u) once and let the rows scan the filtered copies
        Block fnb(c);
        if (level_filter && gba) {
            const uint32_t l0 = elab[a.e0];
            const uint64_t El = 2 * g->edges[l0];
            if (El && (double)gba > FN_FACTOR * (double)El && El < 0xFFFFFFFFull) {
                const uint64_t nw = (El + 63) / 64;
                uint64_t *fbits = ls.get<uint64_t>(nw, "filtered-list bits");
                uint32_t *wcnt = ls.get<uint32_t>(nw, "filtered-list word counts");
                uint64_t *wpre = ls.get<uint64_t>(nw + 1, "filtered-list word offsets");
                const uint32_t *ci_l0 = a.e[a.e0].ci;
                launch(c, "k_fn_bits", 4.0 * El + El / 8.0 + 4.0 * nw, k_fn_bits, nblocks(El, QT * FN_TILES), QT,
                       ci_l0, El, a.Cu,
                       fbits, wcnt);
                exclusive_scan(c, wcnt, nw, wpre, ls, dscal + 3);
                uint64_t kept;
                read_scalars(c, dscal + 3, &kept, 1);
                uint32_t *fn = fnb.get<uint32_t>(kept ? kept : 1, "filtered lists");
                launch(c, "k_fn_compact", 4.0 * El + El / 8.0 + 8.0 * nw + 4.0 * kept, k_fn_compact, nblocks(El), QT,
                       ci_l0, El, (const uint64_t *)fbits, (const uint64_t *)wpre, fn);
                launch(c, "k_fn_relocate", (double)R * (8.0 + 4.0 + 8.0 + 32.0), k_fn_relocate, (uint32_t)nbr, QT, a,
                       (const uint64_t *)fbits, (const uint64_t *)wpre);
                exclusive_scan(c, a.bound, R, F, ls, dscal + 3);
                read_scalars(c, dscal + 3, &gba, 1);
                a.ci_all = fn;
                a.prefiltered = 1;
                st.filtered_levels |= 1u << j;
            }
        }
        st.gba[j] = gba;
        st.other_elems[j] = sc[0];
        st.levels = j;
        if (gba == 0) {
            st.survivors[j] = 0;
            return done();
        }
        a.gba = gba;
        const uint32_t spt = gba >= WIDE_TILE_SLOTS ? 4u : 1u;
        const uint32_t ts = spt * QT;
        const uint64_t ntiles = (gba + ts - 1) / ts;
        // The last level in one pass (join, look-back, rows) when the output
        // can be sized at |GBA| rows, its survivors' upper bound.
        const uint64_t before_rows = (cp.active && !cp.merged) ? cp.count : 0;
        const bool single_pass = final_level && (flags & GSI_SINGLE_PASS) && !(flags & ABL) &&
                                 (count_only || (gba + before_rows) * k * 4 <= c->arena.largest_free() / 2);
        if (single_pass) {
            uint64_t *trow = ls.get<uint64_t>(ntiles + 1, "tile rows");
            a.tile_row = trow;
            launch(c, "k_tile_rows", 8.0 * (R + 1) + 8.0 * (ntiles + 1), k_tile_rows, nblocks(R), QT,
                   (const uint64_t *)F, R, ntiles, ts, trow);
            // look-back status words, then [tile counter, failure flag] and the total
            uint64_t *lbw = ls.get<uint64_t>(ntiles + 2, "look-back words");
            fill_u64(c, lbw, 0, ntiles + 2);
            a.tstat = reinterpret_cast<unsigned long long *>(lbw);
            a.tctr = reinterpret_cast<uint32_t *>(lbw + ntiles);
            a.total = lbw + ntiles + 1;
            a.dig_part = ls.get<uint64_t>(2 * ntiles, "digest partials");
            uint32_t *front = nullptr;
            if (!count_only) {
                front = persist<uint32_t>(c, (gba + before_rows) * k, "result rows");
                a.out = front + before_rows * k;
                res->rows = front;
            }
            a.out_cap = count_only ? 0 : gba;
            // join bytes, plus the rows written and the row values they read
            const double jb = 4.0 * gba + (double)R * (8.0 + 8.0 * ne + 4.0 * j) + 4.0 * (double)sc[0] + 16.0 * ntiles;
            if (spt == 4) launch(c, "k_join_last", jb, k_join_pass<4, true>, (uint32_t)ntiles, QT, a);
            else launch(c, "k_join_last", jb, k_join_pass<1, true>, (uint32_t)ntiles, QT, a);
            uint64_t tw[2];
            read_scalars(c, lbw + ntiles, tw, 2);
            if (tw[0] >> 32) fail(GSI_E_INTERNAL, "look-back of the last level did not complete");
            const uint64_t S = tw[1];
            st.survivors[j] = S;
            if ((c->flags & GSI_CTX_PROFILE) && !c->recs.empty())
                c->recs.back().bytes = jb + (count_only ? 0.0 : 4.0 * k * S) + 4.0 * j * S;
            if (max_rows && S > max_rows) fail(GSI_E_CAPACITY, "rows exceed max_rows at level %u", j);
            reduce_pairs(c, a.dig_part, ntiles, dscal);
            uint64_t dg[2];
            read_scalars(c, dscal, dg, 2);
            if (front) {
                if (S + before_rows == 0) {
                    c->arena.release(front);
                    front = nullptr;
                } else {
                    c->arena.shrink(front, (S + before_rows) * k * 4);
                }
            }
            res->rows = front;
            res->count = S;
            res->digest[0] = dg[0];
            res->digest[1] = dg[1];
            merge_chunks(front);
            st.join_ms = ms_since(tj);
            return finish();
        }
        // An inner level in one pass too, when its rows scan filtered lists
        // and have one linking edge (nearly every slot survives, so the
        // next table, written at |GBA| rows per column, wastes little).
        const bool inner_pass = !final_level && a.prefiltered && ne == 1 && (flags & GSI_SINGLE_PASS) &&
                                !(flags & ABL) &&
                                (uint64_t)(j + 1) * gba * 4 <= c->arena.largest_free() / 2;
        if (inner_pass) {
            uint64_t *trow = ls.get<uint64_t>(ntiles + 1, "tile rows");
            a.tile_row = trow;
            launch(c, "k_tile_rows", 8.0 * (R + 1) + 8.0 * (ntiles + 1), k_tile_rows, nblocks(R), QT,
                   (const uint64_t *)F, R, ntiles, ts, trow);
            uint64_t *lbw = ls.get<uint64_t>(ntiles + 2, "look-back words");
            fill_u64(c, lbw, 0, ntiles + 2);
            a.tstat = reinterpret_cast<unsigned long long *>(lbw);
            a.tctr = reinterpret_cast<uint32_t *>(lbw + ntiles);
            a.total = lbw + ntiles + 1;
            Block Mn(c);
            a.Mn = Mn.get<uint32_t>((uint64_t)(j + 1) * gba, "next table");
            a.out_cap = gba;
            const double jb = 4.0 * gba + (double)R * (8.0 + 8.0 * ne + 4.0 * j) + 16.0 * ntiles;
            if (spt == 4) launch(c, "k_join_pass", jb, k_join_pass<4, false>, (uint32_t)ntiles, QT, a);
            else launch(c, "k_join_pass", jb, k_join_pass<1, false>, (uint32_t)ntiles, QT, a);
            uint64_t tw[2];
            read_scalars(c, lbw + ntiles, tw, 2);
            if (tw[0] >> 32) fail(GSI_E_INTERNAL, "look-back of level %u did not complete", j);
            const uint64_t S = tw[1];
            st.survivors[j] = S;
            if ((c->flags & GSI_CTX_PROFILE) && !c->recs.empty())
                c->recs.back().bytes = jb + 4.0 * (j + 1) * S + 4.0 * j * S;
            if (S == 0) return done();
            if (max_rows && S > max_rows) fail(GSI_E_CAPACITY, "rows exceed max_rows at level %u", j);
            Mb.reset();
            Mb.p = Mn.p;
            Mn.p = nullptr;
            M = a.Mn;
            Mld = gba;
            R = S;
            continue;  // the fused workgroup is not taken back after a one-pass level
        }
        // survivors as (element, row) records when they fit comfortably
        // (8 bytes per |GBA| slot), else as a keep bitmap (and always for the
        // join ablations, which write the bitmap)
        const bool recs = !(flags & ABL) && 8.0 * (double)(ntiles * ts) <= (double)c->arena.largest_free() / 4;
        a.rec_x = a.rec_r = nullptr;
        a.bitmap = nullptr;
        if (recs) {
            a.rec_x = ls.get<uint32_t>(ntiles * ts, "survivor elements");
            a.rec_r = ls.get<uint32_t>(ntiles * ts, "survivor rows");
        } else {
            a.bitmap = ls.get<uint64_t>(ntiles * (ts / 64), "GBA bitmap");
        }
        a.tile_cnt = ls.get<uint32_t>(ntiles, "tile counts");
        uint64_t *toff = ls.get<uint64_t>(ntiles + 1, "tile offsets");
        a.tile_off = toff;
        uint64_t *trow = ls.get<uint64_t>(ntiles + 1, "tile rows");
        a.tile_row = trow;
        // at most 256 rows: the join finds its tiles' rows in F itself
        const bool rows_in_join = nbr == 1 && !(flags & JOIN_ABL);
        if (!rows_in_join)
            launch(c, "k_tile_rows", 8.0 * (R + 1) + 8.0 * (ntiles + 1), k_tile_rows, nblocks(R), QT,
                   (const uint64_t *)F, R, ntiles, ts, trow);
        double jb = 4.0 * gba + (double)R * (8.0 + 8.0 * ne + 4.0 * j) + 4.0 * (double)sc[0] + gba / 8.0 + 4.0 * ntiles;
        a.rows_in_join = rows_in_join ? 1u : 0u;
        if (flags & JOIN_ABL) run_join_ablation(c, a, flags, ntiles, ts, jb, ls);
        else if (spt == 4) launch(c, "k_join", jb, k_join<4>, (uint32_t)ntiles, QT, a);
        else launch(c, "k_join", jb, k_join<1>, (uint32_t)ntiles, QT, a);
        a.rows_in_join = 0;
        const size_t join_rec = c->recs.size();
        exclusive_scan(c, a.tile_cnt, ntiles, toff, ls, dscal + 1);
        uint64_t S;
        read_scalars(c, dscal + 1, &S, 1);
        st.survivors[j] = S;
        // the join wrote 8 bytes per survivor, not the keep bitmap
        if (recs && (c->flags & GSI_CTX_PROFILE) && join_rec > 0 && join_rec <= c->recs.size())
            c->recs[join_rec - 1].bytes += 8.0 * S - gba / 8.0;
        if (S == 0) return done();
        if (max_rows && S > max_rows) fail(GSI_E_CAPACITY, "rows exceed max_rows at level %u", j);
        a.S = S;
        Block Mn(c);
        // the link reads each survivor's record (or re-reads its element and
        // the keep bitmap) and its parent row's j values
        double lb = recs ? (double)S * (8.0 + 4.0 * j) + 8.0 * ntiles
                         : (double)S * (4.0 + 4.0 * j) + gba / 8.0 + 8.0 * ntiles;
        uint32_t *front = nullptr;  // room for the chunk part's rows
        if (final_level) {
            if (!count_only) {
                const uint64_t before = (cp.active && !cp.merged) ? cp.count : 0;
                front = persist<uint32_t>(c, (S + before) * k, "result rows");
                a.out = front + before * k;
                res->rows = front;
                lb += 4.0 * k * S;
            }
            a.dig_part = ls.get<uint64_t>(2 * ntiles, "digest partials");
        } else {
            a.Mn = Mn.get<uint32_t>((uint64_t)(j + 1) * S, "next table");
            lb += 4.0 * (j + 1) * S;
        }
        if (recs) {
            // values a row gathers, in groups of 4 (0: more than 16)
            const uint32_t width = final_level ? k : j;
            const uint32_t wg = width <= 16 ? (width + 3) / 4 : 0;
            launch_link_rec(c, lb, spt, wg, (uint32_t)ntiles, a);
        } else if (spt == 4) {
            launch(c, "k_link", lb, k_link<4>, (uint32_t)ntiles, QT, a);
        } else {
            launch(c, "k_link", lb, k_link<1>, (uint32_t)ntiles, QT, a);
        }
        if (final_level) {
            reduce_pairs(c, a.dig_part, ntiles, dscal);
            uint64_t dg[2];
            read_scalars(c, dscal, dg, 2);
            res->rows = count_only ? nullptr : front;
            res->count = S;
            res->digest[0] = dg[0];
            res->digest[1] = dg[1];
            merge_chunks(front);
            st.join_ms = ms_since(tj);
            return finish();
        }
        // M' replaces M; level scratch goes with `ls`
        Mb.reset();
        Mb.p = Mn.p;
        Mn.p = nullptr;
        M = a.Mn;
        Mld = 0;
        const double slots_per_row = (double)gba / (double)R;
        R = S;
        // back to the single workgroup when the table fits and, at this
        // level's slots per row, so would the next level's |GBA|; not right
        // after it stopped without finishing a level
        if (!cp.active && fused_ok && R <= cap_rows && (double)R * slots_per_row <= cap_slots && fused_stuck != j) {
            uint32_t stop = 0;
            if (run_fused(j + 1, nullptr, stop)) return finish();
            if (stop == j + 1) fused_stuck = j + 1;
            j = stop - 1;  // the loop continues with level `stop`
        }
    }
    return done();
}

}  // namespace gsi
