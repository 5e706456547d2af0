// Device build of the data-graph structures a query needs:
//   * PCSR(G,l) for every edge label l (Sec. IV, Definition 4, Algorithm 1);
//   * the column-first vertex signature table (Sec. III-A).
//
// Layout choices (the paper leaves the hash and overflow placement open):
//   * both directions of every edge are stored, each vertex's l-neighbours
//     ascending;
//   * label l owns |V(D_l)| groups of 16 (vertex, offset) pairs (128 bytes);
//     v's home group is pcsr_home(v, H_l) with H_l = |V(D_l)|;
//   * a group keeps its 15 smallest home keys; further keys go 15 per group
//     to empty groups of the same label, taken in ascending index order and
//     handed to overflowing groups in ascending home index, linked through
//     the GID of pair 15 (0xFFFFFFFF ends a chain).  Claim 1 of the paper
//     guarantees enough empty groups;
//   * ci is written in group order then slot order; an unused slot holds
//     (0xFFFFFFFF, END), so the list in slot s ends at the offset of pair s+1.
//
// Pipeline: expand to directed entries -> stable LSD radix sort by
// (label, src, dst) -> runs of equal (label, src) are the keys of the
// partitions -> home groups -> stable sort of keys by group -> chains ->
// group sizes -> scan -> write groups and scatter neighbour lists.
#include <chrono>
#include <cstring>

#include "gsi_internal.h"

namespace gsi {

constexpr uint32_t BT = 256;

static uint32_t blocks(uint64_t n, uint64_t per = BT) {
    uint64_t b = (n + per - 1) / per;
    if (b == 0) b = 1;
    if (b > 0x7FFFFFFFull) fail(GSI_E_INVALID, "grid too large");
    return (uint32_t)b;
}

static int bits_for(uint64_t maxval) {
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) b++;
    return b;
}

enum : uint32_t { ERR_RANGE = 1, ERR_SELF = 2, ERR_LABEL = 4, ERR_DUP = 8, ERR_CLAIM1 = 16 };

__global__ __launch_bounds__(BT) void k_validate_expand(const uint32_t *src, const uint32_t *dst,
                                                        const uint32_t *el, uint64_t m, uint32_t n, uint32_t *os,
                                                        uint32_t *od, uint32_t *ol, uint32_t *err,
                                                        uint32_t *maxlab_part) {
    uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool valid = e < m;
    uint32_t a = 0, b = 0, l = 0;
    if (valid) {
        a = src[e];
        b = dst[e];
        l = el[e];
        uint32_t f = 0;
        if (a >= n || b >= n) f |= ERR_RANGE;
        if (a == b) f |= ERR_SELF;
        if (l >= GSI_MAX_EDGE_LABELS) f |= ERR_LABEL;
        if (f) {
            atomicOr(err, f);
            a = b = 0;
            l = 0;
        }
    }
    // every lane of the wave takes part in the reduction; one partial maximum
    // per workgroup (no same-address atomics)
    __shared__ uint32_t s_max[BT / 64];
    uint32_t wl = l;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t t = __shfl_xor(wl, o, 64);
        wl = t > wl ? t : wl;
    }
    if (lane_id() == 0) s_max[threadIdx.x >> 6] = wl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t mx = 0;
#pragma unroll
        for (int q = 0; q < BT / 64; q++) mx = s_max[q] > mx ? s_max[q] : mx;
        maxlab_part[blockIdx.x] = mx;
    }
    if (!valid) return;
    os[2 * e] = a;
    od[2 * e] = b;
    ol[2 * e] = l;
    os[2 * e + 1] = b;
    od[2 * e + 1] = a;
    ol[2 * e + 1] = l;
}

__global__ __launch_bounds__(1024) void k_max_u32(const uint32_t *part, uint64_t n, uint32_t *out) {
    __shared__ uint32_t s_m[16];
    uint32_t mx = 0;
    for (uint64_t i = threadIdx.x; i < n; i += 1024) mx = part[i] > mx ? part[i] : mx;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t t = __shfl_xor(mx, o, 64);
        mx = t > mx ? t : mx;
    }
    if (lane_id() == 0) s_m[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < 16; q++) mx = s_m[q] > mx ? s_m[q] : mx;
        *out = mx;
    }
}

// after sorting by (src, dst): equal neighbours are repeated vertex pairs
__global__ void k_check_dup(const uint32_t *s, const uint32_t *d, uint64_t nd, uint32_t *err) {
    uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 || p >= nd) return;
    if (s[p] == s[p - 1] && d[p] == d[p - 1]) atomicOr(err, (uint32_t)ERR_DUP);
}

// multi-labelled graphs, after sorting by (label, src, dst): equal
// neighbours with equal labels are the same labelled edge given twice
__global__ void k_check_dup_labelled(const uint32_t *s, const uint32_t *d, const uint32_t *l, uint64_t nd,
                                     uint32_t *err) {
    uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 || p >= nd) return;
    if (s[p] == s[p - 1] && d[p] == d[p - 1] && l[p] == l[p - 1]) atomicOr(err, (uint32_t)ERR_DUP);
}

// label segment bounds in the (label, src, dst)-sorted entries, and run heads
__global__ void k_segments(const uint32_t *s, const uint32_t *l, uint64_t nd, uint64_t *seg_lo, uint64_t *seg_hi,
                           uint32_t *head) {
    uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nd) return;
    uint32_t lab = l[p];
    bool newlab = p == 0 || l[p - 1] != lab;
    if (newlab) seg_lo[lab] = p;
    if (p + 1 == nd || l[p + 1] != lab) seg_hi[lab] = p + 1;
    head[p] = (newlab || s[p - 1] != s[p]) ? 1u : 0u;
}

// run r = (label, vertex) with its first entry
__global__ void k_runs(const uint32_t *s, const uint32_t *l, const uint32_t *head, const uint64_t *hscan,
                       uint64_t nd, uint32_t *run_start, uint32_t *run_vid, uint32_t *run_lab) {
    uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nd || !head[p]) return;
    uint64_t r = hscan[p];
    run_start[r] = (uint32_t)p;
    run_vid[r] = s[p];
    run_lab[r] = l[p];
}

// per label: first run (= first global group) and run count
__global__ void k_label_runs(const uint64_t *seg_lo, const uint64_t *seg_hi, const uint64_t *hscan, uint32_t nlab,
                             uint64_t *lab_rb, uint64_t *lab_re) {
    uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlab) return;
    uint64_t lo = seg_lo[l], hi = seg_hi[l];
    if (hi > lo) {
        lab_rb[l] = hscan[lo];
        lab_re[l] = hscan[hi];
    } else {
        lab_rb[l] = lab_re[l] = 0;
    }
}

struct LabelTab {
    const uint64_t *rb;   // first global group of label
    const uint32_t *G;    // groups of label
    const uint32_t *H;    // home groups of label
    const uint64_t *seg;  // first directed entry (= first ci entry) of label
};

__global__ void k_home(const uint32_t *run_vid, const uint32_t *run_lab, uint64_t R, LabelTab t, uint32_t *key,
                       uint32_t *rid, uint32_t *cnt) {
    uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    uint32_t l = run_lab[r];
    uint32_t g = (uint32_t)t.rb[l] + pcsr_home(run_vid[r], t.H[l]);
    key[r] = g;
    rid[r] = (uint32_t)r;
    atomicAdd(&cnt[g], 1u);
}

// label of a global group: the last label whose first group is <= grp
// (labels without groups carry the first group of the next label, so the
// search lands on the label that owns grp)
__device__ __forceinline__ uint32_t label_of_group(const uint64_t *rb, uint32_t nlab, uint64_t grp) {
    uint32_t lo = 0, hi = nlab - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (rb[mid] <= grp) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void k_overflow_flags(const uint32_t *cnt, uint64_t R, uint32_t *need, uint32_t *empty) {
    uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= R) return;
    uint32_t c = cnt[g];
    need[g] = c > KEYS_PER_GROUP ? (c - KEYS_PER_GROUP + KEYS_PER_GROUP - 1) / KEYS_PER_GROUP : 0u;
    empty[g] = c == 0 ? 1u : 0u;
}

// the e-th empty group (ascending) of each label, label-relative ids
__global__ void k_empty_list(const uint32_t *empty, const uint64_t *escan, uint64_t R, const uint64_t *rb,
                             const uint32_t *G, uint32_t nlab, uint32_t *elist) {
    uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= R || !empty[g]) return;
    uint32_t l = label_of_group(rb, nlab, g);
    uint64_t base = rb[l];
    uint64_t at = base + (escan[g] - escan[base]);
    if (at < R) elist[at] = (uint32_t)(g - base);
}

__global__ void k_claim1(const uint64_t *nscan, const uint64_t *escan, const uint64_t *rb, const uint32_t *G,
                         uint32_t nlab, uint32_t *err) {
    uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlab || G[l] == 0) return;
    uint64_t a = rb[l], b = a + G[l];
    if (nscan[b] - nscan[a] > escan[b] - escan[a]) atomicOr(err, (uint32_t)ERR_CLAIM1);
}

// chain every overflowing group through its empty groups
__global__ void k_chains(const uint32_t *need, const uint64_t *nscan, const uint32_t *elist, uint64_t R,
                         const uint64_t *rb, const uint32_t *G, uint32_t nlab, uint32_t *next, uint32_t *owner,
                         uint32_t *chain_idx, uint32_t *max_chain) {
    uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= R || need[g] == 0) return;
    uint32_t l = label_of_group(rb, nlab, g);
    uint64_t base = rb[l];
    uint64_t first = nscan[g] - nscan[base];
    uint64_t prev = g;
    if (base + first + need[g] > base + G[l]) return;  // Claim 1 violated: reported by k_claim1
    for (uint32_t m = 1; m <= need[g]; m++) {
        uint32_t e = elist[base + first + m - 1];
        if (e >= G[l]) return;  // never reached when Claim 1 holds
        next[prev] = e;
        owner[base + e] = (uint32_t)(g - base);
        chain_idx[base + e] = m;
        prev = base + e;
    }
    atomicMax(max_chain, need[g] + 1);
}

// keys held by each group and the total length of their lists
__global__ void k_group_keys(const uint32_t *cnt, const uint64_t *gstart, const uint32_t *owner,
                             const uint32_t *chain_idx, const uint32_t *sorted_rid, const uint32_t *run_start,
                             uint64_t R, uint64_t nd, const uint64_t *rb, const uint32_t *G, uint32_t nlab,
                             uint64_t *kfirst, uint32_t *nkeys, uint32_t *gdeg) {
    uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= R) return;
    uint64_t first = 0;
    uint32_t nk = 0;
    uint32_t c = cnt[g];
    if (c > 0) {
        first = gstart[g];
        nk = c < KEYS_PER_GROUP ? c : KEYS_PER_GROUP;
    } else if (owner[g] != NONE32) {
        uint32_t l = label_of_group(rb, nlab, g);
        uint64_t h = rb[l] + owner[g];
        uint32_t mi = chain_idx[g];
        first = gstart[h] + (uint64_t)KEYS_PER_GROUP * mi;
        uint32_t left = cnt[h] - KEYS_PER_GROUP * mi;
        nk = left < KEYS_PER_GROUP ? left : KEYS_PER_GROUP;
    }
    uint32_t deg = 0;
    for (uint32_t s = 0; s < nk; s++) {
        uint32_t r = sorted_rid[first + s];
        uint64_t end = (r + 1 < R) ? run_start[r + 1] : nd;
        deg += (uint32_t)(end - run_start[r]);
    }
    kfirst[g] = first;
    nkeys[g] = nk;
    gdeg[g] = deg;
}

// write the 16 pairs of each group; remember each key's list offset
__global__ void k_write_groups(const uint64_t *kfirst, const uint32_t *nkeys, const uint64_t *gci,
                               const uint32_t *next, const uint32_t *sorted_rid, const uint32_t *run_start,
                               const uint32_t *run_vid, uint64_t R, uint64_t nd, const uint64_t *rb,
                               const uint32_t *G, const uint64_t *seg, uint32_t nlab, uint32_t *gl,
                               uint32_t *run_off) {
    uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= R) return;
    uint32_t l = label_of_group(rb, nlab, g);
    uint64_t lb = seg[l];
    uint32_t pos = (uint32_t)(gci[g] - lb);
    uint32_t end = (uint32_t)(gci[g + 1] - lb);
    uint32_t pr[GROUP_WORDS];
    uint32_t nk = nkeys[g];
    uint64_t first = kfirst[g];
#pragma unroll
    for (uint32_t s = 0; s < KEYS_PER_GROUP; s++) {
        if (s < nk) {
            uint32_t r = sorted_rid[first + s];
            uint64_t e = (r + 1 < R) ? run_start[r + 1] : nd;
            pr[2 * s] = run_vid[r];
            pr[2 * s + 1] = pos;
            run_off[r] = pos;
            pos += (uint32_t)(e - run_start[r]);
        } else {
            pr[2 * s] = NONE32;
            pr[2 * s + 1] = end;
        }
    }
    pr[2 * KEYS_PER_GROUP] = next[g];
    pr[2 * KEYS_PER_GROUP + 1] = end;
    uint4 *dstv = reinterpret_cast<uint4 *>(gl + g * GROUP_WORDS);
#pragma unroll
    for (int i = 0; i < 8; i++) dstv[i] = make_uint4(pr[4 * i], pr[4 * i + 1], pr[4 * i + 2], pr[4 * i + 3]);
}

__global__ void k_scatter_ci(const uint32_t *d, const uint32_t *l, const uint64_t *hscan, const uint32_t *run_start,
                             const uint32_t *run_off, const uint64_t *seg, uint64_t nd, uint32_t *ci) {
    uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nd) return;
    uint64_t r = hscan[p + 1] - 1;
    uint32_t t = (uint32_t)(p - run_start[r]);
    uint64_t at = seg[l[p]] + run_off[r] + t;
    if (at < nd) ci[at] = d[p];
}

// Signatures (Sec. III-A): word 0 = label; each directed entry (v -> w, l)
// adds the pair (l, L_V(w)) to v's two-bit group: the first pair sets the
// low bit (01); any later pair finds it set and raises the high bit (11).
__global__ void k_sig_labels(const uint32_t *vl, uint32_t n, uint32_t *sig) {
    uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    sig[v] = vl[v];
#pragma unroll
    for (int w = 1; w < GSI_SIG_WORDS; w++) sig[(uint64_t)w * n + v] = 0;
}

// Multi-labelled vertices (Sec. VII-B): word 0 holds every label of v
// hashed to one of its 32 bits, so the filter tests containment there and a
// refinement pass checks the label sets exactly.
__global__ void k_sig_labels_multi(const uint32_t *off, const uint32_t *lab, uint32_t n, uint32_t *sig) {
    uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    uint32_t b = 0;
    for (uint32_t t = off[v]; t < off[v + 1]; t++) b |= label_bit(lab[t]);
    sig[v] = b;
#pragma unroll
    for (int w = 1; w < GSI_SIG_WORDS; w++) sig[(uint64_t)w * n + v] = 0;
}

// every directed entry (v -> w, l) adds the pair (l, x) for each label x of w
__global__ void k_sig_pairs_multi(const uint32_t *s, const uint32_t *d, const uint32_t *l, const uint32_t *off,
                                  const uint32_t *lab, uint64_t nd, uint32_t n, uint32_t *sig) {
    uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nd) return;
    const uint32_t w = d[p];
    for (uint32_t t = off[w]; t < off[w + 1]; t++) {
        uint32_t g = sig_group(l[p], lab[t]);
        uint32_t *word = sig + (uint64_t)(1 + g / 16) * n + s[p];
        uint32_t lo = 1u << (2 * (g % 16));
        uint32_t old = atomicOr(word, lo);
        if (old & lo) atomicOr(word, lo << 1);
    }
}

__global__ void k_sig_pairs(const uint32_t *s, const uint32_t *d, const uint32_t *l, const uint32_t *vl, uint64_t nd,
                            uint32_t n, uint32_t *sig) {
    uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nd) return;
    uint32_t g = sig_group(l[p], vl[d[p]]);
    uint32_t *word = sig + (uint64_t)(1 + g / 16) * n + s[p];
    uint32_t lo = 1u << (2 * (g % 16));
    uint32_t old = atomicOr(word, lo);
    if (old & lo) atomicOr(word, lo << 1);
}

void build_graph(gsi_graph *g, const uint32_t *vl, const uint32_t *src, const uint32_t *dst, const uint32_t *el) {
    gsi_ctx *c = g->ctx;
    auto t0 = std::chrono::steady_clock::now();
    const uint32_t n = g->n;
    const uint64_t m = g->m, nd = 2 * m;
    Scratch s(c);

    uint64_t *scal = s.get<uint64_t>(8, "scalars");
    fill_u64(c, scal, 0, 8);
    uint32_t *err = reinterpret_cast<uint32_t *>(scal);       // scal[0] low word
    uint32_t *maxlab = reinterpret_cast<uint32_t *>(scal + 1);
    uint32_t *maxchain = reinterpret_cast<uint32_t *>(scal + 2);

    // persistent signature table first (independent of everything else)
    g->sig = persist<uint32_t>(c, (uint64_t)GSI_SIG_WORDS * n, "signature table");
    // CI_PAD spare elements: searches read aligned windows that may pass a list's end
    g->ci = persist<uint32_t>(c, nd + CI_PAD, "ci");

    uint32_t *A[3], *B[3];
    for (int i = 0; i < 3; i++) {
        A[i] = s.get<uint32_t>(nd, "sort buffer");
        B[i] = s.get<uint32_t>(nd, "sort buffer");
    }
    if (m) {
        uint32_t nb = blocks(m);
        uint32_t *mpart = s.get<uint32_t>(nb, "label maxima");
        launch(c, "k_validate_expand", 12.0 * m + 24.0 * m, k_validate_expand, nb, BT, src, dst, el, m, n, A[0], A[1],
               A[2], err, mpart);
        launch(c, "k_max_u32", 4.0 * nb, k_max_u32, 1, 1024, (const uint32_t *)mpart, (uint64_t)nb, maxlab);
    }
    uint64_t hs[3];
    read_scalars(c, scal, hs, 3);
    uint32_t e0 = (uint32_t)hs[0];
    if (e0 & ERR_RANGE) fail(GSI_E_INVALID, "edge endpoint out of range");
    if (e0 & ERR_SELF) fail(GSI_E_INVALID, "self-loop in data graph");
    if (e0 & ERR_LABEL) fail(GSI_E_INVALID, "edge label >= %u", (unsigned)GSI_MAX_EDGE_LABELS);
    uint32_t nlab = m ? (uint32_t)hs[1] + 1 : 0;
    g->nlab = nlab;

    // (src, dst) order, duplicate check, then stable passes on the label
    int vb = bits_for(n - 1 ? n - 1 : 1), lb = bits_for(nlab > 1 ? nlab - 1 : 0);
    std::vector<SortPass> passes;
    for (int sh = 0; sh < vb; sh += 8) passes.push_back({1, sh});
    for (int sh = 0; sh < vb; sh += 8) passes.push_back({0, sh});
    uint32_t **cur = A;
    if (m) {
        bool t = radix_sort(c, (uint32_t)nd, 3, A, B, passes, s);
        cur = t ? B : A;
        uint32_t **other = t ? A : B;
        if (!g->multi) launch(c, "k_check_dup", 8.0 * nd, k_check_dup, blocks(nd), BT, cur[0], cur[1], nd, err);
        std::vector<SortPass> lp;
        for (int sh = 0; sh < lb; sh += 8) lp.push_back({2, sh});
        bool t2 = radix_sort(c, (uint32_t)nd, 3, cur, other, lp, s);
        if (t2) cur = other;
        if (g->multi)
            launch(c, "k_check_dup", 12.0 * nd, k_check_dup_labelled, blocks(nd), BT, cur[0], cur[1], cur[2], nd,
                   err);
    }
    read_scalars(c, scal, hs, 1);
    if ((uint32_t)hs[0] & ERR_DUP)
        fail(GSI_E_INVALID, g->multi ? "the same labelled edge is given twice in the data graph"
                                     : "repeated vertex pair (parallel edge) in data graph");
    uint32_t *S = cur[0], *D = cur[1], *L = cur[2];

    // label segments and runs
    uint64_t *seg = s.get<uint64_t>(2 * (uint64_t)nlab + 2, "label segments");
    uint64_t *seg_hi = seg + nlab + 1;
    fill_u64(c, seg, 0, 2 * (uint64_t)nlab + 2);
    uint32_t *head = s.get<uint32_t>(nd, "run heads");
    uint64_t *hscan = s.get<uint64_t>(nd + 1, "run scan");
    if (m)
        launch(c, "k_segments", 12.0 * nd, k_segments, blocks(nd), BT, S, L, nd, seg, seg_hi, head);
    exclusive_scan(c, head, nd, hscan, s);
    uint64_t R;
    read_scalars(c, hscan + nd, &R, 1);
    g->total_groups = R;
    const bool keep_cr = (g->flags & GSI_GRAPH_KEEP_CR) != 0;
    uint32_t *run_start = keep_cr ? persist<uint32_t>(c, R ? R : 1, "cr starts") : s.get<uint32_t>(R, "run start");
    uint32_t *run_vid = keep_cr ? persist<uint32_t>(c, R ? R : 1, "cr vertices") : s.get<uint32_t>(R, "run vertex");
    if (keep_cr) {
        g->cr_start = run_start;
        g->cr_vid = run_vid;
    }
    uint32_t *run_lab = s.get<uint32_t>(R, "run label");
    if (m)
        launch(c, "k_runs", 12.0 * nd, k_runs, blocks(nd), BT, S, L, head, hscan, nd, run_start, run_vid, run_lab);
    uint64_t *lab_rb = s.get<uint64_t>(2 * (uint64_t)nlab + 2, "label runs");
    uint64_t *lab_re = lab_rb + nlab + 1;
    if (nlab)
        launch(c, "k_label_runs", 32.0 * nlab, k_label_runs, blocks(nlab), BT, seg, seg_hi, hscan, nlab, lab_rb, lab_re);
    std::vector<uint64_t> h_rb(nlab), h_re(nlab), h_lo(nlab), h_hi(nlab);
    if (nlab) {
        GSI_HIP(hipMemcpyAsync(h_rb.data(), lab_rb, 8ull * nlab, hipMemcpyDeviceToHost, c->stream));
        GSI_HIP(hipMemcpyAsync(h_re.data(), lab_re, 8ull * nlab, hipMemcpyDeviceToHost, c->stream));
        GSI_HIP(hipMemcpyAsync(h_lo.data(), seg, 8ull * nlab, hipMemcpyDeviceToHost, c->stream));
        GSI_HIP(hipMemcpyAsync(h_hi.data(), seg_hi, 8ull * nlab, hipMemcpyDeviceToHost, c->stream));
        sync(c);
    }
    g->group_base.assign(nlab, 0);
    g->G.assign(nlab, 0);
    g->H.assign(nlab, 0);
    g->ci_base.assign(nlab, 0);
    g->edges.assign(nlab, 0);
    // empty labels get the start of the next non-empty label so that group
    // ranges stay sorted for the label-of-group search
    uint64_t nextb = R;
    for (int64_t l = (int64_t)nlab - 1; l >= 0; l--) {
        if (h_re[l] > h_rb[l]) {
            g->group_base[l] = h_rb[l];
            g->G[l] = (uint32_t)(h_re[l] - h_rb[l]);
            g->ci_base[l] = h_lo[l];
            g->edges[l] = (h_hi[l] - h_lo[l]) / 2;
            nextb = h_rb[l];
        } else {
            g->group_base[l] = nextb;
            g->ci_base[l] = 0;
        }
        uint32_t Gl = g->G[l];
        g->H[l] = (g->flags & GSI_GRAPH_TEST_FEW_HOME_GROUPS) ? (Gl + GSI_PCSR_GPN - 1) / GSI_PCSR_GPN : Gl;
    }
    for (uint32_t l = 0; l < nlab; l++)
        if (g->G[l] == 0) g->ci_base[l] = 0;
    // device copy of the label table
    uint64_t *d_rb = s.get<uint64_t>(nlab + 1, "label group base");
    uint32_t *d_G = s.get<uint32_t>(nlab + 1, "label groups");
    uint32_t *d_H = s.get<uint32_t>(nlab + 1, "label home groups");
    uint64_t *d_seg = s.get<uint64_t>(nlab + 1, "label ci base");
    if (nlab) {
        std::vector<uint64_t> segb(nlab);
        for (uint32_t l = 0; l < nlab; l++) segb[l] = g->G[l] ? h_lo[l] : 0;
        GSI_HIP(hipMemcpyAsync(d_rb, g->group_base.data(), 8ull * nlab, hipMemcpyHostToDevice, c->stream));
        GSI_HIP(hipMemcpyAsync(d_G, g->G.data(), 4ull * nlab, hipMemcpyHostToDevice, c->stream));
        GSI_HIP(hipMemcpyAsync(d_H, g->H.data(), 4ull * nlab, hipMemcpyHostToDevice, c->stream));
        GSI_HIP(hipMemcpyAsync(d_seg, segb.data(), 8ull * nlab, hipMemcpyHostToDevice, c->stream));
        sync(c);  // host vectors above are pageable and local
    }
    LabelTab lt{d_rb, d_G, d_H, d_seg};

    g->gl = persist<uint32_t>(c, R * GROUP_WORDS, "pcsr groups");
    g->bytes = 4ull * GSI_SIG_WORDS * n + 4ull * nd + 4ull * GROUP_WORDS * R;

    if (R) {
        // home groups, stable sort of keys by group
        uint32_t *key = s.get<uint32_t>(R, "group key");
        uint32_t *rid = s.get<uint32_t>(R, "run id");
        uint32_t *key2 = s.get<uint32_t>(R, "group key tmp");
        uint32_t *rid2 = s.get<uint32_t>(R, "run id tmp");
        uint32_t *cnt = s.get<uint32_t>(R, "home counts");
        fill_u32(c, cnt, 0, R);
        launch(c, "k_home", 16.0 * R, k_home, blocks(R), BT, run_vid, run_lab, R, lt, key, rid, cnt);
        std::vector<SortPass> kp;
        int kb = bits_for(R - 1);
        for (int sh = 0; sh < kb; sh += 8) kp.push_back({0, sh});
        uint32_t *ka[2] = {key, rid}, *kt[2] = {key2, rid2};
        bool t = radix_sort(c, (uint32_t)R, 2, ka, kt, kp, s);
        uint32_t *sorted_rid = t ? rid2 : rid;

        uint64_t *gstart = s.get<uint64_t>(R + 1, "group key start");
        exclusive_scan(c, cnt, R, gstart, s);
        uint32_t *need = s.get<uint32_t>(R, "overflow need");
        uint32_t *empt = s.get<uint32_t>(R, "empty flag");
        launch(c, "k_overflow_flags", 12.0 * R, k_overflow_flags, blocks(R), BT, cnt, R, need, empt);
        uint64_t *nscan = s.get<uint64_t>(R + 1, "need scan");
        uint64_t *escan = s.get<uint64_t>(R + 1, "empty scan");
        exclusive_scan(c, need, R, nscan, s);
        exclusive_scan(c, empt, R, escan, s);
        uint32_t *elist = s.get<uint32_t>(R, "empty list");
        fill_u32(c, elist, NONE32, R);
        launch(c, "k_empty_list", 16.0 * R, k_empty_list, blocks(R), BT, empt, escan, R, d_rb, d_G, nlab, elist);
        launch(c, "k_claim1", 32.0 * nlab, k_claim1, blocks(nlab), BT, nscan, escan, d_rb, d_G, nlab, err);
        uint32_t *next = s.get<uint32_t>(R, "chain next");
        uint32_t *owner = s.get<uint32_t>(R, "chain owner");
        uint32_t *cidx = s.get<uint32_t>(R, "chain index");
        fill_u32(c, next, NONE32, R);
        fill_u32(c, owner, NONE32, R);
        fill_u32(c, maxchain, 1, 1);
        launch(c, "k_chains", 12.0 * R, k_chains, blocks(R), BT, need, nscan, elist, R, d_rb, d_G, nlab, next, owner, cidx, maxchain);
        uint64_t *kfirst = s.get<uint64_t>(R, "group first key");
        uint32_t *nkeys = s.get<uint32_t>(R, "group keys");
        uint32_t *gdeg = s.get<uint32_t>(R, "group degree");
        launch(c, "k_group_keys", 32.0 * R, k_group_keys, blocks(R), BT, cnt, gstart, owner, cidx, sorted_rid, run_start, R, nd, d_rb, d_G, nlab, kfirst, nkeys, gdeg);
        uint64_t *gci = s.get<uint64_t>(R + 1, "group ci start");
        exclusive_scan(c, gdeg, R, gci, s);
        uint32_t *run_off = keep_cr ? persist<uint32_t>(c, R, "cr offsets") : s.get<uint32_t>(R, "run offset");
        if (keep_cr) g->cr_off = run_off;
        launch(c, "k_write_groups", 128.0 * R + 24.0 * R, k_write_groups, blocks(R), BT, kfirst, nkeys, gci, next, sorted_rid, run_start, run_vid, R, nd, d_rb, d_G, d_seg, nlab, g->gl, run_off);
        launch(c, "k_scatter_ci", 24.0 * nd, k_scatter_ci, blocks(nd), BT, D, L, hscan, run_start, run_off, d_seg, nd, g->ci);
    }
    if (g->multi) {
        launch(c, "k_sig_labels", 8.0 * n + 64.0 * n, k_sig_labels_multi, blocks(n), BT, (const uint32_t *)g->vl_off,
               (const uint32_t *)g->vl_lab, n, g->sig);
        if (nd)
            launch(c, "k_sig_pairs", 24.0 * nd, k_sig_pairs_multi, blocks(nd), BT, S, D, L,
                   (const uint32_t *)g->vl_off, (const uint32_t *)g->vl_lab, nd, n, g->sig);
    } else {
        launch(c, "k_sig_labels", 8.0 * n + 60.0 * n, k_sig_labels, blocks(n), BT, vl, n, g->sig);
        if (nd)
            launch(c, "k_sig_pairs", 20.0 * nd, k_sig_pairs, blocks(nd), BT, S, D, L, vl, nd, n, g->sig);
    }
    read_scalars(c, scal, hs, 3);
    if ((uint32_t)hs[0] & ERR_CLAIM1) fail(GSI_E_INTERNAL, "PCSR: not enough empty groups (Claim 1)");
    g->max_chain = R ? (uint32_t)hs[2] : 0;
    auto t1 = std::chrono::steady_clock::now();
    g->build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
}

}  // namespace gsi
