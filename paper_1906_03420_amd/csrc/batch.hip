// The batched path: many queries over one resident graph.
//
//   filter   one pass of the signature filter per 32 query vertices of the
//            whole batch (query vertices grouped by label), one readback
//   plan     Algorithm 2 per query on the host
//   roots    every query's C(u_first) compacted in one pass
//   tier 1   persistent fused launch, workgroups of the scheduled size pull
//            queries from a shared counter and run all levels per query
//   tier 2   what tier 1 could not hold, in 1024-thread workgroups
//   rest     the level-synchronous engine (wide.hip), all at once
//
// The schedule (tier-1 workgroup size, launched occupancy) is chosen by the
// autotuner, which times every candidate on a sample of the batch.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>

#include "admit.h"
#include "fused.h"
#include "gsi_internal.h"
#include "wide.h"

struct gsi_batch {
    gsi_ctx *ctx = nullptr;
    uint32_t nq = 0;
    bool count_only = false;
    std::unique_ptr<gsi::Slot[]> slots;
    gsi_batch_info info{};
};

namespace gsi {

constexpr uint32_t BQT = 256;
constexpr uint32_t TIER2_THREADS = 1024;

__global__ __launch_bounds__(BQT) void k_roots_popc(const uint64_t *bits, const uint32_t *rows, uint64_t nwords,
                                                   uint64_t total, uint32_t *cnt) {
    const uint64_t idx = (uint64_t)blockIdx.x * BQT + threadIdx.x;
    if (idx >= total) return;
    const uint64_t q = idx / nwords, wi = idx - q * nwords;
    cnt[idx] = (uint32_t)__popcll(bits[(uint64_t)rows[q] * nwords + wi]);
}

__global__ __launch_bounds__(BQT) void k_roots_emit(const uint64_t *bits, const uint32_t *rows, uint64_t nwords,
                                                   uint64_t total, const uint64_t *off, uint32_t *out) {
    const uint64_t idx = (uint64_t)blockIdx.x * BQT + threadIdx.x;
    if (idx >= total) return;
    const uint64_t q = idx / nwords, wi = idx - q * nwords;
    uint64_t b = bits[(uint64_t)rows[q] * nwords + wi];
    uint64_t o = off[idx];
    while (b) {
        const uint32_t t = (uint32_t)__ffsll((unsigned long long)b) - 1;
        out[o++] = (uint32_t)(wi * 64 + t);
        b &= b - 1;
    }
}

static uint32_t bgrid(uint64_t n) {
    uint64_t b = (n + BQT - 1) / BQT;
    if (b == 0) b = 1;
    if (b > 0x7FFFFFFFull) fail(GSI_E_CAPACITY, "grid too large");
    return (uint32_t)b;
}

static double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

static int cu_count(gsi_ctx *c) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || n < 1) n = 1;
    return n;
}

struct FusedQuery {
    uint32_t qi;       // batch index
    uint32_t R0;
    uint64_t plan_off; // bytes
    uint64_t m0_off;   // rows
    uint64_t out_off;  // words
};

// Runs one fused tier over `list`; fills entries of finished queries and
// returns the ones it could not hold.
static std::vector<FusedQuery> run_tier(gsi_graph *g, const std::shared_ptr<Round> &rd,
                                        const std::vector<Slot *> &slots, bool count_only, uint8_t path,
                                        const FTier &t,
                                        uint32_t grid_scale, const std::vector<FusedQuery> &list,
                                        const std::vector<uint32_t> &ks, const uint8_t *d_plans,
                                        const uint32_t *d_M0) {
    gsi_ctx *c = g->ctx;
    std::vector<FusedQuery> left;
    if (list.empty()) return left;
    const uint32_t n = (uint32_t)list.size();
    uint32_t kmax = 2;
    std::vector<FBatchItem> items(n);
    for (uint32_t i = 0; i < n; i++) {
        items[i].plan_off = list[i].plan_off;
        items[i].m0_off = list[i].m0_off;
        items[i].out_off = list[i].out_off;
        items[i].R0 = list[i].R0;
        kmax = std::max(kmax, ks[list[i].qi]);
    }
    const uint64_t per_cu = std::max<uint64_t>(1, (uint64_t)t.blocks_per_cu * grid_scale / 8);
    const uint32_t grid = (uint32_t)std::min<uint64_t>(n, per_cu * cu_count(c));
    const uint64_t slot_words = 2ull * t.cap_rows * kmax + fused_loc_words(kmax, t.cap_rows);
    Scratch ts(c);
    FBatchItem *d_items = ts.get<FBatchItem>(n, "batch items");
    uint32_t *scratch = ts.get<uint32_t>(slot_words * grid, "batch slots");
    FStatus *d_st = reinterpret_cast<FStatus *>(ts.get<uint64_t>((uint64_t)n * sizeof(FStatus) / 8, "batch status"));
    uint32_t *counter = ts.get<uint32_t>(1, "batch counter");
    GSI_HIP(hipMemcpyAsync(d_items, items.data(), sizeof(FBatchItem) * n, hipMemcpyHostToDevice, c->stream));
    fill_u64(c, reinterpret_cast<uint64_t *>(d_st), 0, (uint64_t)n * sizeof(FStatus) / 8);
    fill_u32(c, counter, 0, 1);
    launch_fused_batch(c, t, grid, d_plans, d_items, n, d_M0, scratch, slot_words, kmax, count_only ? nullptr : rd->out,
                       d_st, counter, 0.0);
    std::vector<FStatus> hs(n);
    GSI_HIP(hipMemcpyAsync(hs.data(), d_st, sizeof(FStatus) * n, hipMemcpyDeviceToHost, c->stream));
    sync(c);  // also keeps `items` alive until its copy has run
    for (uint32_t i = 0; i < n; i++) {
        Slot &sl = *slots[list[i].qi];
        if (hs[i].done) {
            sl.done = true;
            sl.path = path;
            sl.count = hs[i].count;
            sl.digest[0] = hs[i].digest[0];
            sl.digest[1] = hs[i].digest[1];
            if (!count_only && hs[i].count) {
                sl.rows = rd->out + list[i].out_off;
                sl.keep = rd;
            }
        } else {
            left.push_back(list[i]);
        }
    }
    return left;
}


static void *round_block(gsi_ctx *c, uint64_t bytes, const char *what) {
    void *p = c->arena.alloc(bytes ? bytes : 256, false);
    if (!p)
        fail(GSI_E_NOMEM, "arena exhausted allocating %llu bytes for %s (largest free block %llu)",
             (unsigned long long)bytes, what, (unsigned long long)c->arena.largest_free());
    return p;
}

void finish_slot(WideQuery &x, Slot &sl) {
    sl.done = true;
    sl.path = PATH_LEVELS;
    sl.status = x.status;
    sl.count = x.count;
    sl.digest[0] = x.digest[0];
    sl.digest[1] = x.digest[1];
    sl.own = x.take_rows();
    sl.rows = sl.own;
}

std::vector<WideQuery> admit_round(gsi_graph *g, const std::vector<const HostQuery *> &hq,
                                   const std::vector<Slot *> &slots, const std::vector<uint64_t> &tags,
                                   bool count_only, bool levels_only, gsi_batch_schedule sched, AdmitStats *st) {
    gsi_ctx *c = g->ctx;
    const uint32_t nq = (uint32_t)hq.size();
    std::vector<WideQuery> wide;
    auto rd = std::make_shared<Round>();
    rd->ctx = c;
    for (uint32_t i = 0; i < nq; i++) {
        slots[i]->ctx = c;
        slots[i]->k = hq[i]->k;
    }
    // queries whose edge labels G lacks have no match
    std::vector<uint32_t> active;
    for (uint32_t i = 0; i < nq; i++) {
        bool ok = true;
        for (uint32_t l : hq[i]->el) ok &= l < g->nlab && g->edges[l] > 0;
        if (ok) {
            active.push_back(i);
        } else {
            slots[i]->done = true;
            st->empty++;
        }
    }
    if (active.empty()) return wide;
    const uint64_t nwords = ((uint64_t)g->n + 63) / 64;
    std::vector<const HostQuery *> aq;
    std::vector<uint32_t> qbase{0};
    for (uint32_t i : active) {
        aq.push_back(hq[i]);
        qbase.push_back(qbase.back() + hq[i]->k);
    }
    const uint64_t nqv = qbase.back();
    auto tf = std::chrono::steady_clock::now();
    rd->bits = round_block(c, nqv * nwords * 8, "candidate bitsets");
    uint64_t *bits = static_cast<uint64_t *>(rd->bits);
    std::vector<uint32_t> cnt(nqv);
    {
        Scratch fs(c);
        uint32_t *dcnt = fs.get<uint32_t>(nqv, "candidate counts");
        run_filter_many(g, aq, qbase, bits, dcnt);
        GSI_HIP(hipMemcpyAsync(cnt.data(), dcnt, 4 * nqv, hipMemcpyDeviceToHost, c->stream));
        sync(c);
    }
    st->filter_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tf).count();

    const FTier t1 = fused_tier(sched.threads), t2 = fused_tier(TIER2_THREADS);
    std::vector<uint32_t> ks(nq);
    for (uint32_t i = 0; i < nq; i++) ks[i] = hq[i]->k;
    struct Planned {
        uint32_t qi, a;
        std::vector<uint32_t> order, e0src;
        std::vector<uint32_t> cand;
        uint32_t R0;
        uint64_t m0_off;
    };
    std::vector<Planned> planned;
    std::vector<uint32_t> single;
    for (size_t a = 0; a < active.size(); a++) {
        const uint32_t qi = active[a];
        const HostQuery &q = *hq[qi];
        std::vector<uint32_t> cand(cnt.begin() + qbase[a], cnt.begin() + qbase[a] + q.k);
        bool empty = false;
        for (uint32_t x : cand) empty |= x == 0;
        if (empty) {
            slots[qi]->done = true;
            st->empty++;
            continue;
        }
        if (q.k < 2) {
            single.push_back(qi);
            continue;
        }
        Planned pl;
        pl.qi = qi;
        pl.a = (uint32_t)a;
        make_plan(g, q, cand, pl.order, pl.e0src);
        pl.R0 = cand[pl.order[0]];
        pl.m0_off = 0;
        pl.cand = cand;
        planned.push_back(std::move(pl));
    }

    std::vector<FusedQuery> fused;
    std::vector<uint8_t> plan_blob;
    std::vector<uint32_t> root_rows;
    uint64_t m0_total = 0, out_total = 0;
    for (auto &pl : planned) {
        const HostQuery &q = *hq[pl.qi];
        pl.m0_off = m0_total;
        m0_total += pl.R0;
        root_rows.push_back(qbase[pl.a] + pl.order[0]);
        if (levels_only || pl.R0 > t2.cap_rows) continue;
        uint32_t n_edges = 0;
        for (uint32_t j = 1; j < q.k; j++)
            for (uint32_t i = 0; i < j; i++)
                for (auto &p : q.adj[pl.order[j]]) n_edges += p.first == pl.order[i];
        const size_t pb = (fplan_bytes(n_edges) + 15) & ~size_t(15);
        const uint64_t off = plan_blob.size();
        plan_blob.resize(off + pb, 0);
        FPlan *hp = reinterpret_cast<FPlan *>(plan_blob.data() + off);
        hp->k = q.k;
        hp->count_only = count_only ? 1u : 0u;
        hp->cap_rows = 0xFFFFFFFFu;  // the tier's own capacities apply
        hp->cap_slots = 0xFFFFFFFFu;
        hp->pick = 1;
        hp->ci_all = g->ci;
        std::vector<uint32_t> col(q.k);
        for (uint32_t j = 0; j < q.k; j++) col[pl.order[j]] = j;
        for (uint32_t v = 0; v < q.k; v++) hp->qcol[v] = col[v];
        uint32_t ei = 0;
        for (uint32_t j = 1; j < q.k; j++) {
            hp->lv_first[j] = ei;
            hp->Cu[j] = bits + (uint64_t)(qbase[pl.a] + pl.order[j]) * nwords;
            uint32_t ne = 0;
            for (uint32_t i = 0; i < j; i++)
                for (auto &p : q.adj[pl.order[j]])
                    if (p.first == pl.order[i]) {
                        const uint32_t l = p.second;
                        FEdge &fe = hp->edges[ei + ne];
                        fe.gl = g->gl + g->group_base[l] * GROUP_WORDS;
                        fe.ci = g->ci + g->ci_base[l];
                        fe.G = g->G[l];
                        fe.H = g->H[l];
                        fe.col = i;
                        fe.ci_off = (uint32_t)g->ci_base[l];
                        if (pl.order[i] == pl.e0src[j]) hp->lv_e0[j] = ne;
                        ne++;
                    }
            hp->lv_ne[j] = ne;
            hp->lv_mmask[j] = 0;
            for (uint32_t c = 0; c < j; c++)
                if (q.multi || q.vl[pl.order[c]] == q.vl[pl.order[j]]) hp->lv_mmask[j] |= 1u << c;
            ei += ne;
        }
        FusedQuery f;
        f.qi = pl.qi;
        f.R0 = pl.R0;
        f.plan_off = off;
        f.m0_off = pl.m0_off;
        f.out_off = out_total;
        out_total += count_only ? 0 : (uint64_t)t2.cap_slots * q.k;
        fused.push_back(f);
    }

    std::vector<uint32_t> to_wide;
    uint32_t *d_M0 = nullptr;
    if (!planned.empty()) {
        Scratch rs(c);
        uint32_t *d_rows = rs.get<uint32_t>(root_rows.size(), "root rows");
        GSI_HIP(hipMemcpyAsync(d_rows, root_rows.data(), 4 * root_rows.size(), hipMemcpyHostToDevice, c->stream));
        const uint64_t tw = (uint64_t)root_rows.size() * nwords;
        rd->m0 = round_block(c, m0_total * 4, "root tables");
        d_M0 = static_cast<uint32_t *>(rd->m0);
        uint32_t *wc = rs.get<uint32_t>(tw, "root word counts");
        uint64_t *wo = rs.get<uint64_t>(tw + 1, "root word offsets");
        launch(c, "k_roots_popc", 12.0 * tw, k_roots_popc, bgrid(tw), BQT, (const uint64_t *)bits,
               (const uint32_t *)d_rows, nwords, tw, wc);
        exclusive_scan(c, wc, tw, wo, rs);
        launch(c, "k_roots_emit", 16.0 * tw + 4.0 * m0_total, k_roots_emit, bgrid(tw), BQT, (const uint64_t *)bits,
               (const uint32_t *)d_rows, nwords, tw, (const uint64_t *)wo, d_M0);
        sync(c);  // host vectors copied above stay alive until here
    }
    if (!fused.empty()) {
        Scratch ps(c);
        uint8_t *d_plans = ps.get<uint8_t>(plan_blob.size(), "fused plans");
        GSI_HIP(hipMemcpyAsync(d_plans, plan_blob.data(), plan_blob.size(), hipMemcpyHostToDevice, c->stream));
        if (!count_only && out_total) rd->out = static_cast<uint32_t *>(round_block(c, out_total * 4, "fused rows"));
        std::vector<FusedQuery> first, second;
        for (auto &f : fused) (f.R0 <= t1.cap_rows ? first : second).push_back(f);
        auto ta = std::chrono::steady_clock::now();
        std::vector<FusedQuery> left = run_tier(g, rd, slots, count_only, PATH_TIER1, t1, sched.grid_scale, first, ks, d_plans, d_M0);
        st->tier1 += (uint32_t)(first.size() - left.size());
        st->tier1_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - ta).count();
        if (t1.threads != t2.threads) {
            second.insert(second.end(), left.begin(), left.end());
            left.clear();
        } else {
            left.insert(left.end(), second.begin(), second.end());
            second.clear();
        }
        auto tb = std::chrono::steady_clock::now();
        std::vector<FusedQuery> left2 = run_tier(g, rd, slots, count_only, PATH_TIER2, t2, 8, second, ks, d_plans, d_M0);
        st->tier2 += (uint32_t)(second.size() - left2.size());
        st->tier2_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tb).count();
        for (auto &f : left) to_wide.push_back(f.qi);
        for (auto &f : left2) to_wide.push_back(f.qi);
    }
    for (auto &pl : planned)
        if (levels_only || pl.R0 > t2.cap_rows) to_wide.push_back(pl.qi);

    // one-vertex queries: the root table is the answer
    for (uint32_t qi : single) {
        gsi_query_options o{};
        o.flags = count_only ? GSI_COUNT_ONLY : 0u;
        gsi_result *r = run_query(g, *hq[qi], &o);
        Slot &sl = *slots[qi];
        sl.res = r;
        sl.done = true;
        sl.path = PATH_SINGLE;
        sl.count = r->count;
        sl.digest[0] = r->digest[0];
        sl.digest[1] = r->digest[1];
        sl.rows = r->rows;
        st->single++;
    }

    std::sort(to_wide.begin(), to_wide.end());
    std::vector<const Planned *> byq(nq, nullptr);
    for (auto &pl : planned) byq[pl.qi] = &pl;
    for (uint32_t qi : to_wide) {
        const Planned &pl = *byq[qi];
        const HostQuery &q = *hq[qi];
        WideQuery x;
        x.ctx = c;
        x.q = &q;
        x.qi = qi;
        x.tag = tags.empty() ? qi : tags[qi];
        x.keep = rd;
        x.order = pl.order;
        x.e0src = pl.e0src;
        x.cand = pl.cand;
        x.col.assign(q.k, 0);
        for (uint32_t j = 0; j < q.k; j++) x.col[pl.order[j]] = j;
        x.Cu.assign(q.k, nullptr);
        for (uint32_t j = 0; j < q.k; j++) x.Cu[j] = bits + (uint64_t)(qbase[pl.a] + pl.order[j]) * nwords;
        x.M = d_M0 + pl.m0_off;
        x.R = pl.R0;
        wide.push_back(std::move(x));
    }
    st->wide += (uint32_t)wide.size();
    return wide;
}

gsi_batch *run_batch(gsi_graph *g, uint32_t nq, const gsi_query_desc *qd, uint32_t flags,
                     gsi_batch_schedule sched) {
    gsi_ctx *c = g->ctx;
    auto t0 = std::chrono::steady_clock::now();
    if (flags & ~(GSI_COUNT_ONLY | GSI_BATCH_LEVELS_ONLY)) fail(GSI_E_INVALID, "unknown batch flag");
    if (sched.threads != 64 && sched.threads != 256 && sched.threads != 1024)
        fail(GSI_E_INVALID, "schedule threads must be 64, 256 or 1024");
    if (sched.grid_scale < 1 || sched.grid_scale > 8) fail(GSI_E_INVALID, "schedule grid_scale must be 1..8");
    if (sched.engine_tiles > 8 || (sched.engine_tiles & (sched.engine_tiles - 1)))
        fail(GSI_E_INVALID, "schedule engine_tiles must be 0, 1, 2, 4 or 8");
    std::vector<HostQuery> hq(nq);
    for (uint32_t i = 0; i < nq; i++) {
        try {
            hq[i] = validate_query(qd[i].k, qd[i].vertex_labels, qd[i].n_edges, qd[i].src, qd[i].dst,
                                   qd[i].edge_labels);
        } catch (const Fail &f) {
            std::string m = std::string("query ") + std::to_string(i) + ": " + gsi_last_error();
            fail(f.st, "%s", m.c_str());
        }
    }
    std::unique_ptr<gsi_batch> b(new gsi_batch());
    b->ctx = c;
    b->nq = nq;
    b->count_only = (flags & GSI_COUNT_ONLY) != 0;
    b->slots.reset(new Slot[nq]);
    b->info.queries = nq;
    b->info.schedule = sched;
    std::vector<const HostQuery *> hp(nq);
    std::vector<Slot *> sp(nq);
    for (uint32_t i = 0; i < nq; i++) {
        hp[i] = &hq[i];
        sp[i] = &b->slots[i];
    }
    AdmitStats as;
    std::vector<WideQuery> wq = admit_round(g, hp, sp, {}, b->count_only, (flags & GSI_BATCH_LEVELS_ONLY) != 0,
                                            sched, &as);
    auto tw0 = std::chrono::steady_clock::now();
    wide_run(g, wq, b->count_only, sched.engine_tiles);
    for (auto &x : wq) finish_slot(x, b->slots[x.qi]);
    b->info.empty = as.empty;
    b->info.tier1 = as.tier1;
    b->info.tier2 = as.tier2;
    b->info.per_level = as.wide + as.single;
    b->info.filter_ms = as.filter_ms;
    b->info.tier1_ms = as.tier1_ms;
    b->info.tier2_ms = as.tier2_ms;
    b->info.per_level_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tw0).count();
    b->info.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return b.release();
}

}  // namespace gsi

using namespace gsi;

namespace {
const Slot &entry(const gsi_batch *b, uint32_t qi) {
    if (!b) fail(GSI_E_INVALID, "null batch");
    if (qi >= b->nq) fail(GSI_E_INVALID, "query index %u out of range (batch of %u)", qi, b->nq);
    return b->slots[qi];
}
}  // namespace

extern "C" {

gsi_status gsi_batch_run(gsi_graph *g, uint32_t nq, const gsi_query_desc *qs, const gsi_batch_options *opt,
                         gsi_batch **out) {
    GSI_TRY({
        if (!g || !out || (nq && !qs)) fail(GSI_E_INVALID, "null argument");
        if (g->multi) fail(GSI_E_INVALID, "multi-labelled graphs run through gsi_query_run_multi only");
        *out = nullptr;
        gsi_batch_schedule sc = opt ? opt->schedule : gsi_batch_schedule{0, 0};
        if (sc.threads == 0) sc = g->tuned;
        if (sc.threads == 0) sc = gsi_batch_schedule{256, 8, 0};
        gsi_ctx *c = g->ctx;
        Busy busy(c);
        GSI_HIP(hipSetDevice(c->device));
        *out = run_batch(g, nq, qs, opt ? opt->flags : 0u, sc);
    })
}

gsi_status gsi_batch_count(const gsi_batch *b, uint32_t qi, uint64_t *rows) {
    GSI_TRY({
        const auto &e = entry(b, qi);
        if (!rows) fail(GSI_E_INVALID, "null argument");
        *rows = e.count;
    })
}

gsi_status gsi_batch_digest(const gsi_batch *b, uint32_t qi, uint64_t out[2]) {
    GSI_TRY({
        const auto &e = entry(b, qi);
        if (!out) fail(GSI_E_INVALID, "null argument");
        out[0] = e.digest[0];
        out[1] = e.digest[1];
    })
}

gsi_status gsi_batch_results(const gsi_batch *b, uint64_t *counts, uint64_t *digests) {
    GSI_TRY({
        if (!b || !counts || !digests) fail(GSI_E_INVALID, "null argument");
        for (uint32_t qi = 0; qi < b->nq; qi++) {
            counts[qi] = b->slots[qi].count;
            digests[2 * (uint64_t)qi] = b->slots[qi].digest[0];
            digests[2 * (uint64_t)qi + 1] = b->slots[qi].digest[1];
        }
    })
}

gsi_status gsi_batch_rows(const gsi_batch *b, uint32_t qi, uint32_t *dst, uint64_t cap) {
    GSI_TRY({
        const auto &e = entry(b, qi);
        if (b->count_only) fail(GSI_E_INVALID, "batch was run with GSI_COUNT_ONLY");
        if (cap < e.count) fail(GSI_E_CAPACITY, "need %llu rows", (unsigned long long)e.count);
        if (e.count == 0) return GSI_OK;
        if (!dst) fail(GSI_E_INVALID, "null buffer");
        gsi_ctx *c = b->ctx;
        GSI_HIP(hipSetDevice(c->device));
        GSI_HIP(hipMemcpyAsync(dst, e.rows, e.count * e.k * 4, hipMemcpyDeviceToHost, c->stream));
        GSI_HIP(hipStreamSynchronize(c->stream));
    })
}

gsi_status gsi_batch_get_info(const gsi_batch *b, gsi_batch_info *out) {
    GSI_TRY({
        if (!b || !out) fail(GSI_E_INVALID, "null argument");
        *out = b->info;
    })
}

gsi_status gsi_batch_free(gsi_batch *b) {
    GSI_TRY({
        if (!b) return GSI_OK;
        gsi_ctx *c = b->ctx;
        GSI_HIP(hipSetDevice(c->device));
        GSI_HIP(hipStreamSynchronize(c->stream));
        delete b;
    })
}

gsi_status gsi_batch_tune(gsi_graph *g, uint32_t nq, const gsi_query_desc *qs, uint32_t sample,
                          gsi_batch_schedule *out, double *out_ms) {
    GSI_TRY({
        if (!g || !out || (nq && !qs)) fail(GSI_E_INVALID, "null argument");
        if (g->multi) fail(GSI_E_INVALID, "multi-labelled graphs run through gsi_query_run_multi only");
        gsi_ctx *c = g->ctx;
        Busy busy(c);
        GSI_HIP(hipSetDevice(c->device));
        const uint32_t n = std::max<uint32_t>(1, std::min(nq, sample ? sample : 128u));
        if (nq == 0) fail(GSI_E_INVALID, "no queries to tune on");
        const gsi_batch_schedule cands[] = {{64, 8, 0},  {64, 4, 0},   {256, 8, 0},
                                            {256, 4, 0}, {1024, 8, 0}, {1024, 4, 0}};
        double best = 1e300;
        gsi_batch_schedule win{256, 8, 0};
        auto trial = [&](const gsi_batch_schedule &sc) {
            auto t0 = std::chrono::steady_clock::now();
            gsi_batch *b = run_batch(g, n, qs, GSI_COUNT_ONLY, sc);
            double ms = ms_since(t0);
            delete b;
            if (ms < best) {
                best = ms;
                win = sc;
            }
        };
        for (const auto &sc : cands) trial(sc);
        // the engine's tiles per workgroup, with the fused tiers chosen
        const gsi_batch_schedule tiers = win;
        for (uint32_t tiles : {1u, 2u, 8u}) trial(gsi_batch_schedule{tiers.threads, tiers.grid_scale, tiles});
        if (win.engine_tiles == 0) win.engine_tiles = 4;
        g->tuned = win;
        *out = win;
        if (out_ms) *out_ms = best / n;
    })
}

}  // extern "C"
