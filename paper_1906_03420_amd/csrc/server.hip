// The serving loop: continuous batching over one resident graph.
//
// Requests wait in arrival order.  Every step admits what the in-flight cap
// and the table budget allow (predicted intermediate-table bytes, see
// predict_peak), runs the admitted set through the batched admission round
// (filter, plans, root tables, fused tiers) and then advances every query in
// the level-synchronous engine by one join level, so that queries admitted
// at different times share the same launches.
#include <algorithm>
#include <chrono>
#include <deque>
#include <memory>
#include <unordered_map>

#include "admit.h"
#include "gsi_internal.h"
#include "wide.h"

namespace gsi {

struct Request {
    uint64_t ticket = 0;
    HostQuery q;
    Slot slot;
    uint64_t pred_pre = 0;   // bytes predicted at submission
    uint64_t pred_now = 0;   // bytes predicted for what is left
    uint64_t peak = 0;       // largest table held between steps
    uint32_t levels = 0;
    double t_submit = 0, t_admit = -1, t_done = -1;
};

}  // namespace gsi

struct gsi_server {
    gsi_graph *g = nullptr;
    gsi_ctx *ctx = nullptr;
    bool count_only = false, solo = true;
    uint32_t max_inflight = 1024, max_admit = 256, solo_queue = 2;
    uint64_t budget = 0;
    gsi_batch_schedule sched{256, 8, 0};
    std::vector<uint64_t> nv;  // vertices per vertex label
    std::unordered_map<uint64_t, std::unique_ptr<gsi::Request>> reqs;
    std::deque<uint64_t> waiting, answered;
    std::unique_ptr<gsi::WideEngine> engine;
    uint64_t next_ticket = 1;
    uint64_t inflight_pred = 0;
    gsi_server_info info{};
    std::chrono::steady_clock::time_point t0;
};

namespace gsi {

static double now_ms(const gsi_server *s) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - s->t0).count();
}

static uint64_t clamp_bytes(double b) {
    if (!(b > 0)) return 0;
    if (b > 4.0e18) return 4000000000000000000ull;
    return (uint64_t)b;
}

// Predicted largest step (bytes held at once) of the join levels j0..k-1 of a
// query whose table has R rows before level j0, following Algorithm 3: the
// e0 lists of a level hold R times the mean |N(v,l)| of the PCSR of l
// (2|E_l| over its |V(D_l)| vertices, Sec. IV); a fraction |C(u)|/|V(D_l)|
// of them are candidates, and every other linking edge keeps a vertex with
// probability mean |N(v,l')| / |V(D_l')|.  A step holds the current table,
// the per-row lookups and offsets, the |GBA| keep bitmap and the next table
// (or the result rows).
static uint64_t predict_peak(const gsi_graph *g, const HostQuery &q, const std::vector<uint32_t> &order,
                             const std::vector<uint32_t> &e0src, const std::vector<uint32_t> &cand, uint32_t j0,
                             double R, bool count_only) {
    const uint32_t k = q.k;
    std::vector<uint32_t> pos(k, NONE32);
    for (uint32_t i = 0; i < k; i++) pos[order[i]] = i;
    double peak = 4.0 * j0 * R;
    for (uint32_t j = j0; j < k; j++) {
        const uint32_t u = order[j];
        double fan0 = 0, keep = 1, ne = 0;
        for (auto &p : q.adj[u]) {
            if (pos[p.first] >= j) continue;
            const uint32_t l = p.second;
            const double Gl = l < g->nlab ? (double)g->G[l] : 0.0;
            const double fan = Gl > 0 ? 2.0 * (double)g->edges[l] / Gl : 0.0;
            ne += 1;
            if (p.first == e0src[j]) {
                fan0 = fan;
                keep *= Gl > 0 ? std::min(1.0, (double)cand[u] / Gl) : 0.0;
            } else {
                keep *= Gl > 0 ? std::min(1.0, fan / Gl) : 0.0;
            }
        }
        const double gba = R * fan0;
        const double S = gba * keep;
        const bool last = j + 1 == k;
        const double next = last ? (count_only ? 0.0 : 4.0 * k * S) : 4.0 * (j + 1) * S;
        const double step = 4.0 * j * R + R * (8.0 * ne + 20.0) + gba / 8.0 + next;
        peak = std::max(peak, step);
        R = S;
    }
    return clamp_bytes(peak);
}

// Prediction before the filter has run: |C(u)| taken as the number of
// vertices with u's label, and the plan Algorithm 2 gives for those counts.
static uint64_t predict_submitted(const gsi_server *s, const HostQuery &q) {
    std::vector<uint32_t> cand(q.k);
    for (uint32_t u = 0; u < q.k; u++) {
        const uint32_t L = q.vl[u];
        cand[u] = L < s->nv.size() ? (uint32_t)std::min<uint64_t>(s->nv[L], 0xFFFFFFFFu) : 0u;
        if (cand[u] == 0) return 0;  // the filter will answer it
    }
    if (q.k < 2) return clamp_bytes(4.0 * cand[0]);
    std::vector<uint32_t> order, e0src;
    make_plan(s->g, q, cand, order, e0src);
    return predict_peak(s->g, q, order, e0src, cand, 1, (double)cand[order[0]], s->count_only);
}

static void answer(gsi_server *s, Request &r) {
    r.t_done = now_ms(s);
    r.pred_now = 0;
    s->answered.push_back(r.ticket);
    s->info.answered++;
}

static void refresh_predictions(gsi_server *s) {
    uint64_t sum = 0;
    for (auto &x : s->engine->queries()) {
        if (x.done) continue;
        Request &r = *s->reqs.at(x.tag);
        r.peak = std::max<uint64_t>(r.peak, 4ull * x.j * x.R);
        r.pred_now = predict_peak(s->g, r.q, x.order, x.e0src, x.cand, x.j, (double)x.R, s->count_only);
        sum += r.pred_now;
    }
    s->inflight_pred = sum;
}

// Admits `adm` (already taken off the waiting queue).  An arena failure
// retries on the first half; a single query that cannot be admitted while
// nothing else is in flight is answered with GSI_E_NOMEM.
static uint32_t admit(gsi_server *s, std::vector<Request *> adm) {
    uint32_t finished = 0;
    while (!adm.empty()) {
        std::vector<const HostQuery *> hq;
        std::vector<Slot *> sl;
        std::vector<uint64_t> tags;
        for (auto *r : adm) {
            hq.push_back(&r->q);
            sl.push_back(&r->slot);
            tags.push_back(r->ticket);
        }
        AdmitStats st;
        std::vector<WideQuery> wq;
        try {
            wq = admit_round(s->g, hq, sl, tags, s->count_only, false, s->sched, &st);
        } catch (const Fail &f) {
            if (f.st != GSI_E_NOMEM) throw;
            clear_error();
            for (auto *r : adm) r->slot.reset();
            if (adm.size() > 1 || s->engine->in_flight() > 0) {
                // put the back half (or, alone, the query itself) in front
                // of the queue again, in order
                const size_t keep = adm.size() > 1 ? adm.size() / 2 : 0;
                for (size_t i = adm.size(); i-- > keep;) s->waiting.push_front(adm[i]->ticket);
                adm.resize(keep);
                continue;
            }
            Request &r = *adm[0];
            r.slot.ctx = s->ctx;
            r.slot.k = r.q.k;
            r.slot.done = true;
            r.slot.status = GSI_E_NOMEM;
            r.t_admit = now_ms(s);
            s->info.admitted++;
            answer(s, r);
            return finished + 1;
        }
        s->info.admit_rounds++;
        const double t = now_ms(s);
        for (auto *r : adm) {
            r->t_admit = t;
            s->info.admitted++;
            if (r->slot.done) {
                answer(s, *r);
                finished++;
            }
        }
        for (auto &x : wq) {
            Request &r = *s->reqs.at(x.tag);
            r.peak = 4ull * x.R;
            r.pred_now = predict_peak(s->g, r.q, x.order, x.e0src, x.cand, 1, (double)x.R, s->count_only);
            s->inflight_pred += r.pred_now;
            s->engine->add(std::move(x));
        }
        break;
    }
    return finished;
}

// Low load: the oldest request alone through the single-query path.
static uint32_t solo_step(gsi_server *s) {
    const auto ta = std::chrono::steady_clock::now();
    Request &r = *s->reqs.at(s->waiting.front());
    s->waiting.pop_front();
    r.t_admit = now_ms(s);
    s->info.admitted++;
    s->info.solo++;
    r.slot.ctx = s->ctx;
    r.slot.k = r.q.k;
    gsi_query_options o{};
    o.flags = s->count_only ? GSI_COUNT_ONLY : 0u;
    try {
        gsi_result *res = run_query(s->g, r.q, &o);
        r.slot.res = res;
        r.slot.rows = res->rows;
        r.slot.count = res->count;
        r.slot.digest[0] = res->digest[0];
        r.slot.digest[1] = res->digest[1];
        r.peak = 0;
    } catch (const Fail &f) {
        if (f.st != GSI_E_NOMEM) throw;
        clear_error();
        r.slot.status = GSI_E_NOMEM;
        r.slot.count = 0;
    }
    r.slot.path = PATH_SOLO;
    r.slot.done = true;
    answer(s, r);
    s->info.admit_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - ta).count();
    s->info.steps++;
    return 1;
}

static uint32_t server_step(gsi_server *s) {
    if (s->solo && s->engine->in_flight() == 0 && !s->waiting.empty() && s->waiting.size() <= s->solo_queue)
        return solo_step(s);
    uint32_t finished = 0;
    const auto ta = std::chrono::steady_clock::now();
    std::vector<Request *> adm;
    uint64_t pred = s->inflight_pred;
    const size_t inflight = s->engine->in_flight();
    while (!s->waiting.empty() && adm.size() < s->max_admit && inflight + adm.size() < s->max_inflight) {
        Request *r = s->reqs.at(s->waiting.front()).get();
        const bool alone = inflight == 0 && adm.empty();
        if (!alone && pred + r->pred_pre > s->budget) break;
        pred += r->pred_pre;
        adm.push_back(r);
        s->waiting.pop_front();
    }
    if (!adm.empty()) finished += admit(s, std::move(adm));
    s->info.peak_predicted = std::max(s->info.peak_predicted, s->inflight_pred);
    const auto tl = std::chrono::steady_clock::now();
    s->info.admit_ms += std::chrono::duration<double, std::milli>(tl - ta).count();
    if (!s->engine->idle()) {
        s->engine->step();
        s->info.level_steps++;
        for (auto &x : s->engine->take_done()) {
            Request &r = *s->reqs.at(x.tag);
            r.levels = x.levels;
            finish_slot(x, r.slot);
            answer(s, r);
            finished++;
        }
        refresh_predictions(s);
    }
    s->info.level_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tl).count();
    s->info.steps++;
    return finished;
}

static Request &answered_request(const gsi_server *s, uint64_t ticket) {
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) fail(GSI_E_INVALID, "unknown or released ticket %llu", (unsigned long long)ticket);
    Request &r = *it->second;
    if (!r.slot.done) fail(GSI_E_INVALID, "ticket %llu is not answered yet", (unsigned long long)ticket);
    return r;
}

}  // namespace gsi

using namespace gsi;

extern "C" {

gsi_status gsi_server_create(gsi_graph *g, const gsi_server_options *opt, gsi_server **out) {
    GSI_TRY({
        if (!g || !out) fail(GSI_E_INVALID, "null argument");
        if (g->multi) fail(GSI_E_INVALID, "multi-labelled graphs run through gsi_query_run_multi only");
        *out = nullptr;
        gsi_server_options o = opt ? *opt : gsi_server_options{};
        if (o.flags & ~(GSI_COUNT_ONLY | GSI_SERVER_NO_SOLO)) fail(GSI_E_INVALID, "unknown server flag");
        gsi_batch_schedule sc = o.schedule;
        if (sc.threads == 0) sc = g->tuned;
        if (sc.threads == 0) sc = gsi_batch_schedule{256, 8, 0};
        if (sc.threads != 64 && sc.threads != 256 && sc.threads != 1024)
            fail(GSI_E_INVALID, "schedule threads must be 64, 256 or 1024");
        if (sc.grid_scale < 1 || sc.grid_scale > 8) fail(GSI_E_INVALID, "schedule grid_scale must be 1..8");
        if (sc.engine_tiles > 8 || (sc.engine_tiles & (sc.engine_tiles - 1)))
            fail(GSI_E_INVALID, "schedule engine_tiles must be 0, 1, 2, 4 or 8");
        gsi_ctx *c = g->ctx;
        Busy busy(c);
        GSI_HIP(hipSetDevice(c->device));
        std::unique_ptr<gsi_server> s(new gsi_server());
        s->g = g;
        s->ctx = c;
        s->count_only = (o.flags & GSI_COUNT_ONLY) != 0;
        s->max_inflight = o.max_inflight ? o.max_inflight : 1024u;
        s->max_admit = o.max_admit ? o.max_admit : 256u;
        s->solo = !(o.flags & GSI_SERVER_NO_SOLO);
        s->solo_queue = o.solo_queue ? o.solo_queue : 2u;
        s->budget = o.table_budget ? o.table_budget : c->arena.largest_free() / 2;
        s->sched = sc;
        s->engine.reset(new WideEngine(g, s->count_only, true, sc.engine_tiles));
        // vertices per label: word 0 of every signature is the exact label
        std::vector<uint32_t> lab(g->n);
        GSI_HIP(hipMemcpyAsync(lab.data(), g->sig, 4ull * g->n, hipMemcpyDeviceToHost, c->stream));
        sync(c);
        uint32_t maxl = 0;
        for (uint32_t x : lab) maxl = std::max(maxl, x);
        s->nv.assign((size_t)maxl + 1, 0);
        for (uint32_t x : lab) s->nv[x]++;
        s->info.table_budget = s->budget;
        s->t0 = std::chrono::steady_clock::now();
        *out = s.release();
    })
}

gsi_status gsi_server_submit(gsi_server *s, const gsi_query_desc *qd, uint64_t *ticket) {
    GSI_TRY({
        if (!s || !qd || !ticket) fail(GSI_E_INVALID, "null argument");
        *ticket = 0;
        std::unique_ptr<Request> r(new Request());
        r->q = validate_query(qd->k, qd->vertex_labels, qd->n_edges, qd->src, qd->dst, qd->edge_labels);
        r->ticket = s->next_ticket++;
        r->t_submit = now_ms(s);
        r->pred_pre = predict_submitted(s, r->q);
        s->waiting.push_back(r->ticket);
        *ticket = r->ticket;
        s->reqs.emplace(r->ticket, std::move(r));
        s->info.submitted++;
    })
}

gsi_status gsi_server_step(gsi_server *s, uint32_t *finished) {
    GSI_TRY({
        if (!s) fail(GSI_E_INVALID, "null argument");
        if (finished) *finished = 0;
        Busy busy(s->ctx);
        GSI_HIP(hipSetDevice(s->ctx->device));
        const uint32_t n = server_step(s);
        if (finished) *finished = n;
    })
}

gsi_status gsi_server_poll(gsi_server *s, uint64_t *tickets, uint32_t capacity, uint32_t *n) {
    GSI_TRY({
        if (!s || !n || (capacity && !tickets)) fail(GSI_E_INVALID, "null argument");
        uint32_t i = 0;
        while (i < capacity && !s->answered.empty()) {
            tickets[i++] = s->answered.front();
            s->answered.pop_front();
        }
        *n = i;
    })
}

gsi_status gsi_server_answer_get(const gsi_server *s, uint64_t ticket, gsi_server_answer *out) {
    GSI_TRY({
        if (!s || !out) fail(GSI_E_INVALID, "null argument");
        const Request &r = answered_request(s, ticket);
        gsi_server_answer a{};
        a.status = r.slot.status;
        a.k = r.q.k;
        a.count = r.slot.count;
        a.digest[0] = r.slot.digest[0];
        a.digest[1] = r.slot.digest[1];
        a.path = r.slot.path;
        a.levels = r.levels;
        a.predicted_bytes = r.pred_pre;
        a.peak_table_bytes = r.peak;
        a.submit_ms = r.t_submit;
        a.admit_ms = r.t_admit;
        a.done_ms = r.t_done;
        *out = a;
    })
}

gsi_status gsi_server_rows(gsi_server *s, uint64_t ticket, uint32_t *dst, uint64_t cap) {
    GSI_TRY({
        if (!s) fail(GSI_E_INVALID, "null argument");
        const Request &r = answered_request(s, ticket);
        if (s->count_only) fail(GSI_E_INVALID, "server was created with GSI_COUNT_ONLY");
        if (r.slot.status != GSI_OK) fail(GSI_E_INVALID, "ticket %llu has no rows (status %d)",
                                          (unsigned long long)ticket, (int)r.slot.status);
        if (cap < r.slot.count) fail(GSI_E_CAPACITY, "need %llu rows", (unsigned long long)r.slot.count);
        if (r.slot.count == 0) return GSI_OK;
        if (!dst) fail(GSI_E_INVALID, "null buffer");
        Busy busy(s->ctx);
        GSI_HIP(hipSetDevice(s->ctx->device));
        GSI_HIP(hipMemcpyAsync(dst, r.slot.rows, r.slot.count * r.q.k * 4, hipMemcpyDeviceToHost, s->ctx->stream));
        GSI_HIP(hipStreamSynchronize(s->ctx->stream));
    })
}

gsi_status gsi_server_release(gsi_server *s, uint64_t ticket) {
    GSI_TRY({
        if (!s) fail(GSI_E_INVALID, "null argument");
        answered_request(s, ticket);
        Busy busy(s->ctx);
        GSI_HIP(hipSetDevice(s->ctx->device));
        // a later launch may still read nothing of it, but the copy out of
        // it may be in flight on the stream
        GSI_HIP(hipStreamSynchronize(s->ctx->stream));
        s->reqs.erase(ticket);
        s->info.released++;
    })
}

gsi_status gsi_server_get_info(const gsi_server *s, gsi_server_info *out) {
    GSI_TRY({
        if (!s || !out) fail(GSI_E_INVALID, "null argument");
        gsi_server_info i = s->info;
        i.waiting = (uint32_t)s->waiting.size();
        i.in_flight = (uint32_t)s->engine->in_flight();
        i.predicted_in_flight = s->inflight_pred;
        *out = i;
    })
}

gsi_status gsi_server_free(gsi_server *s) {
    GSI_TRY({
        if (!s) return GSI_OK;
        Busy busy(s->ctx);
        GSI_HIP(hipSetDevice(s->ctx->device));
        GSI_HIP(hipStreamSynchronize(s->ctx->stream));
        s->engine.reset();
        s->reqs.clear();
        delete s;
    })
}

}  // extern "C"
