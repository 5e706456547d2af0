// Level-synchronous joins of many queries (wide.hip).
#pragma once

#include <memory>

#include "gsi_internal.h"

namespace gsi {

// one query in the level-synchronous engine
struct WideQuery {
    gsi_ctx *ctx = nullptr;
    const HostQuery *q = nullptr;
    uint32_t qi = 0;                      // index in the caller's batch
    uint64_t tag = 0;                     // caller's handle (request id)
    std::shared_ptr<void> keep;           // keeps the bitsets / root tables alive
    std::vector<uint32_t> order, e0src;   // Algorithm 2 order, first edges
    std::vector<uint32_t> cand;           // |C(u)| per query vertex
    std::vector<uint32_t> col;            // query vertex -> column
    std::vector<const uint64_t *> Cu;     // level j: bitset C(order[j])
    uint32_t j = 1;                       // next level to join
    const uint32_t *M = nullptr;          // current table (column-major)
    uint64_t R = 0;
    void *own = nullptr;                  // arena block of M when owned
    void *next = nullptr;
    bool done = false;
    gsi_status status = GSI_OK;           // GSI_E_NOMEM: a level did not fit alone
    uint64_t count = 0;
    uint64_t digest[2] = {0, 0};
    uint32_t *rows = nullptr;             // result rows (arena, high end)
    uint32_t levels = 0;
    uint64_t stats_rows[GSI_MAX_K] = {0}, stats_gba[GSI_MAX_K] = {0}, stats_surv[GSI_MAX_K] = {0};

    void release_table() {
        if (own) ctx->arena.release(own);
        own = nullptr;
    }
    void finish_empty() {
        release_table();
        count = 0;
        done = true;
    }
    // hands the result rows to the caller
    uint32_t *take_rows() {
        uint32_t *r = rows;
        rows = nullptr;
        return r;
    }
    WideQuery() = default;
    WideQuery(const WideQuery &) = delete;
    WideQuery &operator=(const WideQuery &) = delete;
    WideQuery(WideQuery &&o) noexcept { *this = std::move(o); }
    WideQuery &operator=(WideQuery &&o) noexcept {
        ctx = o.ctx; q = o.q; qi = o.qi; tag = o.tag; keep = std::move(o.keep); order = std::move(o.order); e0src = std::move(o.e0src); cand = std::move(o.cand);
        col = std::move(o.col); Cu = std::move(o.Cu); j = o.j; M = o.M; R = o.R; own = o.own; next = o.next;
        done = o.done; status = o.status; count = o.count; digest[0] = o.digest[0]; digest[1] = o.digest[1]; rows = o.rows;
        levels = o.levels;
        for (int i = 0; i < GSI_MAX_K; i++) {
            stats_rows[i] = o.stats_rows[i];
            stats_gba[i] = o.stats_gba[i];
            stats_surv[i] = o.stats_surv[i];
        }
        o.own = o.next = nullptr;
        o.rows = nullptr;
        return *this;
    }
    ~WideQuery() {
        if (!ctx) return;
        if (own) ctx->arena.release(own);
        if (next) ctx->arena.release(next);
        if (rows) ctx->arena.release(rows);
    }
};

// Holds queries in flight; each step() advances the active ones by one
// join level in shared launches (a prefix of them when the arena cannot
// hold a step for all: a step that fails to allocate is retried on half as
// many queries, the others keep their state).  A query whose level does not
// fit even alone raises GSI_E_NOMEM, or, in a tolerant engine, is moved
// behind the others; when it is the only query left it is finished with
// status GSI_E_NOMEM.
class WideEngine {
  public:
    // tiles: 256-slot tiles per workgroup of the join and link (1, 2, 4 or
    // 8; anything else: 4)
    WideEngine(gsi_graph *g, bool count_only, bool tolerant = false, uint32_t tiles = 0);
    void add(WideQuery &&q);
    bool idle() const;
    uint32_t step();                   // returns how many are done now
    std::vector<WideQuery> take_done();  // removes and returns finished queries
    size_t in_flight() const { return qs_.size(); }
    uint64_t steps() const { return steps_; }
    std::vector<WideQuery> &queries() { return qs_; }

  private:
    gsi_graph *g_;
    bool count_only_, tolerant_;
    uint32_t tpw_;
    std::vector<WideQuery> qs_;
    uint64_t steps_ = 0;
};

// Runs every query of `wq` to completion (count, digest and, unless
// count_only, rows); `wq` comes back holding the finished queries.
void wide_run(gsi_graph *g, std::vector<WideQuery> &wq, bool count_only, uint32_t tiles = 0);

}  // namespace gsi
