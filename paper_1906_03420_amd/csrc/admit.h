// Admission of a set of queries (shared by the batched path and the server):
// filter, plans, root tables and the fused tiers; what they cannot finish is
// returned for the level-synchronous engine.
#pragma once

#include <memory>

#include "gsi_internal.h"
#include "wide.h"

namespace gsi {

// device blocks of one admission round, released with the last owner
struct Round {
    gsi_ctx *ctx = nullptr;
    Round() = default;
    Round(const Round &) = delete;
    Round &operator=(const Round &) = delete;
    void *bits = nullptr;  // candidate bitsets of every query vertex
    void *m0 = nullptr;    // root tables
    uint32_t *out = nullptr;  // rows written by the fused tiers
    ~Round() {
        if (!ctx) return;
        ctx->arena.release(bits);
        ctx->arena.release(m0);
        ctx->arena.release(out);
    }
};

// where one query's answer lives
enum SlotPath : uint8_t {
    PATH_NONE = 0, PATH_TIER1 = 1, PATH_TIER2 = 2, PATH_SINGLE = 3, PATH_LEVELS = 4, PATH_SOLO = 5
};

struct Slot {
    uint32_t k = 0;
    bool done = false;
    uint8_t path = PATH_NONE;         // which engine produced the answer
    gsi_status status = GSI_OK;
    uint64_t count = 0;
    uint64_t digest[2] = {0, 0};
    const uint32_t *rows = nullptr;  // device rows (count x k), if any
    uint32_t *own = nullptr;         // arena block owned by the slot
    gsi_result *res = nullptr;       // or a result of the single-query path
    std::shared_ptr<Round> keep;     // or rows inside a round's output block
    gsi_ctx *ctx = nullptr;
    void clear() {
        if (res) {
            ctx->arena.release(res->rows);
            delete res;
        }
        if (own) ctx->arena.release(own);
        res = nullptr;
        own = nullptr;
        rows = nullptr;
        keep.reset();
    }
    // back to "not answered" (an admission that has to be retried)
    void reset() {
        if (ctx) clear();
        done = false;
        path = PATH_NONE;
        status = GSI_OK;
        count = 0;
        digest[0] = digest[1] = 0;
    }
    Slot() = default;
    Slot(const Slot &) = delete;
    Slot &operator=(const Slot &) = delete;
    ~Slot() {
        if (ctx) clear();
    }
};

struct AdmitStats {
    uint32_t empty = 0, tier1 = 0, tier2 = 0, single = 0, wide = 0;
    double filter_ms = 0, tier1_ms = 0, tier2_ms = 0;
};

// Admits queries hq[i] (answers go to slots[i]): finished ones get their
// slot filled; the others come back as WideQuery objects (tag = tags[i]).
std::vector<WideQuery> admit_round(gsi_graph *g, const std::vector<const HostQuery *> &hq,
                                   const std::vector<Slot *> &slots, const std::vector<uint64_t> &tags,
                                   bool count_only, bool levels_only, gsi_batch_schedule sched, AdmitStats *st);

// Moves a finished WideQuery's answer into its slot.
void finish_slot(WideQuery &x, Slot &sl);

}  // namespace gsi
