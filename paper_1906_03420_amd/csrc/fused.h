// Descriptor and status of the fused small-table join (fused.hip).
#pragma once

#include "gsi_internal.h"

namespace gsi {

constexpr uint32_t FUSED_MAX_ROWS = 4096;    // rows of any table the workgroup holds
constexpr uint32_t FUSED_MAX_SLOTS = 16384;  // |GBA| of any level it joins
constexpr uint32_t FSTATUS_IN_FIRST = 2;     // M is still the first table

struct FEdge {            // one linking edge of a level
    const uint32_t *gl;   // PCSR groups of its label
    const uint32_t *ci;   // neighbour lists of its label
    uint32_t G, H;        // groups, home groups
    uint32_t col;         // column of M with the placed endpoint
    uint32_t pad;
};

struct FPlan {
    uint32_t k, count_only, cap_rows, cap_slots;
    uint32_t qcol[GSI_MAX_K];     // query vertex -> column
    uint32_t lv_ne[GSI_MAX_K];    // level j: linking edges
    uint32_t lv_e0[GSI_MAX_K];    // level j: first edge (index within the level)
    uint32_t lv_first[GSI_MAX_K]; // level j: first entry in edges[]
    const uint64_t *Cu[GSI_MAX_K];
    FEdge edges[1];               // all levels' edges follow
};

inline size_t fplan_bytes(uint32_t n_edges) {
    return sizeof(FPlan) + (n_edges ? n_edges - 1 : 0) * sizeof(FEdge);
}

struct FStatus {
    uint64_t done;    // 1: every level finished (count/digest valid)
    uint64_t level;   // else: level the workgroup could not hold
    uint64_t rows;    // rows of M entering that level
    uint64_t mloc;    // M's buffer: 0, 1, or FSTATUS_IN_FIRST
    uint64_t levels;  // levels finished
    uint64_t count;
    uint64_t digest[2];
    uint64_t lv_rows[GSI_MAX_K], lv_gba[GSI_MAX_K], lv_surv[GSI_MAX_K];
};

// one query of a batch: where its plan, root table and output rows live
struct FBatchItem {
    uint64_t plan_off;  // byte offset of its FPlan in the plan buffer
    uint64_t m0_off;    // first root row in the concatenated root tables
    uint64_t out_off;   // first output word in the output buffer
    uint32_t R0;        // root rows
    uint32_t pad;
};

// a workgroup size of the persistent batch kernel and what it can hold
struct FTier {
    uint32_t threads;    // 64, 256 or 1024
    uint32_t cap_rows;   // 4 x threads
    uint32_t cap_slots;  // 16 x threads
    uint32_t blocks_per_cu;
};
FTier fused_tier(uint32_t threads);
void launch_fused_batch(gsi_ctx *c, const FTier &t, uint32_t grid, const uint8_t *plans, const FBatchItem *items,
                        uint32_t nitems, const uint32_t *M0all, uint32_t *scratch, uint64_t slot_words, uint32_t kmax,
                        uint32_t *outall, FStatus *sts, uint32_t *counter, double bytes);

void launch_fused(gsi_ctx *c, const FPlan *d_plan, const uint32_t *M0, uint32_t R0, uint32_t *buf0, uint32_t *buf1,
                  uint32_t *loc, uint32_t *out, FStatus *d_status, double alg_bytes);

}  // namespace gsi
