// Descriptor and status of the fused small-table join (fused.hip).
#pragma once

#include "gsi_internal.h"

namespace gsi {

constexpr uint32_t FUSED_MAX_ROWS = 4096;    // rows of any table the workgroup holds
constexpr uint32_t FUSED_MAX_SLOTS = 16384;  // |GBA| of any level it joins
constexpr uint32_t FSTATUS_IN_FIRST = 2;     // M is still the first table
constexpr uint32_t CHUNK_MIN_ROWS = FUSED_MAX_ROWS + 1;  // root chunks above one workgroup's rows
constexpr uint32_t CHUNK_MAX = 16384;        // chunks of one launch

struct FEdge {            // one linking edge of a level
    const uint32_t *gl;   // PCSR groups of its label
    const uint32_t *ci;   // neighbour lists of its label
    uint32_t G, H;        // groups, home groups
    uint32_t col;         // column of M with the placed endpoint
    uint32_t ci_off;      // offset of its label's lists in the whole ci array
};

// Lookups of the fused kernels: rows x (2 ne + 2) words per level (starts,
// lengths, start of the scanned list in the whole ci array, its edge).
inline uint64_t fused_loc_words(uint32_t k, uint64_t rows) { return 2ull * k * rows; }

struct FPlan {
    uint32_t k, count_only, cap_rows, cap_slots;
    uint32_t pick;                // 1: each row scans its shortest linking list
    uint32_t homo;                // 1: homomorphism (no subtraction of m_i)
    const uint32_t *ci_all;       // every label's lists
    uint32_t qcol[GSI_MAX_K];     // query vertex -> column
    uint32_t lv_ne[GSI_MAX_K];    // level j: linking edges
    uint32_t lv_e0[GSI_MAX_K];    // level j: first edge (index within the level)
    uint32_t lv_first[GSI_MAX_K]; // level j: first entry in edges[]
    uint32_t lv_mmask[GSI_MAX_K]; // level j: columns of m_i whose query vertex
                                  // has u's label (all on multi-labelled graphs)
    const uint64_t *Cu[GSI_MAX_K];
    FEdge edges[1];               // all levels' edges follow
};

constexpr size_t fplan_bytes(uint32_t n_edges) {
    return sizeof(FPlan) + (n_edges ? n_edges - 1 : 0) * sizeof(FEdge);
}

// A plan of up to FPLAN_ARG_EDGES edges passed by value as a kernel argument
// (no upload before the launch); its edges continue into `more`.
constexpr uint32_t FPLAN_ARG_EDGES = 64;
struct FPlanArg {
    FPlan p;
    FEdge more[FPLAN_ARG_EDGES - 1];
};
static_assert(sizeof(FPlanArg) == fplan_bytes(FPLAN_ARG_EDGES), "plan edges are contiguous");
static_assert(sizeof(FPlanArg) <= 3072, "kernel arguments stay under 4 KiB");

struct FStatus {
    uint64_t done;    // 1: every level finished (count/digest valid)
    uint64_t level;   // else: level the workgroup could not hold
    uint64_t rows;    // rows of M entering that level
    uint64_t mloc;    // M's buffer: 0, 1, or FSTATUS_IN_FIRST
    uint64_t levels;  // levels finished
    uint64_t count;
    uint64_t digest[2];
    uint64_t out_base;  // chunked runs: first output word it reserved
    uint64_t lv_rows[GSI_MAX_K], lv_gba[GSI_MAX_K], lv_surv[GSI_MAX_K];
};

// Totals of a chunked run (k_chunk_summary).
struct FChunkSummary {
    uint64_t all_done;  // every chunk finished
    uint64_t count;
    uint64_t digest[2];
    uint64_t levels;    // most levels any chunk ran
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

// One query split into chunks of `chunk_rows` rows of its table M0 (R0
// rows, j0 columns, column stride R0; the rows of M are independent at
// every level of Algorithm 3): a persistent launch of the tier's workgroups
// takes chunks from `counter` and runs levels j0 .. k-1 of each.
// Finished chunks reserve their output rows in `staging` (capacity
// `staging_words`) through `ocount`.  A chunk that cannot hold a level, or
// whose rows do not fit the staging buffer, is left undone; once more than
// `max_fail` chunks are, `abort` (two words: flag, failures) is set and the
// launch stops taking chunks.  The totals of the finished chunks are added
// into `sum` (zeroed by the caller) as they finish; k_chunk_summary then
// writes each chunk's first output row (chunk order), a done flag per chunk
// and the row total.
void launch_fused_chunks(gsi_ctx *c, const FTier &t, uint32_t grid, const FPlan *plan, uint32_t j0, const uint32_t *M0,
                         uint32_t R0, uint32_t chunk_rows, uint32_t nchunks, uint32_t *scratch, uint64_t slot_words,
                         uint32_t k, uint32_t *staging, uint64_t staging_words, unsigned long long *ocount,
                         uint32_t *abort, uint32_t max_fail, FStatus *sts, uint32_t *counter, uint64_t *offs,
                         uint32_t *done, FChunkSummary *sum);
// Rows of the finished chunks into `out` in chunk order, which is the order
// the per-level path gives those roots.
void launch_chunk_gather(gsi_ctx *c, uint32_t nchunks, const FStatus *sts, const uint64_t *offs,
                         const uint32_t *staging, uint32_t k, uint32_t *out, uint64_t words);
// Concatenates the rows (`ncols` columns) of the chunks in `list` (pairs:
// chunk, position) into dst, a table of `rows` rows.
void launch_take_rows(gsi_ctx *c, uint32_t nlist, const uint32_t *M0, uint32_t R0, uint32_t ncols,
                      uint32_t chunk_rows, const uint32_t *list, uint32_t *dst, uint64_t rows);

// The single-workgroup fused kernel, levels j0.. of the table M0 (R0 rows,
// j0 columns, column stride R0); with b0 (the bitset of C(u_first), nwords
// words; j0 = 1 only) it also writes M0 itself, `b0_runs` being the set bits
// of each of the BITS_RUNS runs of that bitset.  The plan is d_plan in
// device memory or, when d_plan is null, `inl`.
void launch_fused(gsi_ctx *c, const FPlan *d_plan, const FPlanArg &inl, uint32_t j0, uint32_t *M0, uint32_t R0,
                  const uint32_t *b0_runs, const uint64_t *b0,
                  uint64_t nwords, uint32_t *buf0, uint32_t *buf1, uint32_t *loc, uint32_t *out, FStatus *d_status,
                  double alg_bytes);

}  // namespace gsi
