// Fused join levels for small tables: one 1024-thread workgroup runs the
// levels of Algorithm 3 (with Algorithm 4's pre-allocation) back to back,
// with F, the GBA keep bits and the survivor prefix sums in LDS, so a level
// costs no kernel launch and no host round trip.  The workgroup stops at the
// first level whose rows, slots (|GBA|) or survivors exceed its capacity and
// reports where; the caller finishes the query from that level with the
// per-level kernels.  Results are identical to the per-level path (same
// tests, same order: parent row, then ascending x).
#include <cstring>

#include "fused.h"
#include "join_device.h"

namespace gsi {

// exclusive prefix sum over v (one value per thread), total in *total
template <uint32_t FT>
__device__ __forceinline__ uint32_t wg_exclusive_sum(uint32_t v, uint32_t *s_w, uint32_t *total) {
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t inc = wave_inclusive_sum(v);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (uint32_t q = 0; q < FT / 64; q++) {
        uint32_t x = s_w[q];
        off += q < w ? x : 0u;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// largest i in [0, R) with F[i] <= p (F in LDS, F[0] = 0 <= p)
__device__ __forceinline__ uint32_t lds_row(const uint32_t *F, uint32_t R, uint32_t p) {
    uint32_t lo = 0, hi = R - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (F[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// LDS of one fused workgroup with FT threads, CR rows and CS slots
template <uint32_t FT, uint32_t CR, uint32_t CS>
struct FusedLds {
    uint32_t F[CR + 1];
    uint64_t bits[CS / 64];
    uint32_t wpre[CS / 64];
    uint32_t w[FT / 64];
    uint64_t d[2][FT / 64];
};

// All join levels of one query in one workgroup (see the file comment).
// FT threads; at most CR rows per table (CR = 4 FT) and CS slots per level.
template <uint32_t FT, uint32_t CR, uint32_t CS>
__device__ void fused_query(const FPlan *plan, const uint32_t *M0, uint32_t R0, uint32_t *buf0, uint32_t *buf1,
                            uint32_t *loc, uint32_t *out, FStatus *st, FusedLds<FT, CR, CS> &L) {
    static_assert(CR == 4 * FT, "each thread scans four rows");
    static_assert(CS / 64 <= FT, "one thread per bitmap word in the survivor scan");
    uint32_t *s_F = L.F;
    uint64_t *s_bits = L.bits;
    uint32_t *s_wpre = L.wpre;
    uint32_t *s_w = L.w;

    const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
    const uint32_t k = plan->k;
    const uint32_t cap_rows = plan->cap_rows < CR ? plan->cap_rows : CR;
    const uint32_t cap_slots = plan->cap_slots < CS ? plan->cap_slots : CS;
    const uint32_t *M = M0;
    uint32_t R = R0;
    uint32_t mloc = FSTATUS_IN_FIRST;  // where M lives
    uint32_t *bufs[2] = {buf0, buf1};
    uint32_t next = 0;

    for (uint32_t j = 1; j < k; j++) {
        const uint32_t ne = plan->lv_ne[j], ef = plan->lv_first[j], e0 = plan->lv_e0[j];
        const uint64_t *Cu = plan->Cu[j];
        const bool final_level = (j == k - 1);
        const FEdge &E0 = plan->edges[ef + e0];
        if (tid == 0) st->lv_rows[j] = R;

        // locate N(v, l) for every row and linking edge; bound = |N(v'_i, l0)|
        for (uint32_t i = tid; i < R; i += FT) {
            for (uint32_t e = 0; e < ne; e++) {
                const FEdge &ed = plan->edges[ef + e];
                const uint32_t v = M[(uint64_t)ed.col * R + i];
                const uint2 r = pcsr_find(ed.gl, ed.G, ed.H, v);
                loc[(uint64_t)e * R + i] = r.x;
                loc[(uint64_t)(ne + e) * R + i] = r.y;
                if (e == e0) s_F[i] = r.y;
            }
        }
        __syncthreads();
        // F = exclusive prefix sum of the bounds (each thread owns 4 rows)
        {
            uint32_t v4[4], sum = 0;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                uint32_t i = 4 * tid + q;
                v4[q] = i < R ? s_F[i] : 0u;
                sum += v4[q];
            }
            uint32_t tot;
            uint32_t run = wg_exclusive_sum<FT>(sum, s_w, &tot);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                uint32_t i = 4 * tid + q;
                if (i < R) s_F[i] = run;
                run += v4[q];
            }
            if (tid == 0) s_F[R] = tot;
            __syncthreads();
        }
        const uint32_t gba = s_F[R];
        if (tid == 0) st->lv_gba[j] = gba;
        if (gba > cap_slots) {
            if (tid == 0) {
                st->level = j;
                st->rows = R;
                st->mloc = mloc;
            }
            return;
        }
        if (gba == 0) {
            if (tid == 0) {
                st->lv_surv[j] = 0;
                st->levels = j;
                st->done = 1;
            }
            return;
        }
        const uint32_t nw = (gba + 63) / 64;

        // join: keep x = N(v'_i, l0)[p - F[i]] iff x not in m_i, x in C(u),
        // x in every other linking list; one ballot word per 64 slots
        for (uint32_t word = w; word < nw; word += FT / 64) {
            const uint32_t p = word * 64 + lane;
            bool keep = false;
            if (p < gba) {
                const uint32_t i = lds_row(s_F, R, p);
                const uint32_t x = E0.ci[loc[(uint64_t)e0 * R + i] + (p - s_F[i])];
                keep = (Cu[x >> 6] >> (x & 63)) & 1ull;
                for (uint32_t c = 0; keep && c < j; c++) keep = M[(uint64_t)c * R + i] != x;
                for (uint32_t e = 0; keep && e < ne; e++) {
                    if (e == e0) continue;
                    keep = in_sorted(plan->edges[ef + e].ci + loc[(uint64_t)e * R + i],
                                     loc[(uint64_t)(ne + e) * R + i], x);
                }
            }
            const uint64_t mask = __ballot(keep);
            if (lane == 0) s_bits[word] = mask;
        }
        __syncthreads();
        // survivor positions: prefix sum of the words' popcounts
        uint32_t S;
        {
            uint32_t c = tid < nw ? (uint32_t)__popcll(s_bits[tid]) : 0u;
            uint32_t ex = wg_exclusive_sum<FT>(c, s_w, &S);
            if (tid < nw) s_wpre[tid] = ex;
            __syncthreads();
        }
        if (tid == 0) st->lv_surv[j] = S;
        if (S == 0) {
            if (tid == 0) {
                st->levels = j;
                st->done = 1;
            }
            return;
        }
        if (!final_level && S > cap_rows) {
            if (tid == 0) {
                st->level = j;
                st->rows = R;
                st->mloc = mloc;
            }
            return;
        }

        // link: (m_i, x) at its position; the last level writes rows in
        // query-vertex order and hashes them
        uint32_t *Mn = bufs[next];
        uint64_t hs = 0, hx = 0;
        for (uint32_t word = w; word < nw; word += FT / 64) {
            const uint64_t bits = s_bits[word];
            if (!((bits >> lane) & 1ull)) continue;
            const uint32_t p = word * 64 + lane;
            const uint32_t pos = s_wpre[word] + rank_below(bits);
            const uint32_t i = lds_row(s_F, R, p);
            const uint32_t x = E0.ci[loc[(uint64_t)e0 * R + i] + (p - s_F[i])];
            if (!final_level) {
                for (uint32_t c = 0; c < j; c++) Mn[(uint64_t)c * S + pos] = M[(uint64_t)c * R + i];
                Mn[(uint64_t)j * S + pos] = x;
            } else {
                uint64_t f = 14695981039346656037ull;
                for (uint32_t u = 0; u < k; u++) {
                    const uint32_t c = plan->qcol[u];
                    const uint32_t val = c < j ? M[(uint64_t)c * R + i] : x;
                    if (!plan->count_only) out[(uint64_t)pos * k + u] = val;
                    f = fnv_word(f, val);
                }
                const uint64_t h = mix64(f);
                hs += h;
                hx ^= h;
            }
        }
        if (final_level) {
            hs = wave_sum(hs);
            hx = wave_xor(hx);
            if (lane == 0) {
                L.d[0][w] = hs;
                L.d[1][w] = hx;
            }
            __syncthreads();
            if (tid == 0) {
                uint64_t ts = 0, tx = 0;
                for (uint32_t q = 0; q < FT / 64; q++) {
                    ts += L.d[0][q];
                    tx ^= L.d[1][q];
                }
                st->digest[0] = ts;
                st->digest[1] = tx;
                st->count = S;
                st->levels = j;
                st->done = 1;
            }
            return;
        }
        __syncthreads();  // M' complete before it is read as M
        M = Mn;
        R = S;
        mloc = next;
        next ^= 1u;
    }
}

__global__ __launch_bounds__(1024) void k_fused_levels(const FPlan *plan, const uint32_t *M0, uint32_t R0,
                                                      uint32_t *buf0, uint32_t *buf1, uint32_t *loc, uint32_t *out,
                                                      FStatus *st) {
    __shared__ FusedLds<1024, FUSED_MAX_ROWS, FUSED_MAX_SLOTS> L;
    fused_query<1024, FUSED_MAX_ROWS, FUSED_MAX_SLOTS>(plan, M0, R0, buf0, buf1, loc, out, st, L);
}

void launch_fused(gsi_ctx *c, const FPlan *d_plan, const uint32_t *M0, uint32_t R0, uint32_t *buf0, uint32_t *buf1,
                  uint32_t *loc, uint32_t *out, FStatus *d_status, double alg_bytes) {
    launch(c, "k_fused_levels", alg_bytes, k_fused_levels, 1, 1024, d_plan, M0, R0, buf0, buf1, loc, out, d_status);
}

// Persistent batch: each workgroup takes the next query from a shared
// counter until none is left (every workgroup leaves once the counter passes
// the item count), and runs all its levels in its own scratch slot.
template <uint32_t FT, uint32_t CR, uint32_t CS>
__global__ __launch_bounds__(FT) void k_fused_batch(const uint8_t *plans, const FBatchItem *items, uint32_t nitems,
                                                   const uint32_t *M0all, uint32_t *scratch, uint64_t slot_words,
                                                   uint32_t kmax, uint32_t *outall, FStatus *sts,
                                                   uint32_t *counter) {
    __shared__ FusedLds<FT, CR, CS> L;
    __shared__ uint32_t s_q;
    uint32_t *slot = scratch + (uint64_t)blockIdx.x * slot_words;
    uint32_t *buf0 = slot, *buf1 = slot + (uint64_t)CR * kmax, *loc = slot + 2ull * CR * kmax;
    for (;;) {
        if (threadIdx.x == 0) s_q = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t qi = s_q;
        __syncthreads();
        if (qi >= nitems) break;
        const FBatchItem it = items[qi];
        fused_query<FT, CR, CS>(reinterpret_cast<const FPlan *>(plans + it.plan_off), M0all + it.m0_off, it.R0,
                                buf0, buf1, loc, outall ? outall + it.out_off : nullptr, sts + qi, L);
        __syncthreads();
    }
}

template <uint32_t FT>
static void launch_batch_t(gsi_ctx *c, uint32_t grid, const uint8_t *plans, const FBatchItem *items,
                           uint32_t nitems, const uint32_t *M0all, uint32_t *scratch, uint64_t slot_words,
                           uint32_t kmax, uint32_t *outall, FStatus *sts, uint32_t *counter, double bytes) {
    constexpr uint32_t CR = 4 * FT, CS = 16 * FT;
    launch(c, FT == 64 ? "k_fused_batch<64>" : FT == 256 ? "k_fused_batch<256>" : "k_fused_batch<1024>", bytes,
           k_fused_batch<FT, CR, CS>, grid, FT, plans, items, nitems, M0all, scratch, slot_words, kmax, outall, sts,
           counter);
}

FTier fused_tier(uint32_t threads) {
    FTier t;
    t.threads = threads;
    t.cap_rows = 4 * threads;
    t.cap_slots = 16 * threads;
    int per_cu = 0;
    hipError_t e = hipSuccess;
    if (threads == 64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused_batch<64, 256, 1024>, 64, 0);
    else if (threads == 256)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused_batch<256, 1024, 4096>, 256, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused_batch<1024, 4096, 16384>, 1024, 0);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    t.blocks_per_cu = (uint32_t)per_cu;
    return t;
}

void launch_fused_batch(gsi_ctx *c, const FTier &t, uint32_t grid, const uint8_t *plans, const FBatchItem *items,
                        uint32_t nitems, const uint32_t *M0all, uint32_t *scratch, uint64_t slot_words, uint32_t kmax,
                        uint32_t *outall, FStatus *sts, uint32_t *counter, double bytes) {
    if (t.threads == 64)
        launch_batch_t<64>(c, grid, plans, items, nitems, M0all, scratch, slot_words, kmax, outall, sts, counter, bytes);
    else if (t.threads == 256)
        launch_batch_t<256>(c, grid, plans, items, nitems, M0all, scratch, slot_words, kmax, outall, sts, counter,
                            bytes);
    else
        launch_batch_t<1024>(c, grid, plans, items, nitems, M0all, scratch, slot_words, kmax, outall, sts, counter,
                             bytes);
}

}  // namespace gsi
