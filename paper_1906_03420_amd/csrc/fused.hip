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

// LDS of one fused workgroup with FT threads, CR rows and CS slots: F, the
// start of each row's scanned list, the keep bits and their prefix sums,
// and (XS) each slot's element x, so that the link re-reads no list
template <uint32_t FT, uint32_t CR, uint32_t CS, bool XS>
struct FusedLds {
    uint32_t F[CR + 1];
    uint32_t st[CR];
    uint64_t bits[CS / 64];
    uint32_t wpre[CS / 64];
    uint32_t w[FT / 64];
    uint64_t d[2][FT / 64];
    uint64_t obase;
    uint32_t x[XS ? CS : 1];
};

// All join levels of one query in one workgroup (see the file comment).
// FT threads; at most CR rows per table (CR = 4 FT) and CS slots per level.
// With `ocount` set, the last level reserves its S*k output words from that
// counter (words of `out`, at most `ocap`) instead of writing at out[0].
template <uint32_t FT, uint32_t CR, uint32_t CS, bool XS>
__device__ void fused_query(const FPlan *plan, const uint32_t *M0, uint32_t R0, uint32_t *buf0, uint32_t *buf1,
                            uint32_t *loc, uint32_t *out, FStatus *st, FusedLds<FT, CR, CS, XS> &L,
                            unsigned long long *ocount = nullptr, uint64_t ocap = 0) {
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
    if (R0 > cap_rows) {  // the first table does not fit
        if (tid == 0) {
            st->level = 1;
            st->rows = R0;
            st->mloc = mloc;
        }
        return;
    }

    for (uint32_t j = 1; j < k; j++) {
        const uint32_t ne = plan->lv_ne[j], ef = plan->lv_first[j], e0 = plan->lv_e0[j];
        const uint64_t *Cu = plan->Cu[j];
        const bool final_level = (j == k - 1);
        const uint32_t *ci_all = plan->ci_all;
        if (tid == 0) st->lv_rows[j] = R;

        // locate N(v, l) for every row and linking edge; the row scans the
        // list of e0 (Algorithm 4) or, with `pick`, its shortest one
        for (uint32_t i = tid; i < R; i += FT) {
            uint32_t s0 = 0, l0 = 0, ob = NONE32, os = 0, ol = 0xFFFFFFFFu;
            for (uint32_t e = 0; e < ne; e++) {
                const FEdge &ed = plan->edges[ef + e];
                const uint32_t v = M[(uint64_t)ed.col * R + i];
                const uint2 r = pcsr_find(ed.gl, ed.G, ed.H, v);
                loc[(uint64_t)e * R + i] = r.x;
                loc[(uint64_t)(ne + e) * R + i] = r.y;
                if (e == e0) {
                    s0 = r.x;
                    l0 = r.y;
                } else if (r.y < ol) {
                    ob = e;
                    os = r.x;
                    ol = r.y;
                }
            }
            uint32_t be = e0, bs = s0, bl = l0;
            if (plan->pick && ob != NONE32 && ol < l0) {
                be = ob;
                bs = os;
                bl = ol;
            }
            s_F[i] = bl;
            L.st[i] = plan->edges[ef + be].ci_off + bs;
            if (ne > 1) loc[(uint64_t)(2 * ne + 1) * R + i] = be;
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
        // values every thread reads from LDS are made wave-uniform, so that
        // the exits below are uniform branches
        const uint32_t gba = __builtin_amdgcn_readfirstlane(s_F[R]);
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
                const uint32_t x = ci_all[L.st[i] + (p - s_F[i])];
                if (XS) L.x[p] = x;
                keep = (Cu[x >> 6] >> (x & 63)) & 1ull;
                for (uint32_t c = 0; keep && !plan->homo && c < j; c++) keep = M[(uint64_t)c * R + i] != x;
                const uint32_t be = (keep && ne > 1) ? loc[(uint64_t)(2 * ne + 1) * R + i] : e0;
                for (uint32_t e = 0; keep && e < ne; e++) {
                    if (e == be) continue;
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
            S = __builtin_amdgcn_readfirstlane(S);
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

        // a chunk reserves its output rows
        if (final_level && ocount && !plan->count_only) {
            if (tid == 0) {
                const unsigned long long need = (unsigned long long)S * k;
                const unsigned long long b = atomicAdd(ocount, need);
                L.obase = (b + need <= ocap) ? (uint64_t)b : ~0ull;
            }
            __syncthreads();
            const uint64_t lb = L.obase;
            const uint64_t b = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(lb >> 32)) << 32) |
                               __builtin_amdgcn_readfirstlane((uint32_t)lb);
            if (b == ~0ull) {
                if (tid == 0) {
                    st->level = j;
                    st->rows = R;
                    st->mloc = mloc;
                }
                return;
            }
            out += b;
            if (tid == 0) st->out_base = b;
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
            const uint32_t x = XS ? L.x[p] : ci_all[L.st[i] + (p - s_F[i])];
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

// One query in one workgroup.  The status is cleared here (no separate
// fill), and, when `b0` is given, the first table M0 = C(u_first) is
// written here too from its bitset (ascending vertex order, R0 entries):
// each thread counts the set bits of a run of bitset words, an exclusive
// scan over the workgroup places the runs, and each thread writes its ids.
__global__ __launch_bounds__(1024) void k_fused_levels(const FPlan *plan, uint32_t *M0, uint32_t R0,
                                                      const uint64_t *b0, uint64_t nwords, uint32_t *buf0,
                                                      uint32_t *buf1, uint32_t *loc, uint32_t *out, FStatus *st) {
    __shared__ FusedLds<1024, FUSED_MAX_ROWS, FUSED_MAX_SLOTS, true> L;
    uint64_t *sw = reinterpret_cast<uint64_t *>(st);
    for (uint32_t t = threadIdx.x; t < sizeof(FStatus) / 8; t += 1024) sw[t] = 0;
    if (b0) {
        // each wave owns a contiguous run of words, read 64 at a time
        // (coalesced): count, place the runs, then emit with wave scans
        const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
        const uint64_t per = (nwords + 15) / 16;
        const uint64_t ws = per * wv < nwords ? per * wv : nwords;
        const uint64_t we = ws + per < nwords ? ws + per : nwords;
        uint32_t cnt = 0;
        for (uint64_t q = ws + lane; q < we; q += 64) cnt += (uint32_t)__popcll(b0[q]);
        cnt = wave_sum(cnt);
        if (lane == 0) L.w[wv] = cnt;
        __syncthreads();
        uint32_t at = 0;
        for (uint32_t v = 0; v < wv; v++) at += L.w[v];
        for (uint64_t base = ws; base < we; base += 64) {
            const uint64_t q = base + lane;
            uint64_t m = q < we ? b0[q] : 0ull;
            const uint32_t pc = (uint32_t)__popcll(m);
            const uint32_t inc = wave_inclusive_sum(pc);
            uint32_t o = at + inc - pc;
            while (m) {
                const uint32_t b = (uint32_t)__builtin_ctzll(m);
                if (o < R0) M0[o] = (uint32_t)(q * 64 + b);
                o++;
                m &= m - 1;
            }
            at += __shfl(inc, 63, 64);
        }
    }
    __syncthreads();  // status cleared and M0 written before the levels read them
    fused_query<1024, FUSED_MAX_ROWS, FUSED_MAX_SLOTS, true>(plan, M0, R0, buf0, buf1, loc, out, st, L);
}

void launch_fused(gsi_ctx *c, const FPlan *d_plan, uint32_t *M0, uint32_t R0, const uint64_t *b0, uint64_t nwords,
                  uint32_t *buf0, uint32_t *buf1, uint32_t *loc, uint32_t *out, FStatus *d_status, double alg_bytes) {
    launch(c, "k_fused_levels", alg_bytes, k_fused_levels, 1, 1024, d_plan, M0, R0, b0, nwords, buf0, buf1, loc, out,
           d_status);
}

// Persistent batch: each workgroup takes the next query from a shared
// counter until none is left (every workgroup leaves once the counter passes
// the item count), and runs all its levels in its own scratch slot.
template <uint32_t FT, uint32_t CR, uint32_t CS>
__global__ __launch_bounds__(FT) void k_fused_batch(const uint8_t *plans, const FBatchItem *items, uint32_t nitems,
                                                   const uint32_t *M0all, uint32_t *scratch, uint64_t slot_words,
                                                   uint32_t kmax, uint32_t *outall, FStatus *sts,
                                                   uint32_t *counter) {
    __shared__ FusedLds<FT, CR, CS, false> L;
    __shared__ uint32_t s_q;
    uint32_t *slot = scratch + (uint64_t)blockIdx.x * slot_words;
    uint32_t *buf0 = slot, *buf1 = slot + (uint64_t)CR * kmax, *loc = slot + 2ull * CR * kmax;
    for (;;) {
        if (threadIdx.x == 0) s_q = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t qi = __builtin_amdgcn_readfirstlane(s_q);
        __syncthreads();
        if (qi >= nitems) break;
        const FBatchItem it = items[qi];
        fused_query<FT, CR, CS, false>(reinterpret_cast<const FPlan *>(plans + it.plan_off), M0all + it.m0_off, it.R0,
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

// Chunks of one query (see launch_fused_chunks).  Every workgroup leaves
// once the chunk counter passes nchunks or the abort flag is set.
template <uint32_t FT, uint32_t CR, uint32_t CS>
__global__ __launch_bounds__(FT) void k_fused_chunks(const FPlan *plan, const uint32_t *M0, uint32_t R0,
                                                    uint32_t chunk_rows, uint32_t nchunks, uint32_t *scratch,
                                                    uint64_t slot_words, uint32_t k, uint32_t *staging,
                                                    uint64_t staging_words, unsigned long long *ocount,
                                                    uint32_t *abort, uint32_t max_fail, FStatus *sts,
                                                    uint32_t *counter) {
    __shared__ FusedLds<FT, CR, CS, true> L;
    __shared__ uint32_t s_q;
    uint32_t *slot = scratch + (uint64_t)blockIdx.x * slot_words;
    uint32_t *buf0 = slot, *buf1 = slot + (uint64_t)CR * k, *loc = slot + 2ull * CR * k;
    // The only thread-0 block of the loop is at its head, and the chunk index
    // is made wave-uniform: the loop then stays one uniform loop around the
    // barriers (a thread-0 block after the last barrier let the compiler
    // split it so that the other lanes of wave 0 spun without thread 0).
    uint32_t prev = 0xFFFFFFFFu;  // chunk run last (read by thread 0 only)
    for (;;) {
        if (threadIdx.x == 0) {
            // too many chunks that do not fit: leave the rest to the caller
            if (prev != 0xFFFFFFFFu && !sts[prev].done && atomicAdd(abort + 1, 1u) + 1 > max_fail)
                atomicOr(abort, 1u);
            s_q = __atomic_load_n(abort, __ATOMIC_RELAXED) ? nchunks : atomicAdd(counter, 1u);
        }
        __syncthreads();
        const uint32_t qi = __builtin_amdgcn_readfirstlane(s_q);
        __syncthreads();
        if (qi >= nchunks) break;
        const uint32_t first = qi * chunk_rows;
        const uint32_t rows = min(chunk_rows, R0 - first);
        fused_query<FT, CR, CS, true>(plan, M0 + first, rows, buf0, buf1, loc, staging, sts + qi, L, ocount,
                                      staging_words);
        prev = qi;
        __syncthreads();
    }
}

// Totals of a chunked run and each chunk's first output row (exclusive
// prefix of the counts, chunk order).  One 1024-thread workgroup.
__global__ __launch_bounds__(1024) void k_chunk_summary(const FStatus *sts, uint32_t n, uint32_t nlevels,
                                                       uint64_t *offs, uint32_t *done, FChunkSummary *sum) {
    __shared__ uint64_t s_w[16];
    __shared__ uint64_t s_d[3][16];
    __shared__ uint32_t s_nd[16], s_lv[16];
    const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
    uint64_t carry = 0, ds = 0, dx = 0;
    uint32_t notdone = 0, lv = 0;
    for (uint32_t base = 0; base < n; base += 1024) {
        const uint32_t i = base + tid;
        uint64_t c = 0;
        if (i < n) {
            const FStatus &st = sts[i];
            c = st.done ? st.count : 0ull;
            done[i] = st.done ? 1u : 0u;
            notdone += st.done ? 0u : 1u;
            if (st.done) {
                ds += st.digest[0];
                dx ^= st.digest[1];
                lv = max(lv, (uint32_t)st.levels);
            }
        }
        const uint64_t inc = wave_inclusive_sum(c);
        if (lane == 63) s_w[w] = inc;
        __syncthreads();
        uint64_t off = carry, tot = 0;
        for (uint32_t q = 0; q < 16; q++) {
            off += q < w ? s_w[q] : 0ull;
            tot += s_w[q];
        }
        if (i < n) offs[i] = off + inc - c;
        carry += tot;
        __syncthreads();
    }
    ds = wave_sum(ds);
    dx = wave_xor(dx);
    notdone = wave_sum(notdone);
    for (uint32_t o = 32; o; o >>= 1) lv = max(lv, (uint32_t)__shfl_xor((int)lv, (int)o));
    if (lane == 0) {
        s_d[0][w] = ds;
        s_d[1][w] = dx;
        s_nd[w] = notdone;
        s_lv[w] = lv;
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t a = 0, b = 0;
        uint32_t nd = 0, l = 0;
        for (uint32_t q = 0; q < 16; q++) {
            a += s_d[0][q];
            b ^= s_d[1][q];
            nd += s_nd[q];
            l = max(l, s_lv[q]);
        }
        offs[n] = carry;
        sum->all_done = nd == 0 ? 1u : 0u;
        sum->count = carry;
        sum->digest[0] = a;
        sum->digest[1] = b;
        sum->levels = l;
    }
    // per-level sums: wave w takes levels w, w + 16
    for (uint32_t j = w; j < nlevels; j += 16) {
        uint64_t r = 0, gb = 0, sv = 0;
        for (uint32_t i = lane; i < n; i += 64) {
            const bool d = sts[i].done != 0;
            r += d ? sts[i].lv_rows[j] : 0ull;
            gb += d ? sts[i].lv_gba[j] : 0ull;
            sv += d ? sts[i].lv_surv[j] : 0ull;
        }
        r = wave_sum(r);
        gb = wave_sum(gb);
        sv = wave_sum(sv);
        if (lane == 0) {
            sum->lv_rows[j] = r;
            sum->lv_gba[j] = gb;
            sum->lv_surv[j] = sv;
        }
    }
}

// Rows of every finished chunk into `out`, in chunk order.  One workgroup
// per chunk.
__global__ __launch_bounds__(256) void k_chunk_gather(const FStatus *sts, const uint64_t *offs,
                                                     const uint32_t *staging, uint32_t k, uint32_t *out) {
    const FStatus &st = sts[blockIdx.x];
    if (!st.done) return;
    const uint64_t words = st.count * k;
    if (words == 0) return;
    const uint32_t *src = staging + st.out_base;
    uint32_t *dst = out + offs[blockIdx.x] * k;
    for (uint64_t t = threadIdx.x; t < words; t += 256) dst[t] = src[t];
}

template <uint32_t FT>
static void launch_chunks_t(gsi_ctx *c, uint32_t grid, const FPlan *plan, const uint32_t *M0, uint32_t R0,
                            uint32_t chunk_rows, uint32_t nchunks, uint32_t *scratch, uint64_t slot_words, uint32_t k,
                            uint32_t *staging, uint64_t staging_words, unsigned long long *ocount, uint32_t *abort,
                            uint32_t max_fail, FStatus *sts, uint32_t *counter, double bytes) {
    constexpr uint32_t CR = 4 * FT, CS = 16 * FT;
    launch(c, "k_fused_chunks", bytes, k_fused_chunks<FT, CR, CS>, grid, FT, plan, M0, R0, chunk_rows, nchunks,
           scratch, slot_words, k, staging, staging_words, ocount, abort, max_fail, sts, counter);
}

void launch_fused_chunks(gsi_ctx *c, const FTier &t, uint32_t grid, const FPlan *plan, const uint32_t *M0,
                         uint32_t R0, uint32_t chunk_rows, uint32_t nchunks, uint32_t *scratch, uint64_t slot_words,
                         uint32_t k, uint32_t *staging, uint64_t staging_words, unsigned long long *ocount,
                         uint32_t *abort, uint32_t max_fail, FStatus *sts, uint32_t *counter, uint64_t *offs,
                         uint32_t *done, FChunkSummary *sum) {
    if (t.threads == 64)
        launch_chunks_t<64>(c, grid, plan, M0, R0, chunk_rows, nchunks, scratch, slot_words, k, staging,
                            staging_words, ocount, abort, max_fail, sts, counter, 0.0);
    else if (t.threads == 256)
        launch_chunks_t<256>(c, grid, plan, M0, R0, chunk_rows, nchunks, scratch, slot_words, k, staging,
                             staging_words, ocount, abort, max_fail, sts, counter, 0.0);
    else
        launch_chunks_t<1024>(c, grid, plan, M0, R0, chunk_rows, nchunks, scratch, slot_words, k, staging,
                              staging_words, ocount, abort, max_fail, sts, counter, 0.0);
    launch(c, "k_chunk_summary", (double)nchunks * sizeof(FStatus), k_chunk_summary, 1, 1024, (const FStatus *)sts,
           nchunks, k, offs, done, sum);
}

void launch_chunk_gather(gsi_ctx *c, uint32_t nchunks, const FStatus *sts, const uint64_t *offs,
                         const uint32_t *staging, uint32_t k, uint32_t *out, uint64_t words) {
    launch(c, "k_chunk_gather", 8.0 * words, k_chunk_gather, nchunks, 256, sts, offs, staging, k, out);
}

// Root rows of the given chunks, concatenated: workgroup i copies chunk
// list[2i] to position list[2i+1].
__global__ __launch_bounds__(256) void k_take_roots(const uint32_t *M0, uint32_t R0, uint32_t chunk_rows,
                                                   const uint32_t *list, uint32_t *dst) {
    const uint32_t ch = list[2 * blockIdx.x], at = list[2 * blockIdx.x + 1];
    const uint32_t first = ch * chunk_rows;
    const uint32_t rows = min(chunk_rows, R0 - first);
    for (uint32_t t = threadIdx.x; t < rows; t += 256) dst[at + t] = M0[first + t];
}

void launch_take_roots(gsi_ctx *c, uint32_t nlist, const uint32_t *M0, uint32_t R0, uint32_t chunk_rows,
                       const uint32_t *list, uint32_t *dst, uint64_t rows) {
    launch(c, "k_take_roots", 8.0 * rows, k_take_roots, nlist, 256, M0, R0, chunk_rows, list, dst);
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
