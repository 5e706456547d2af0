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

// Rows of U slots at once: for each r, the largest i < R with F[i] <= p[r]
// (F in LDS, non-decreasing, F[0] = 0), with Fi[r] = F[i].  A branch-free
// binary lifting with the same number of steps for every lane, so the U
// searches interleave their LDS reads.  F[R] (|GBA|) is read in place of
// indices past the table; it exceeds every slot below |GBA|.
template <uint32_t U>
__device__ __forceinline__ void lds_rows(const uint32_t *F, uint32_t R, const uint32_t *p, uint32_t *row,
                                         uint32_t *Fi) {
#pragma unroll
    for (uint32_t r = 0; r < U; r++) {
        row[r] = 0;
        Fi[r] = 0;
    }
    for (uint32_t b = R > 1 ? 1u << (31 - __builtin_clz(R - 1)) : 0u; b; b >>= 1) {
#pragma unroll
        for (uint32_t r = 0; r < U; r++) {
            const uint32_t m = row[r] + b;
            const uint32_t f = F[m < R ? m : R];
            if (m < R && f <= p[r]) {
                row[r] = m;
                Fi[r] = f;
            }
        }
    }
}

// Position of the r-th set bit (r from 0) of m, which has more than r set bits.
__device__ __forceinline__ uint32_t nth_set_bit(uint64_t m, uint32_t r) {
    uint32_t pos = 0;
#pragma unroll
    for (uint32_t sh = 32; sh; sh >>= 1) {
        const uint32_t c = (uint32_t)__popcll(m & ((1ull << sh) - 1));
        if (r >= c) {
            r -= c;
            m >>= sh;
            pos += sh;
        }
    }
    return pos;
}

// For U survivors q[r] < S: the bitmap word holding each (the largest w <
// nw with pre[w] <= q, pre being the exclusive prefix of the words' set
// bits, in LDS) and the survivor's rank within it.  Branch-free, as lds_rows.
template <uint32_t U>
__device__ __forceinline__ void lds_words(const uint32_t *pre, uint32_t nw, const uint32_t *q, uint32_t *wd,
                                          uint32_t *rk) {
#pragma unroll
    for (uint32_t r = 0; r < U; r++) {
        wd[r] = 0;
        rk[r] = q[r];
    }
    for (uint32_t b = nw > 1 ? 1u << (31 - __builtin_clz(nw - 1)) : 0u; b; b >>= 1) {
#pragma unroll
        for (uint32_t r = 0; r < U; r++) {
            const uint32_t m = wd[r] + b;
            const uint32_t f = pre[m < nw ? m : nw - 1];
            if (m < nw && f <= q[r]) {
                wd[r] = m;
                rk[r] = q[r] - f;
            }
        }
    }
}

// bitmap words a wave takes per round of the fused join and link
constexpr uint32_t FU = 2;

// Words of each of the two LDS buffers that hold intermediate tables small
// enough (rows x columns), sized to what the workgroup's LDS has left.
template <uint32_t FT, bool XS>
constexpr uint32_t fused_table_words() {
    return FT == 1024 ? (XS ? 7168u : 14336u) : FT == 256 ? 1536u : 384u;
}

// LDS of one fused workgroup with FT threads, CR rows and CS slots: F, the
// start of each row's scanned list, the keep bits and their prefix sums,
// (XS) each slot's element x, so that the link re-reads no list, and two
// table buffers
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
    uint32_t mt[2][fused_table_words<FT, XS>()];
};
static_assert(sizeof(FusedLds<1024, 4096, 16384, true>) <= 160 * 1024, "fused workgroup LDS");

// Join levels j0 .. k-1 of one query in one workgroup (see the file
// comment), starting from the table M0 of R0 rows and j0 columns (column c
// at M0 + c * ld0).  FT threads; at most CR rows per table (CR = 4 FT) and
// CS slots per level.  With `ocount` set, the last level reserves its S*k
// output words from that counter (words of `out`, at most `ocap`) instead of
// writing at out[0].
template <uint32_t FT, uint32_t CR, uint32_t CS, bool XS>
__device__ __forceinline__ void fused_query(const FPlan *plan, uint32_t j0, const uint32_t *M0, uint32_t R0,
                                            uint32_t ld0, uint32_t *buf0, uint32_t *buf1, uint32_t *loc,
                                            uint32_t *out, FStatus *st, FusedLds<FT, CR, CS, XS> &L,
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
    uint32_t ld = ld0;  // column stride of M
    uint32_t mloc = FSTATUS_IN_FIRST;  // where M lives
    // A table of at most MT words is written to (and read from) LDS instead
    // of global memory; M then has column stride R.  M sits at index
    // next ^ 1 of its space (global or LDS), M' goes to index `next`.
    constexpr uint32_t MT = fused_table_words<FT, XS>();
    bool m_lds = false;
    uint32_t next = 0;
    // level j does not fit: record where, and where its input M lives (a
    // table in LDS is copied to buf0 for the caller)
    auto stop = [&](uint32_t j) {
        if (m_lds) {
            for (uint32_t t = tid; t < R * j; t += FT) buf0[t] = M[t];
            mloc = 0;
        }
        if (tid == 0) {
            st->level = j;
            st->rows = R;
            st->mloc = mloc;
        }
    };
    if (R0 > cap_rows) {  // the first table does not fit
        stop(j0);
        return;
    }

    for (uint32_t j = j0; j < k; j++) {
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
                const uint32_t v = M[(uint64_t)ed.col * ld + i];
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
            stop(j);
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
        // x in every other linking list; one ballot word per 64 slots.  A
        // wave takes FU words per round (words base + r * waves + w) and
        // issues each step's loads for all of them together, so a round
        // costs one chain of dependent loads, not FU.
        for (uint32_t base = 0; base < nw; base += FU * (FT / 64)) {
            uint32_t pr[FU], ir[FU], fr[FU], xr[FU];
            bool kp[FU];
#pragma unroll
            for (uint32_t r = 0; r < FU; r++) {
                pr[r] = (base + r * (FT / 64) + w) * 64 + lane;
                kp[r] = pr[r] < gba;
                xr[r] = 0;
            }
            lds_rows<FU>(s_F, R, pr, ir, fr);
            // Loads are issued unconditionally, a slot past |GBA| reading
            // valid addresses (element 0, row 0, column j - 1), and masked
            // afterwards: a load behind a branch waits for the one before.
#pragma unroll
            for (uint32_t r = 0; r < FU; r++) {
                if (!kp[r]) ir[r] = 0;
                xr[r] = ci_all[kp[r] ? L.st[ir[r]] + (pr[r] - fr[r]) : 0u];
                if (!kp[r]) xr[r] = 0;
            }
            {
                uint64_t cw[FU];
#pragma unroll
                for (uint32_t r = 0; r < FU; r++) cw[r] = Cu[xr[r] >> 6];
#pragma unroll
                for (uint32_t r = 0; r < FU; r++) {
                    if (XS && kp[r]) L.x[pr[r]] = xr[r];
                    kp[r] = kp[r] && ((cw[r] >> (xr[r] & 63)) & 1ull);
                }
            }
            if (!plan->homo) {
                // x not among the row's values in the columns that can hold
                // it (those of u's label), four columns at a time; past the
                // last one the last is read again
                uint32_t mm = plan->lv_mmask[j];
                const uint32_t last = mm ? 31u - (uint32_t)__builtin_clz(mm) : 0u;
                while (mm) {
                    uint32_t cq[4];
#pragma unroll
                    for (uint32_t q = 0; q < 4; q++) {
                        cq[q] = mm ? (uint32_t)__builtin_ctz(mm) : last;
                        mm &= mm - 1;
                    }
                    uint32_t mv[FU][4];
#pragma unroll
                    for (uint32_t r = 0; r < FU; r++)
#pragma unroll
                        for (uint32_t q = 0; q < 4; q++) mv[r][q] = M[(uint64_t)cq[q] * ld + ir[r]];
#pragma unroll
                    for (uint32_t r = 0; r < FU; r++)
#pragma unroll
                        for (uint32_t q = 0; q < 4; q++) kp[r] = kp[r] && mv[r][q] != xr[r];
                }
            }
            if (ne > 1) {
#pragma unroll
                for (uint32_t r = 0; r < FU; r++) {
                    bool keep = kp[r];
                    const uint32_t i = ir[r];
                    const uint32_t be = keep ? loc[(uint64_t)(2 * ne + 1) * R + i] : e0;
                    for (uint32_t e = 0; keep && e < ne; e++) {
                        if (e == be) continue;
                        keep = in_sorted(plan->edges[ef + e].ci + loc[(uint64_t)e * R + i],
                                         loc[(uint64_t)(ne + e) * R + i], xr[r]);
                    }
                    kp[r] = keep;
                }
            }
#pragma unroll
            for (uint32_t r = 0; r < FU; r++) {
                const uint64_t mask = __ballot(kp[r]);
                const uint32_t word = base + r * (FT / 64) + w;
                if (lane == 0 && word < nw) s_bits[word] = mask;
            }
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
            stop(j);
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
                stop(j);
                return;
            }
            out += b;
            if (tid == 0) st->out_base = b;
        }

        // link: (m_i, x) at its position; the last level writes rows in
        // query-vertex order and hashes them.  Threads take survivors, not
        // slots (survivor q is at position q; its slot is found from the
        // keep bits' prefix sums), so the waves are dense however sparse the
        // keep bits are; FU survivors per thread and round.
        const bool n_lds = !final_level && (uint64_t)S * (j + 1) <= MT;
        // (selects, not an indexed pointer array, which would live in scratch)
        uint32_t *Mn = n_lds ? (next ? L.mt[1] : L.mt[0]) : (next ? buf1 : buf0);
        uint64_t hs = 0, hx = 0;
        for (uint32_t base = 0; base < S; base += FU * FT) {
            uint32_t pr[FU], ir[FU], fr[FU], pos[FU], xr[FU], wd[FU], rk[FU];
            bool kp[FU];
#pragma unroll
            for (uint32_t r = 0; r < FU; r++) {
                pos[r] = base + r * FT + tid;
                kp[r] = pos[r] < S;
            }
            lds_words<FU>(s_wpre, nw, pos, wd, rk);
#pragma unroll
            for (uint32_t r = 0; r < FU; r++) pr[r] = kp[r] ? wd[r] * 64 + nth_set_bit(s_bits[wd[r]], rk[r]) : 0u;
            lds_rows<FU>(s_F, R, pr, ir, fr);
            // unconditional loads from valid addresses, masked afterwards
#pragma unroll
            for (uint32_t r = 0; r < FU; r++) {
                if (!kp[r]) ir[r] = 0;
                if (XS) xr[r] = L.x[kp[r] ? pr[r] : 0u];
                else xr[r] = ci_all[kp[r] ? L.st[ir[r]] + (pr[r] - fr[r]) : 0u];
                if (!kp[r]) xr[r] = 0;
            }
            if (!final_level) {
                for (uint32_t c = 0; c < j; c += 4) {
                    uint32_t mv[FU][4];
#pragma unroll
                    for (uint32_t r = 0; r < FU; r++)
#pragma unroll
                        for (uint32_t q = 0; q < 4; q++)
                            mv[r][q] = M[(uint64_t)(c + q < j ? c + q : j - 1) * ld + ir[r]];
#pragma unroll
                    for (uint32_t r = 0; r < FU; r++)
#pragma unroll
                        for (uint32_t q = 0; q < 4; q++)
                            if (kp[r] && c + q < j) Mn[(uint64_t)(c + q) * S + pos[r]] = mv[r][q];
                }
#pragma unroll
                for (uint32_t r = 0; r < FU; r++)
                    if (kp[r]) Mn[(uint64_t)j * S + pos[r]] = xr[r];
            } else {
                uint64_t f[FU];
#pragma unroll
                for (uint32_t r = 0; r < FU; r++) f[r] = 14695981039346656037ull;
                for (uint32_t u0 = 0; u0 < k; u0 += 4) {
                    uint32_t val[FU][4];
#pragma unroll
                    for (uint32_t q = 0; q < 4; q++) {
                        const uint32_t c = u0 + q < k ? plan->qcol[u0 + q] : j;
#pragma unroll
                        for (uint32_t r = 0; r < FU; r++) {
                            const uint32_t mv = M[(uint64_t)(c < j ? c : 0u) * ld + ir[r]];
                            val[r][q] = c < j ? mv : xr[r];
                        }
                    }
#pragma unroll
                    for (uint32_t q = 0; q < 4; q++)
#pragma unroll
                        for (uint32_t r = 0; r < FU; r++) {
                            if (!kp[r] || u0 + q >= k) continue;
                            if (!plan->count_only) out[(uint64_t)pos[r] * k + u0 + q] = val[r][q];
                            f[r] = fnv_word(f[r], val[r][q]);
                        }
                }
#pragma unroll
                for (uint32_t r = 0; r < FU; r++) {
                    if (!kp[r]) continue;
                    const uint64_t h = mix64(f[r]);
                    hs += h;
                    hx ^= h;
                }
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
        ld = S;
        m_lds = n_lds;
        if (!n_lds) mloc = next;
        next ^= 1u;
    }
}

// One query in one workgroup.  The status is cleared here (no separate
// fill), and, when `b0` is given, the first table M0 = C(u_first) is
// written here too from its bitset (ascending vertex order, R0 entries):
// each thread counts the set bits of a run of bitset words, an exclusive
// scan over the workgroup places the runs, and each thread writes its ids.
// INL: the plan is the kernel argument `inl` (read with scalar loads from
// the argument segment), else d_plan in device memory.  Two instances, not a
// select: a pointer that may address either space is generic, and every
// plan field would be read with vector loads.
template <bool INL>
__global__ __launch_bounds__(1024) void k_fused_levels(const FPlan *d_plan, FPlanArg inl, uint32_t j0, uint32_t *M0,
                                                      uint32_t R0, const uint32_t *b0_runs,
                                                      const uint64_t *b0, uint64_t nwords, uint32_t *buf0,
                                                      uint32_t *buf1, uint32_t *loc, uint32_t *out, FStatus *st) {
    __shared__ FusedLds<1024, FUSED_MAX_ROWS, FUSED_MAX_SLOTS, true> L;
    const FPlan *plan = INL ? &inl.p : d_plan;
    uint64_t *sw = reinterpret_cast<uint64_t *>(st);
    for (uint32_t t = threadIdx.x; t < sizeof(FStatus) / 8; t += 1024) sw[t] = 0;
    if (b0) {
        // each wave owns a contiguous run of words (the split the filter's
        // counts used, whose per-run set bits `b0_runs` give the wave its
        // first output row), read 64 at a time (coalesced) with eight such
        // reads in flight, and emits with wave scans
        const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
        const uint64_t per = (nwords + BITS_RUNS - 1) / BITS_RUNS;
        const uint64_t ws = per * wv < nwords ? per * wv : nwords;
        const uint64_t we = ws + per < nwords ? ws + per : nwords;
        uint32_t at = wave_sum(lane < wv ? b0_runs[lane] : 0u);
        for (uint64_t base = ws; base < we; base += 512) {
            uint64_t m[8];
#pragma unroll
            for (uint32_t t = 0; t < 8; t++) {
                const uint64_t qq = base + 64 * t + lane;
                m[t] = qq < we ? b0[qq] : 0ull;
            }
#pragma unroll
            for (uint32_t t = 0; t < 8; t++) {
                const uint32_t pc = (uint32_t)__popcll(m[t]);
                const uint32_t inc = wave_inclusive_sum(pc);
                uint32_t o = at + inc - pc;
                uint64_t mm = m[t];
                const uint64_t qq = base + 64 * t + lane;
                while (mm) {
                    const uint32_t b = (uint32_t)__builtin_ctzll(mm);
                    if (o < R0) M0[o] = (uint32_t)(qq * 64 + b);
                    o++;
                    mm &= mm - 1;
                }
                at += __shfl(inc, 63, 64);
            }
        }
    }
    __syncthreads();  // status cleared and M0 written before the levels read them
    fused_query<1024, FUSED_MAX_ROWS, FUSED_MAX_SLOTS, true>(plan, j0, M0, R0, R0, buf0, buf1, loc, out, st, L);
}

void launch_fused(gsi_ctx *c, const FPlan *d_plan, const FPlanArg &inl, uint32_t j0, uint32_t *M0, uint32_t R0,
                  const uint32_t *b0_runs, const uint64_t *b0, uint64_t nwords, uint32_t *buf0, uint32_t *buf1, uint32_t *loc, uint32_t *out,
                  FStatus *d_status, double alg_bytes) {
    if (d_plan)
        launch(c, "k_fused_levels", alg_bytes, k_fused_levels<false>, 1, 1024, d_plan, inl, j0, M0, R0, b0_runs, b0,
               nwords, buf0, buf1, loc, out, d_status);
    else
        launch(c, "k_fused_levels", alg_bytes, k_fused_levels<true>, 1, 1024, d_plan, inl, j0, M0, R0, b0_runs, b0,
               nwords, buf0, buf1, loc, out, d_status);
}

// Persistent batch: each workgroup takes the next query from a shared
// counter until none is left (every workgroup leaves once the counter passes
// the item count), and runs all its levels in its own scratch slot.
template <uint32_t FT, uint32_t CR, uint32_t CS>
// (the 256-thread tier is held to four waves per SIMD: left alone the
// compiler takes a few more registers and one workgroup per CU fewer fits)
__global__ __launch_bounds__(FT, FT == 256 ? 4 : 1) void k_fused_batch(const uint8_t *plans, const FBatchItem *items, uint32_t nitems,
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
        fused_query<FT, CR, CS, false>(reinterpret_cast<const FPlan *>(plans + it.plan_off), 1, M0all + it.m0_off,
                                       it.R0, it.R0, buf0, buf1, loc, outall ? outall + it.out_off : nullptr,
                                       sts + qi, L);
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
__global__ __launch_bounds__(FT) void k_fused_chunks(const FPlan *plan, uint32_t j0, const uint32_t *M0, uint32_t R0,
                                                    uint32_t chunk_rows, uint32_t nchunks, uint32_t *scratch,
                                                    uint64_t slot_words, uint32_t k, uint32_t *staging,
                                                    uint64_t staging_words, unsigned long long *ocount,
                                                    uint32_t *abort, uint32_t max_fail, FStatus *sts,
                                                    uint32_t *counter, FChunkSummary *sum) {
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
            if (prev != 0xFFFFFFFFu) {
                // thread 0 wrote the chunk's status itself
                const FStatus &p = sts[prev];
                if (p.done) {
                    // totals of the finished chunks
                    atomicAdd(&sum->digest[0], p.digest[0]);
                    atomicXor(&sum->digest[1], p.digest[1]);
                    atomicMax(&sum->levels, p.levels);
                    for (uint32_t j = j0; j <= p.levels && j < k; j++) {
                        atomicAdd(&sum->lv_rows[j], p.lv_rows[j]);
                        atomicAdd(&sum->lv_gba[j], p.lv_gba[j]);
                        atomicAdd(&sum->lv_surv[j], p.lv_surv[j]);
                    }
                } else if (atomicAdd(abort + 1, 1u) + 1 > max_fail) {
                    // too many chunks that do not fit: leave the rest to the caller
                    atomicOr(abort, 1u);
                }
            }
            s_q = __atomic_load_n(abort, __ATOMIC_RELAXED) ? nchunks : atomicAdd(counter, 1u);
        }
        __syncthreads();
        const uint32_t qi = __builtin_amdgcn_readfirstlane(s_q);
        __syncthreads();
        if (qi >= nchunks) break;
        const uint32_t first = qi * chunk_rows;
        const uint32_t rows = min(chunk_rows, R0 - first);
        fused_query<FT, CR, CS, true>(plan, j0, M0 + first, rows, R0, buf0, buf1, loc, staging, sts + qi, L,
                                      ocount, staging_words);
        prev = qi;
        __syncthreads();
    }
}

// Each chunk's first output row (exclusive prefix of the counts, chunk
// order), its done flag, the row total and whether every chunk finished.
// The other totals were added by the chunk kernel.  One 1024-thread
// workgroup.
__global__ __launch_bounds__(1024) void k_chunk_summary(const FStatus *sts, uint32_t n, uint64_t *offs, uint32_t *done,
                                                       FChunkSummary *sum) {
    __shared__ uint64_t s_w[16];
    __shared__ uint32_t s_nd[16];
    const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
    uint64_t carry = 0;
    uint32_t notdone = 0;
    for (uint32_t base = 0; base < n; base += 1024) {
        const uint32_t i = base + tid;
        uint64_t c = 0;
        if (i < n) {
            const bool d = sts[i].done != 0;
            c = d ? sts[i].count : 0ull;
            done[i] = d ? 1u : 0u;
            notdone += d ? 0u : 1u;
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
    notdone = wave_sum(notdone);
    if (lane == 0) s_nd[w] = notdone;
    __syncthreads();
    if (tid == 0) {
        uint32_t nd = 0;
        for (uint32_t q = 0; q < 16; q++) nd += s_nd[q];
        offs[n] = carry;
        sum->all_done = nd == 0 ? 1u : 0u;
        sum->count = carry;
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
static void launch_chunks_t(gsi_ctx *c, uint32_t grid, const FPlan *plan, uint32_t j0, const uint32_t *M0, uint32_t R0,
                            uint32_t chunk_rows, uint32_t nchunks, uint32_t *scratch, uint64_t slot_words, uint32_t k,
                            uint32_t *staging, uint64_t staging_words, unsigned long long *ocount, uint32_t *abort,
                            uint32_t max_fail, FStatus *sts, uint32_t *counter, FChunkSummary *sum, double bytes) {
    constexpr uint32_t CR = 4 * FT, CS = 16 * FT;
    launch(c, "k_fused_chunks", bytes, k_fused_chunks<FT, CR, CS>, grid, FT, plan, j0, M0, R0, chunk_rows, nchunks,
           scratch, slot_words, k, staging, staging_words, ocount, abort, max_fail, sts, counter, sum);
}

void launch_fused_chunks(gsi_ctx *c, const FTier &t, uint32_t grid, const FPlan *plan, uint32_t j0, const uint32_t *M0,
                         uint32_t R0, uint32_t chunk_rows, uint32_t nchunks, uint32_t *scratch, uint64_t slot_words,
                         uint32_t k, uint32_t *staging, uint64_t staging_words, unsigned long long *ocount,
                         uint32_t *abort, uint32_t max_fail, FStatus *sts, uint32_t *counter, uint64_t *offs,
                         uint32_t *done, FChunkSummary *sum) {
    if (t.threads == 64)
        launch_chunks_t<64>(c, grid, plan, j0, M0, R0, chunk_rows, nchunks, scratch, slot_words, k, staging,
                            staging_words, ocount, abort, max_fail, sts, counter, sum, 0.0);
    else if (t.threads == 256)
        launch_chunks_t<256>(c, grid, plan, j0, M0, R0, chunk_rows, nchunks, scratch, slot_words, k, staging,
                             staging_words, ocount, abort, max_fail, sts, counter, sum, 0.0);
    else
        launch_chunks_t<1024>(c, grid, plan, j0, M0, R0, chunk_rows, nchunks, scratch, slot_words, k, staging,
                              staging_words, ocount, abort, max_fail, sts, counter, sum, 0.0);
    launch(c, "k_chunk_summary", 16.0 * nchunks, k_chunk_summary, 1, 1024, (const FStatus *)sts, nchunks, offs, done,
           sum);
}

void launch_chunk_gather(gsi_ctx *c, uint32_t nchunks, const FStatus *sts, const uint64_t *offs,
                         const uint32_t *staging, uint32_t k, uint32_t *out, uint64_t words) {
    launch(c, "k_chunk_gather", 8.0 * words, k_chunk_gather, nchunks, 256, sts, offs, staging, k, out);
}

// Rows of the given chunks, concatenated: workgroup i copies the `ncols`
// columns of chunk list[2i] to row list[2i+1] of dst (column stride `rows`).
__global__ __launch_bounds__(256) void k_take_rows(const uint32_t *M0, uint32_t R0, uint32_t ncols,
                                                  uint32_t chunk_rows, const uint32_t *list, uint32_t *dst,
                                                  uint64_t rows) {
    const uint32_t ch = list[2 * blockIdx.x], at = list[2 * blockIdx.x + 1];
    const uint32_t first = ch * chunk_rows;
    const uint32_t n = min(chunk_rows, R0 - first);
    for (uint32_t col = 0; col < ncols; col++)
        for (uint32_t t = threadIdx.x; t < n; t += 256)
            dst[(uint64_t)col * rows + at + t] = M0[(uint64_t)col * R0 + first + t];
}

void launch_take_rows(gsi_ctx *c, uint32_t nlist, const uint32_t *M0, uint32_t R0, uint32_t ncols,
                      uint32_t chunk_rows, const uint32_t *list, uint32_t *dst, uint64_t rows) {
    launch(c, "k_take_rows", 8.0 * rows * ncols, k_take_rows, nlist, 256, M0, R0, ncols, chunk_rows, list, dst,
           rows);
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
