// C ABI entry points, error reporting, the device arena and kernel timing.
#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <set>
#include <vector>
#include <cstdio>
#include <cstring>

#include "gsi_internal.h"

namespace gsi {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}
void clear_error() { g_err[0] = 0; }

void fail(gsi_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    throw Fail{st};
}

// ------------------------------------------------------------------- arena
static constexpr uint64_t ALIGN = 256;
static inline uint64_t round_up(uint64_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

void Arena::init(void *base, uint64_t size) {
    uintptr_t b = (uintptr_t)base;
    base_ = b;
    size_ = size & ~(ALIGN - 1);
    free_.clear();
    live_.clear();
    free_[0] = size_;
    used_ = peak_ = 0;
}

void *Arena::alloc(uint64_t bytes, bool high) {
    bytes = round_up(bytes ? bytes : 1);
    if (high) {
        for (auto it = free_.rbegin(); it != free_.rend(); ++it) {
            if (it->second >= bytes) {
                uint64_t off = it->first, sz = it->second;
                uint64_t at = off + sz - bytes;
                free_.erase(off);
                if (sz > bytes) free_[off] = sz - bytes;
                live_[at] = bytes;
                used_ += bytes;
                if (used_ > peak_) peak_ = used_;
                return (void *)(base_ + at);
            }
        }
    } else {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                uint64_t off = it->first, sz = it->second;
                free_.erase(it);
                if (sz > bytes) free_[off + bytes] = sz - bytes;
                live_[off] = bytes;
                used_ += bytes;
                if (used_ > peak_) peak_ = used_;
                return (void *)(base_ + off);
            }
        }
    }
    return nullptr;
}

void Arena::release(void *p) {
    if (!p) return;
    uint64_t off = (uintptr_t)p - base_;
    auto it = live_.find(off);
    if (it == live_.end()) return;
    uint64_t sz = it->second;
    live_.erase(it);
    used_ -= sz;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + sz) {
        sz += nx->second;
        free_.erase(nx);
    }
    auto pv = free_.lower_bound(off);
    if (pv != free_.begin()) {
        --pv;
        if (pv->first + pv->second == off) {
            pv->second += sz;
            return;
        }
    }
    free_[off] = sz;
}

void Arena::shrink(void *p, uint64_t bytes) {
    if (!p) return;
    uint64_t off = (uintptr_t)p - base_;
    auto it = live_.find(off);
    if (it == live_.end()) return;
    uint64_t keep = round_up(bytes ? bytes : 1);
    if (keep >= it->second) return;
    uint64_t tail = it->second - keep;
    it->second = keep;
    used_ -= tail;
    live_[off + keep] = tail;  // hand the tail back through release()
    used_ += tail;
    release((void *)(base_ + off + keep));
}

uint64_t Arena::largest_free() const {
    uint64_t b = 0;
    for (auto &kv : free_) b = kv.second > b ? kv.second : b;
    return b;
}

// --------------------------------------------------------------- timing
int kernel_id(gsi_ctx *c, const char *name) {
    for (size_t i = 0; i < c->knames.size(); i++)
        if (c->knames[i] == name) return (int)i;
    c->knames.push_back(name);
    gsi_kernel_stat st{};
    snprintf(st.name, sizeof(st.name), "%s", name);
    c->acc.push_back(st);
    return (int)c->knames.size() - 1;
}

hipEvent_t take_event(gsi_ctx *c) {
    if (!c->free_events.empty()) {
        hipEvent_t e = c->free_events.back();
        c->free_events.pop_back();
        return e;
    }
    hipEvent_t e;
    GSI_HIP(hipEventCreate(&e));
    return e;
}

// launches with at least this many algorithmic bytes are also summed under
// "<kernel>@large", so bandwidth-bound launches can be read apart from the
// latency-bound small ones
static constexpr double LARGE_LAUNCH_BYTES = 16.0 * (1 << 20);

static void drain_records(gsi_ctx *c) {
    if (c->recs.empty()) return;
    GSI_HIP(hipStreamSynchronize(c->stream));
    for (auto &r : c->recs) {
        float ms = 0;
        GSI_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        c->acc[r.kid].launches++;
        c->acc[r.kid].total_ms += ms;
        c->acc[r.kid].alg_bytes += r.bytes;
        if (r.bytes >= LARGE_LAUNCH_BYTES) {
            std::string big = c->knames[r.kid] + "@large";
            int kb = kernel_id(c, big.c_str());
            c->acc[kb].launches++;
            c->acc[kb].total_ms += ms;
            c->acc[kb].alg_bytes += r.bytes;
        }
        c->free_events.push_back(r.a);
        c->free_events.push_back(r.b);
    }
    c->recs.clear();
}

// how long wait_mailbox spins for the completion word before it
// synchronises the stream instead
constexpr int64_t SEQ_SPIN_US = 500;

// posts the completion word once every earlier launch on the stream is done
__global__ void k_post(uint64_t *slot, uint64_t value) {
    if (threadIdx.x == 0) post_seq(slot, value);
}

void wait_mailbox(gsi_ctx *c) {
    if (!c->seq_armed) {
        // no kernel posts the word after its scalars: a one-wave launch that
        // runs after every earlier one does (still ~4 us sooner than a
        // stream sync)
        const uint64_t v = ++c->seq;
        launch(c, "k_post", 0.0, k_post, 1, 64, c->mbox_dev + MBOX_SEQ, v);
        c->seq_armed = true;
    }
    bool seen = false;
    const volatile uint64_t *w = c->mbox_host + MBOX_SEQ;
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t it = 0;; it++) {
        if (*w == c->seq) {
            seen = true;
            break;
        }
        if ((it & 255) == 255 && std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(SEQ_SPIN_US)) break;
    }
    c->seq_armed = false;
    if (!seen) GSI_HIP(hipStreamSynchronize(c->stream));
    std::atomic_thread_fence(std::memory_order_acquire);
}

void read_scalars(gsi_ctx *c, const uint64_t *dev, uint64_t *host, int n) {
    if (c->mbox_dev && dev >= c->mbox_dev && dev + n <= c->mbox_dev + MAILBOX_WORDS) {
        wait_mailbox(c);
        memcpy(host, c->mbox_host + (dev - c->mbox_dev), sizeof(uint64_t) * n);
        return;
    }
    GSI_HIP(hipMemcpyAsync(c->pinned, dev, sizeof(uint64_t) * n, hipMemcpyDeviceToHost, c->stream));
    GSI_HIP(hipStreamSynchronize(c->stream));
    memcpy(host, c->pinned, sizeof(uint64_t) * n);
}

void sync(gsi_ctx *c) { GSI_HIP(hipStreamSynchronize(c->stream)); }

}  // namespace gsi

using namespace gsi;

#define REQUIRE(cond, ...)                   \
    do {                                     \
        if (!(cond)) fail(GSI_E_INVALID, __VA_ARGS__); \
    } while (0)

extern "C" {

const char *gsi_last_error(void) { return gsi::g_err; }
const char *gsi_version(void) { return "gsi-mi355x 0.1 (gfx950)"; }

gsi_status gsi_ctx_create(const gsi_options *o, gsi_ctx **out) {
    GSI_TRY({
        REQUIRE(o && out, "null argument");
        *out = nullptr;
        REQUIRE(o->arena_ptr && ((uintptr_t)o->arena_ptr % 256) == 0, "arena must be non-null and 256-byte aligned");
        REQUIRE(o->arena_bytes >= (1ull << 20), "arena must hold at least 1 MiB");
        GSI_HIP(hipSetDevice(o->device));
        noalloc_init(o->device);
        gsi_ctx *c = new gsi_ctx();
        c->device = o->device;
        c->stream = (hipStream_t)o->hip_stream;
        c->flags = o->flags;
        c->arena.init(o->arena_ptr, o->arena_bytes);
        hipError_t e = hipHostMalloc((void **)&c->pinned, 65536, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&c->mbox_host, MAILBOX_WORDS * 8, hipHostMallocCoherent | hipHostMallocMapped);
        if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&c->mbox_dev, c->mbox_host, 0);
        if (e != hipSuccess) {
            if (c->pinned) (void)hipHostFree(c->pinned);
            if (c->mbox_host) (void)hipHostFree(c->mbox_host);
            delete c;
            fail(GSI_E_DEVICE, "hipHostMalloc failed: %s", hipGetErrorString(e));
        }
        *out = c;
    })
}

gsi_status gsi_ctx_destroy(gsi_ctx *c) {
    GSI_TRY({
        if (!c) return GSI_OK;
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        for (auto *r : c->results) delete r;
        for (auto *g : c->graphs) delete g;
        for (auto &r : c->recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : c->free_events) (void)hipEventDestroy(e);
        if (c->pinned) (void)hipHostFree(c->pinned);
        if (c->mbox_host) (void)hipHostFree(c->mbox_host);
        delete c;
    })
}

gsi_status gsi_ctx_memory(const gsi_ctx *c, uint64_t *live, uint64_t *peak) {
    GSI_TRY({
        REQUIRE(c, "null context");
        if (live) *live = c->arena.used();
        if (peak) *peak = c->arena.peak();
    })
}

gsi_status gsi_ctx_kernel_stats(gsi_ctx *c, gsi_kernel_stat *out, uint32_t cap, uint32_t *n) {
    GSI_TRY({
        REQUIRE(c && n, "null argument");
        GSI_HIP(hipSetDevice(c->device));
        drain_records(c);
        uint32_t cnt = 0;
        for (size_t i = 0; i < c->acc.size() && cnt < cap; i++) out[cnt++] = c->acc[i];
        *n = cnt;
    })
}

gsi_status gsi_ctx_kernel_stats_reset(gsi_ctx *c) {
    GSI_TRY({
        REQUIRE(c, "null context");
        GSI_HIP(hipSetDevice(c->device));
        drain_records(c);
        for (auto &a : c->acc) {
            a.launches = 0;
            a.total_ms = 0;
            a.alg_bytes = 0;
        }
    })
}

gsi_status gsi_graph_bytes_needed(uint32_t n, uint64_t m, uint64_t *out) {
    GSI_TRY({
        REQUIRE(out, "null argument");
        uint64_t d = 2 * m;
        // persistent: signatures 64 B per vertex, at most one 128 B group per
        // directed edge, ci 4 B per directed edge
        uint64_t persistent = 64ull * n + 128ull * d + 4ull * d;
        // build scratch (see build_graph): sort buffers 6 x 4 B, scans 3 x 8 B
        // and the per-run / per-group arrays, bounded by directed edges
        uint64_t scratch = d * (24 + 8) + d * 96 + 4ull * n + (64ull << 20);
        *out = persistent + scratch;
    })
}

static gsi_status load_common(gsi_ctx *c, uint32_t n, const uint32_t *vl, uint64_t m, const uint32_t *s,
                              const uint32_t *d, const uint32_t *l, uint32_t flags, gsi_graph **out,
                              bool device) {
    GSI_TRY({
        REQUIRE(c && out, "null argument");
        *out = nullptr;
        REQUIRE(n > 0 && n < 0xFFFFFFFFu, "n_vertices must be in [1, 2^32-2]");
        REQUIRE(m <= 0x7FFFFFFFull, "at most 2^31-1 edges");
        REQUIRE(vl && (m == 0 || (s && d && l)), "null input array");
        REQUIRE((flags & ~(GSI_GRAPH_TEST_FEW_HOME_GROUPS | GSI_GRAPH_KEEP_CR)) == 0, "unknown graph flag");
        Busy busy(c);
        GSI_HIP(hipSetDevice(c->device));
        gsi_graph *g = new gsi_graph();
        g->ctx = c;
        g->n = n;
        g->m = m;
        g->flags = flags;
        try {
            if (device) {
                build_graph(g, vl, s, d, l);
            } else {
                Scratch sc(c);
                uint32_t *dv = sc.get<uint32_t>(n, "vertex labels");
                uint32_t *ds = sc.get<uint32_t>(m, "src");
                uint32_t *dd = sc.get<uint32_t>(m, "dst");
                uint32_t *de = sc.get<uint32_t>(m, "edge labels");
                GSI_HIP(hipMemcpyAsync(dv, vl, 4ull * n, hipMemcpyHostToDevice, c->stream));
                if (m) {
                    GSI_HIP(hipMemcpyAsync(ds, s, 4ull * m, hipMemcpyHostToDevice, c->stream));
                    GSI_HIP(hipMemcpyAsync(dd, d, 4ull * m, hipMemcpyHostToDevice, c->stream));
                    GSI_HIP(hipMemcpyAsync(de, l, 4ull * m, hipMemcpyHostToDevice, c->stream));
                }
                build_graph(g, dv, ds, dd, de);
                sync(c);
            }
        } catch (...) {
            (void)hipStreamSynchronize(c->stream);
            c->arena.release(g->vl_off);
            c->arena.release(g->vl_lab);
            c->arena.release(g->sig);
            c->arena.release(g->gl);
            c->arena.release(g->ci);
            c->arena.release(g->cr_vid);
            c->arena.release(g->cr_start);
            c->arena.release(g->cr_off);
            delete g;
            throw;
        }
        c->graphs.insert(g);
        *out = g;
    })
}

gsi_status gsi_graph_load(gsi_ctx *c, uint32_t n, const uint32_t *vl, uint64_t m, const uint32_t *s,
                          const uint32_t *d, const uint32_t *l, uint32_t flags, gsi_graph **out) {
    return load_common(c, n, vl, m, s, d, l, flags, out, false);
}

gsi_status gsi_graph_load_device(gsi_ctx *c, uint32_t n, const uint32_t *vl, uint64_t m, const uint32_t *s,
                                 const uint32_t *d, const uint32_t *l, uint32_t flags, gsi_graph **out) {
    return load_common(c, n, vl, m, s, d, l, flags, out, true);
}

gsi_status gsi_graph_load_multi(gsi_ctx *c, uint32_t n, const uint64_t *off, const uint32_t *lab, uint64_t m,
                                const uint32_t *s, const uint32_t *d, const uint32_t *l, uint32_t flags,
                                gsi_graph **out) {
    GSI_TRY({
        REQUIRE(c && out, "null argument");
        *out = nullptr;
        REQUIRE(n > 0 && n < 0xFFFFFFFFu, "n_vertices must be in [1, 2^32-2]");
        REQUIRE(m <= 0x7FFFFFFFull, "at most 2^31-1 edges");
        REQUIRE(off && (off[n] == 0 || lab) && (m == 0 || (s && d && l)), "null input array");
        REQUIRE(off[0] == 0 && off[n] < 0xFFFFFFFFull, "label offsets must start at 0 and stay below 2^32-1");
        REQUIRE((flags & ~(GSI_GRAPH_TEST_FEW_HOME_GROUPS | GSI_GRAPH_KEEP_CR)) == 0, "unknown graph flag");
        // label sets, each sorted and without repeats, as 32-bit offsets
        std::vector<uint32_t> hoff(n + 1), hlab;
        hlab.reserve(off[n]);
        for (uint32_t v = 0; v < n; v++) {
            REQUIRE(off[v + 1] >= off[v], "label offsets must not decrease");
            std::vector<uint32_t> ls(lab + off[v], lab + off[v + 1]);
            std::sort(ls.begin(), ls.end());
            ls.erase(std::unique(ls.begin(), ls.end()), ls.end());
            hoff[v] = (uint32_t)hlab.size();
            hlab.insert(hlab.end(), ls.begin(), ls.end());
        }
        hoff[n] = (uint32_t)hlab.size();
        Busy busy(c);
        GSI_HIP(hipSetDevice(c->device));
        gsi_graph *g = new gsi_graph();
        g->ctx = c;
        g->n = n;
        g->m = m;
        g->flags = flags;
        g->multi = true;
        try {
            g->vl_off = persist<uint32_t>(c, n + 1ull, "vertex label offsets");
            g->vl_lab = persist<uint32_t>(c, hlab.size() + 1, "vertex label sets");
            GSI_HIP(hipMemcpyAsync(g->vl_off, hoff.data(), 4ull * (n + 1), hipMemcpyHostToDevice, c->stream));
            if (!hlab.empty())
                GSI_HIP(hipMemcpyAsync(g->vl_lab, hlab.data(), 4ull * hlab.size(), hipMemcpyHostToDevice, c->stream));
            Scratch sc(c);
            uint32_t *ds = sc.get<uint32_t>(m, "src");
            uint32_t *dd = sc.get<uint32_t>(m, "dst");
            uint32_t *de = sc.get<uint32_t>(m, "edge labels");
            if (m) {
                GSI_HIP(hipMemcpyAsync(ds, s, 4ull * m, hipMemcpyHostToDevice, c->stream));
                GSI_HIP(hipMemcpyAsync(dd, d, 4ull * m, hipMemcpyHostToDevice, c->stream));
                GSI_HIP(hipMemcpyAsync(de, l, 4ull * m, hipMemcpyHostToDevice, c->stream));
            }
            build_graph(g, nullptr, ds, dd, de);
            sync(c);
        } catch (...) {
            (void)hipStreamSynchronize(c->stream);
            c->arena.release(g->vl_off);
            c->arena.release(g->vl_lab);
            c->arena.release(g->sig);
            c->arena.release(g->gl);
            c->arena.release(g->ci);
            c->arena.release(g->cr_vid);
            c->arena.release(g->cr_start);
            c->arena.release(g->cr_off);
            delete g;
            throw;
        }
        c->graphs.insert(g);
        *out = g;
    })
}

gsi_status gsi_graph_free(gsi_graph *g) {
    GSI_TRY({
        if (!g) return GSI_OK;
        gsi_ctx *c = g->ctx;
        Busy busy(c);
        GSI_HIP(hipSetDevice(c->device));
        GSI_HIP(hipStreamSynchronize(c->stream));
        c->arena.release(g->vl_off);
        c->arena.release(g->vl_lab);
        c->arena.release(g->sig);
        c->arena.release(g->gl);
        c->arena.release(g->ci);
        c->arena.release(g->cr_vid);
        c->arena.release(g->cr_start);
        c->arena.release(g->cr_off);
        c->graphs.erase(g);
        delete g;
    })
}

gsi_status gsi_graph_get_info(const gsi_graph *g, gsi_graph_info *out) {
    GSI_TRY({
        REQUIRE(g && out, "null argument");
        out->n_vertices = g->n;
        out->n_edges = g->m;
        out->n_edge_labels = g->nlab;
        out->total_groups = g->total_groups;
        out->max_chain = g->max_chain;
        out->device_bytes = g->bytes;
        out->build_ms = g->build_ms;
    })
}

gsi_status gsi_graph_label_edges(const gsi_graph *g, uint32_t label, uint64_t *out) {
    GSI_TRY({
        REQUIRE(g && out, "null argument");
        *out = label < g->nlab ? g->edges[label] : 0;
    })
}

gsi_status gsi_graph_copy_signatures(const gsi_graph *g, uint32_t *dst, uint64_t cap) {
    GSI_TRY({
        REQUIRE(g && dst, "null argument");
        uint64_t need = (uint64_t)GSI_SIG_WORDS * g->n;
        if (cap < need) fail(GSI_E_CAPACITY, "need %llu words", (unsigned long long)need);
        gsi_ctx *c = g->ctx;
        Busy busy(c);
        GSI_HIP(hipSetDevice(c->device));
        GSI_HIP(hipMemcpyAsync(dst, g->sig, need * 4, hipMemcpyDeviceToHost, c->stream));
        GSI_HIP(hipStreamSynchronize(c->stream));
    })
}

gsi_status gsi_graph_copy_pcsr(const gsi_graph *g, uint32_t label, uint32_t *hgl, uint64_t glcap, uint32_t *hci,
                               uint64_t cicap, uint64_t *out_groups, uint64_t *out_ci) {
    GSI_TRY({
        REQUIRE(g, "null graph");
        uint64_t groups = label < g->nlab ? g->G[label] : 0;
        uint64_t cil = label < g->nlab ? 2 * g->edges[label] : 0;
        if (out_groups) *out_groups = groups;
        if (out_ci) *out_ci = cil;
        if (glcap == 0 && cicap == 0) return GSI_OK;
        if (glcap < groups * GROUP_WORDS || cicap < cil) fail(GSI_E_CAPACITY, "buffers too small");
        REQUIRE(hgl && hci, "null buffer");
        gsi_ctx *c = g->ctx;
        Busy busy(c);
        GSI_HIP(hipSetDevice(c->device));
        if (groups)
            GSI_HIP(hipMemcpyAsync(hgl, g->gl + g->group_base[label] * GROUP_WORDS, groups * GROUP_WORDS * 4,
                                   hipMemcpyDeviceToHost, c->stream));
        if (cil)
            GSI_HIP(hipMemcpyAsync(hci, g->ci + g->ci_base[label], cil * 4, hipMemcpyDeviceToHost, c->stream));
        GSI_HIP(hipStreamSynchronize(c->stream));
    })
}

gsi_status gsi_query_run(gsi_graph *g, uint32_t k, const uint32_t *vl, uint32_t qm, const uint32_t *s,
                         const uint32_t *d, const uint32_t *l, const gsi_query_options *opt, gsi_result **out) {
    GSI_TRY({
        REQUIRE(g && out, "null argument");
        *out = nullptr;
        HostQuery q = validate_query(k, vl, qm, s, d, l);
        if (g->multi) make_multi(q);
        gsi_ctx *c = g->ctx;
        Busy busy(c);
        GSI_HIP(hipSetDevice(c->device));
        gsi_result *r = run_query(g, q, opt);
        c->results.insert(r);
        *out = r;
    })
}

gsi_status gsi_query_run_multi(gsi_graph *g, uint32_t k, const uint32_t *off, const uint32_t *lab, uint32_t qm,
                               const uint32_t *s, const uint32_t *d, const uint32_t *l, const gsi_query_options *opt,
                               gsi_result **out) {
    GSI_TRY({
        REQUIRE(g && out, "null argument");
        *out = nullptr;
        HostQuery q = validate_query_multi(k, off, lab, qm, s, d, l);
        gsi_ctx *c = g->ctx;
        Busy busy(c);
        GSI_HIP(hipSetDevice(c->device));
        gsi_result *r = nullptr;
        bool single = !g->multi;
        for (uint32_t u = 0; single && u < k; u++) single = q.vls[u].size() == 1;
        if (!g->multi && !single) {
            // one label per data vertex: a query vertex asking two or none
            // (a pair asking two labels fails the same way below) has no image
            r = new gsi_result();
            r->ctx = c;
            r->k = k;
            r->count_only = opt && (opt->flags & GSI_COUNT_ONLY);
            r->stats.k = k;
        } else {
            if (!g->multi) {
                // pairs with two labels cannot match a single-label graph
                std::set<std::pair<uint32_t, uint32_t>> seen;
                bool parallel = false;
                for (uint32_t e = 0; e < q.src.size(); e++)
                    parallel |= !seen.insert({std::min(q.src[e], q.dst[e]), std::max(q.src[e], q.dst[e])}).second;
                if (parallel) {
                    r = new gsi_result();
                    r->ctx = c;
                    r->k = k;
                    r->count_only = opt && (opt->flags & GSI_COUNT_ONLY);
                    r->stats.k = k;
                } else {
                    q.multi = false;
                }
            }
            if (!r) r = run_query(g, q, opt);
        }
        c->results.insert(r);
        *out = r;
    })
}

gsi_status gsi_query_filter(gsi_graph *g, uint32_t k, const uint32_t *vl, uint32_t qm, const uint32_t *s,
                            const uint32_t *d, const uint32_t *l, uint64_t *hbits, uint64_t cap, uint32_t *hcounts) {
    GSI_TRY({
        REQUIRE(g && hbits && hcounts, "null argument");
        HostQuery q = validate_query(k, vl, qm, s, d, l);
        uint64_t words = ((uint64_t)g->n + 63) / 64;
        if (cap < words * k) fail(GSI_E_CAPACITY, "need %llu words", (unsigned long long)(words * k));
        gsi_ctx *c = g->ctx;
        Busy busy(c);
        GSI_HIP(hipSetDevice(c->device));
        Scratch sc(c);
        uint64_t *bits = sc.get<uint64_t>(words * k, "candidate bitsets");
        uint32_t *cnt = sc.get<uint32_t>(k, "candidate counts");
        if (g->multi) make_multi(q);
        run_filter(g, q, bits, cnt);
        GSI_HIP(hipMemcpyAsync(hbits, bits, words * k * 8, hipMemcpyDeviceToHost, c->stream));
        GSI_HIP(hipMemcpyAsync(hcounts, cnt, 4ull * k, hipMemcpyDeviceToHost, c->stream));
        GSI_HIP(hipStreamSynchronize(c->stream));
    })
}

gsi_status gsi_result_count(const gsi_result *r, uint64_t *rows) {
    GSI_TRY({
        REQUIRE(r && rows, "null argument");
        *rows = r->count;
    })
}

gsi_status gsi_result_rows(const gsi_result *r, uint32_t *dst, uint64_t cap) {
    GSI_TRY({
        REQUIRE(r, "null result");
        REQUIRE(!r->count_only, "result was computed with GSI_COUNT_ONLY");
        if (cap < r->count) fail(GSI_E_CAPACITY, "need %llu rows", (unsigned long long)r->count);
        if (r->count == 0) return GSI_OK;
        REQUIRE(dst, "null buffer");
        gsi_ctx *c = r->ctx;
        GSI_HIP(hipSetDevice(c->device));
        GSI_HIP(hipMemcpyAsync(dst, r->rows, r->count * r->k * 4, hipMemcpyDeviceToHost, c->stream));
        GSI_HIP(hipStreamSynchronize(c->stream));
    })
}

gsi_status gsi_result_device_rows(const gsi_result *r, const uint32_t **p) {
    GSI_TRY({
        REQUIRE(r && p, "null argument");
        REQUIRE(!r->count_only, "result was computed with GSI_COUNT_ONLY");
        *p = r->rows;
    })
}

gsi_status gsi_result_digest(const gsi_result *r, uint64_t out[2]) {
    GSI_TRY({
        REQUIRE(r && out, "null argument");
        out[0] = r->digest[0];
        out[1] = r->digest[1];
    })
}

gsi_status gsi_result_stats(const gsi_result *r, gsi_stats *out) {
    GSI_TRY({
        REQUIRE(r && out, "null argument");
        *out = r->stats;
    })
}

gsi_status gsi_result_free(gsi_result *r) {
    GSI_TRY({
        if (!r) return GSI_OK;
        gsi_ctx *c = r->ctx;
        GSI_HIP(hipSetDevice(c->device));
        GSI_HIP(hipStreamSynchronize(c->stream));
        c->arena.release(r->rows);
        c->results.erase(r);
        delete r;
    })
}

}  // extern "C"
