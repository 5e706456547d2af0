// A single-query entry point that allocates no device memory.
//
// gsi_query_run takes every scratch buffer of a query (candidate bitsets,
// the join tables M, F, locate records, keep bitmaps, tile counts, root
// chunk slots) and its result rows from the context's arena.  Callers that
// cannot have memory handed out during a call -- code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation -- call
// gsi_query_run_noalloc instead: the same path runs with its scratch carved
// out of `scratch`, a fixed array in the library's own device memory, and
// the rows are copied into a device buffer the caller owns.
//
// `scratch` is a host-side stand-in in host code: its device address is
// taken once per device with hipGetSymbolAddress (at context creation, with
// the context's device current) and only that address is ever used.  Every
// context on a device shares the array, and the array keeps what the last
// call left in it: nothing in the query path reads scratch memory it has not
// written in the same call.  Two calls that overlap on one device race on
// it; calls on one context are serialised by its busy flag, calls on
// different contexts of one device must be serialised by the caller.
#include <cstdio>
#include <map>
#include <mutex>
#include <utility>

#include "gsi_internal.h"

namespace gsi {

static __device__ __align__(256) uint8_t scratch[GSI_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, void *> g_scratch_ptr;  // device ordinal -> device address of `scratch`

// Takes the device address of `scratch` on `device`, which must be current.
// Called by gsi_ctx_create, once per device.
void noalloc_init(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        fail(GSI_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", device, hipGetErrorString(e));
    if ((uintptr_t)p % 256) fail(GSI_E_INTERNAL, "scratch array is not 256-byte aligned");
    g_scratch_ptr[device] = p;
}

static void *scratch_ptr(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it == g_scratch_ptr.end()) fail(GSI_E_INTERNAL, "no scratch address for device %d", device);
    return it->second;
}

// Puts a scratch arena in place of the context's arena for one call and
// restores it on scope exit, whatever the call's outcome.
struct ArenaSwap {
    gsi_ctx *c;
    Arena saved;
    ArenaSwap(gsi_ctx *cc, void *base, uint64_t bytes) : c(cc) {
        saved.init(base, bytes);
        std::swap(c->arena, saved);
    }
    ~ArenaSwap() { std::swap(c->arena, saved); }
};

}  // namespace gsi

using namespace gsi;

extern "C" gsi_status gsi_query_run_noalloc(gsi_graph *g, uint32_t k, const uint32_t *vl, uint32_t qm,
                                            const uint32_t *s, const uint32_t *d, const uint32_t *l, uint32_t flags,
                                            uint32_t *dev_rows, uint64_t capacity_rows, uint64_t *out_count,
                                            uint64_t out_digest[2]) {
    GSI_TRY({
        if (!g || !out_count || !out_digest) fail(GSI_E_INVALID, "null argument");
        *out_count = 0;
        out_digest[0] = out_digest[1] = 0;
        const bool count_only = (flags & GSI_COUNT_ONLY) != 0;
        if (!count_only && capacity_rows && !dev_rows) fail(GSI_E_INVALID, "null row buffer");
        if (g->multi) fail(GSI_E_INVALID, "gsi_query_run_noalloc takes single-label graphs");
        HostQuery q = validate_query(k, vl, qm, s, d, l);
        gsi_ctx *c = g->ctx;
        // the candidate bitsets alone must fit the scratch
        const uint64_t bitset_bytes = ((uint64_t)g->n + 63) / 64 * 8 * k;
        if (bitset_bytes > GSI_NOALLOC_SCRATCH_BYTES / 2)
            fail(GSI_E_CAPACITY,
                 "a %u-vertex query on %u data vertices needs %llu bytes of candidate bitsets, more than half of "
                 "the %llu-byte fixed scratch",
                 k, g->n, (unsigned long long)bitset_bytes, (unsigned long long)GSI_NOALLOC_SCRATCH_BYTES);
        Busy busy(c);
        GSI_HIP(hipSetDevice(c->device));
        void *base = scratch_ptr(c->device);
        gsi_query_options o{};
        o.flags = flags;
        gsi_result *r = nullptr;
        {
            ArenaSwap swap(c, base, GSI_NOALLOC_SCRATCH_BYTES);
            try {
                r = run_query(g, q, &o);
            } catch (const Fail &f) {
                if (f.st == GSI_E_NOMEM) {
                    char why[512];
                    snprintf(why, sizeof(why), "%s", gsi_last_error());
                    fail(GSI_E_CAPACITY, "the query needs more than the %llu-byte fixed scratch (%s)",
                         (unsigned long long)GSI_NOALLOC_SCRATCH_BYTES, why);
                }
                throw;
            }
            // the rows live in the scratch until they are copied out
            struct Drop {
                gsi_ctx *c;
                gsi_result *r;
                ~Drop() {
                    c->arena.release(r->rows);
                    delete r;
                }
            } drop{c, r};
            *out_count = r->count;
            out_digest[0] = r->digest[0];
            out_digest[1] = r->digest[1];
            if (!count_only && r->count) {
                if (r->count > capacity_rows)
                    fail(GSI_E_CAPACITY, "%llu rows do not fit the caller's %llu", (unsigned long long)r->count,
                         (unsigned long long)capacity_rows);
                GSI_HIP(hipMemcpyAsync(dev_rows, r->rows, r->count * (uint64_t)k * 4, hipMemcpyDeviceToDevice,
                                       c->stream));
            }
            // the next call may overwrite the scratch: the copy ends first
            GSI_HIP(hipStreamSynchronize(c->stream));
        }
    })
}
