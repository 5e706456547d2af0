// Workgroup scan used by the join kernels to map slots to rows.
#pragma once

#include "gsi_internal.h"

namespace gsi {

// Inclusive max-scan of s[0 .. NT*SPT) in place by a workgroup of NT
// threads, each taking SPT consecutive entries; s_w holds NT/64 words.
// Called by the whole workgroup; ends with a barrier.
template <uint32_t NT, uint32_t SPT>
__device__ __forceinline__ void block_max_scan(uint32_t *s, uint32_t *s_w) {
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t v[SPT], run = 0;
#pragma unroll
    for (uint32_t k = 0; k < SPT; k++) {
        run = max(run, s[threadIdx.x * SPT + k]);
        v[k] = run;
    }
    uint32_t inc = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o, 64);
        if (lane >= (uint32_t)o) inc = max(inc, t);
    }
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t pre = __shfl_up(inc, 1, 64);
    if (lane == 0) pre = 0;
    for (uint32_t q = 0; q < w; q++) pre = max(pre, s_w[q]);
#pragma unroll
    for (uint32_t k = 0; k < SPT; k++) s[threadIdx.x * SPT + k] = max(v[k], pre);
    __syncthreads();
}

}  // namespace gsi
