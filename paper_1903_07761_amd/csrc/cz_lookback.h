// Single-pass decoupled look-back (an exclusive prefix sum of sizes over
// items taken in ticket order), shared by the block kernels and the lossless
// stage's encoder.  It places each compressed piece after all earlier ones,
// the exclusive scan of compressed sizes of arXiv 1903.07761, Sec. 2.2.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "cz_kernels.h"

namespace czk {

static constexpr uint64_t FLAG_AGG = 1ull << 62;
static constexpr uint64_t FLAG_INC = 2ull << 62;
static constexpr uint64_t FLAG_VAL = (1ull << 62) - 1;
static constexpr uint32_t LOOKBACK_SPIN_LIMIT = 1u << 24;

__device__ __forceinline__ uint64_t atomic_load_u64(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_store_u64(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decoupled look-back over the blocks of a field, run by one wavefront:
// publish this block's record size (FLAG_AGG), sum the sizes of the earlier
// blocks back to the nearest inclusive prefix, publish the inclusive prefix
// (FLAG_INC) and return the exclusive one (on every lane).  Lane k examines
// the flag of the (k+1)-th nearest earlier block, so one step covers 64
// predecessors; the lanes up to the nearest inclusive prefix must all have
// published before their sizes are summed.  Every wait is bounded: on
// exhaustion the status word gets STATUS_TIMEOUT.
//
// lookback_publish and lookback_resolve are its two halves, for callers that
// do other work in between (the predecessors then have more time to publish):
// publish first, resolve later; block 0 publishes its inclusive prefix at once.
__device__ inline void lookback_publish(uint64_t *flags, uint64_t b, uint64_t size)
{
    if (__lane_id() == 0)
        atomic_store_u64(&flags[b], (b == 0 ? FLAG_INC : FLAG_AGG) | size);
}

__device__ inline uint64_t lookback_resolve(uint64_t *flags, uint64_t b, uint64_t size, uint32_t *status,
                                            uint32_t *fstatus)
{
    const uint32_t lane = __lane_id();
    if (b == 0)
        return 0;
    uint64_t excl = 0;
    uint64_t top = b;  // this step covers blocks [top - 64, top)
    uint32_t spins = 0;
    while (true) {
        const bool valid = top > (uint64_t)lane;
        const uint64_t f = valid ? atomic_load_u64(&flags[top - 1 - lane]) : FLAG_INC;
        const uint64_t st = f & ~FLAG_VAL;
        const uint64_t inc = __ballot(st == FLAG_INC);
        const uint64_t empty = __ballot(st == 0);
        const uint32_t first = inc ? (uint32_t)__builtin_ctzll(inc) : 64u;
        const uint64_t upto = first >= 63 ? ~0ull : ((2ull << first) - 1ull);  // lanes [0, first]
        if (empty & upto) {
            if (++spins > LOOKBACK_SPIN_LIMIT) {
                if (lane == 0) {
                    atomicOr(status, STATUS_TIMEOUT);
                    if (fstatus)
                        atomicOr(fstatus, STATUS_TIMEOUT);
                }
                break;
            }
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        uint64_t v = lane <= first ? (f & FLAG_VAL) : 0ull;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            v += __shfl_xor(v, o);
        excl += v;
        if (inc)
            break;
        top -= 64;
    }
    if (lane == 0)
        atomic_store_u64(&flags[b], FLAG_INC | (excl + size));
    return excl;
}

__device__ inline uint64_t lookback_wave(uint64_t *flags, uint64_t b, uint64_t size, uint32_t *status, uint32_t *fstatus)
{
    lookback_publish(flags, b, size);
    return lookback_resolve(flags, b, size, status, fstatus);
}

}  // namespace czk
