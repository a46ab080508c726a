// atomics.h -- device helper for maxima that every workgroup reports to one
// address (list lengths, cell occupancy).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// atomicMax that skips the atomic when the stored value is already at least
// v.  Thousands of workgroups updating one word otherwise queue up on the
// same L2 channel; after the first few, almost every call takes the skip.
__device__ __forceinline__ void atomic_max_rare(int32_t *p, int32_t v)
{
    if (v > __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(p, v);
}
