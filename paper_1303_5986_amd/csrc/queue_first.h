// queue_first.h -- the first work-queue position of each wave of a
// persistent propagation kernel.
//
// The queue lists the walkers busiest bin first.  Taken by a queue atomic
// alone, its front would go to whichever waves ask first -- in practice the
// waves of the first blocks, so the busiest walkers would share the SIMDs of
// a few CUs while the last CUs idle.  Instead the first position of wave wv
// of block b is wv * gridDim.x + b: the front of the queue lands on wave 0
// of every block (one per CU, one SIMD each), the next stretch on wave 1,
// and so on; afterwards a wave takes position gridDim.x * waves_per_block +
// (queue atomic).  Each position still goes to exactly one wave, and no
// result depends on which wave runs a walker.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace {
__device__ __forceinline__ uint32_t first_position() {
    return (uint32_t)(threadIdx.x >> 6) * gridDim.x + blockIdx.x;
}
}  // namespace
