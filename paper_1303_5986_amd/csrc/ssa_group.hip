// ssa_group.hip -- the group kernel: L lanes per walker, 64 / L walkers per
// wave (gfx950), for networks between the lane kernels' register tables and
// the wave kernels' 64-reaction chunks.  The event loop is group_walker
// (ssa_group_body.h).
//
// Persistent grid: each wave takes 64 / L consecutive walkers of the work
// queue (the live walkers of every run, in bin segments ordered by their
// events per walker, built by launch_work_queue) with one atomic, runs them
// through the interval, and takes the next batch until the queue is empty.
// Counts live in LDS (S ints per walker, 64 / L walkers per wave, four waves
// per block); descriptors and changes are read through the cache.
#include "ssa_group_body.h"
#include "we_internal.h"

#include <algorithm>

#define GROUP_WAVES 4

template <int L>
__global__ __launch_bounds__(64 * GROUP_WAVES) void ssa_group_kernel(SimArgs a, int32_t *__restrict__ xs) {
    extern __shared__ int32_t glds[];
    constexpr int G = 64 / L;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int grp = lane / L;
    int32_t *lx = glds + ((size_t)wv * G + grp) * a.S;
    const uint32_t iter = *a.iter_dev;
    const uint32_t M = (uint32_t)a.m_targ, cap = (uint32_t)a.cap;
    const uint32_t total = a.queue[1] * M;
    for (;;) {
        // every lane executes the atomic (lane 0 adds G, the others zero) and
        // lane 0's result is broadcast, so no lane leaves the wave's path
        const uint32_t got = atomicAdd(&a.queue[0], lane == 0 ? (uint32_t)G : 0u);
        const uint32_t q0 = (uint32_t)__shfl((int)got, 0, 64);
        if (q0 >= total) break;
        const uint32_t q = q0 + (uint32_t)grp;
        bool live = false;
        int32_t run = 0, k = 0;
        if (q < total) {
            const uint32_t sg = q / M, o = q - sg * M;
            const int2 seg = a.seg[sg];
            if ((int32_t)o < seg.y) {
                const uint32_t g = (uint32_t)seg.x + o;
                run = (int32_t)(g / cap);
                k = (int32_t)(g - (uint32_t)run * cap);
                live = true;
            }
        }
        group_walker<L>(a, xs, run, k, live, iter, lx);
    }
}

namespace {
int group_cus() {
    static int n = 0;
    if (n == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
            n = 1;
    }
    return n;
}

template <int L>
hipError_t launch_group(const SimArgs &a, int32_t *xs, hipStream_t st) {
    constexpr int G = 64 / L;
    const size_t shmem = sizeof(int32_t) * (size_t)GROUP_WAVES * G * a.S;
    static size_t last_shmem = 0;
    static int per_cu = 0;
    if (per_cu == 0 || shmem != last_shmem) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ssa_group_kernel<L>, 64 * GROUP_WAVES, shmem) !=
                hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        last_shmem = shmem;
    }
    const int64_t walkers = (int64_t)a.n_runs * a.cap;
    const int64_t need = (walkers + (int64_t)GROUP_WAVES * G - 1) / ((int64_t)GROUP_WAVES * G);
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)per_cu * group_cus()));
    hipLaunchKernelGGL(ssa_group_kernel<L>, dim3(blocks), dim3(64 * GROUP_WAVES), shmem, st, a, xs);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_ssa_group(const SimArgs &a, int32_t *xs, int32_t lanes, hipStream_t st) {
    if (!group_kernel_fits(a.S, a.R, lanes)) return hipErrorInvalidValue;
    switch (lanes) {
    case 2: return launch_group<2>(a, xs, st);
    case 4: return launch_group<4>(a, xs, st);
    case 8: return launch_group<8>(a, xs, st);
    case 16: return launch_group<16>(a, xs, st);
    default: return launch_group<32>(a, xs, st);
    }
}

const char *ssa_group_name(int32_t lanes) {
    switch (lanes) {
    case 2: return "ssa_group_kernel<2>";
    case 4: return "ssa_group_kernel<4>";
    case 8: return "ssa_group_kernel<8>";
    case 16: return "ssa_group_kernel<16>";
    default: return "ssa_group_kernel<32>";
    }
}
