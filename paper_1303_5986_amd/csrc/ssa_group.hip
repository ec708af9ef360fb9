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
// per block); the descriptors and changes are copied to LDS beside them when
// they take at most 48 KB (ssa_group_kernel<L, true>), else read through the
// cache (<L, false>).
#include "ssa_group_body.h"
#include "we_internal.h"

#include <algorithm>

#define GROUP_WAVES 4

// LDS copy of the network tables (descriptors, change offsets, changes),
// 16-byte aligned, in front of the walkers' counts.
__host__ __device__ inline size_t group_tables_bytes(int32_t R, int32_t n_chg) {
    return (16 * (size_t)R + 4 * ((size_t)R + 1 + (size_t)n_chg) + 15) & ~(size_t)15;
}

template <int L, bool LT, int BR>
__global__ __launch_bounds__(64 * GROUP_WAVES) void ssa_group_kernel(SimArgs a, int32_t *__restrict__ xs) {
    extern __shared__ __align__(16) unsigned char gsm[];
    constexpr int G = 64 / L;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int grp = lane / L;
    GroupTables tb{a.desc, a.chg_ptr, a.chg};
    size_t off = 0;
    if constexpr (LT) {
        const int32_t R = a.R;
        uint4 *ld = reinterpret_cast<uint4 *>(gsm);
        int32_t *lcp = reinterpret_cast<int32_t *>(gsm + 16 * (size_t)R);
        int32_t *lcg = lcp + R + 1;
        const uint4 *gd = reinterpret_cast<const uint4 *>(a.desc);
        for (int32_t i = threadIdx.x; i < R; i += blockDim.x) ld[i] = gd[i];
        for (int32_t i = threadIdx.x; i <= R; i += blockDim.x) lcp[i] = a.chg_ptr[i];
        for (int32_t i = threadIdx.x; i < a.n_chg; i += blockDim.x) lcg[i] = a.chg[i];
        __syncthreads();
        tb.desc = reinterpret_cast<const RxnDesc *>(ld);
        tb.chg_ptr = lcp;
        tb.chg = lcg;
        off = group_tables_bytes(R, a.n_chg);
    }
    int32_t *lx = reinterpret_cast<int32_t *>(gsm + off) + ((size_t)wv * G + grp) * a.S;
    const uint32_t iter = *a.iter_dev;
    const uint32_t M = (uint32_t)a.m_targ, cap = (uint32_t)a.cap;
    const uint32_t total = a.queue[1] * M;
    // G positions per wave: the first G at the wave's static first position
    uint32_t q0 = first_position() * (uint32_t)G;
    for (;;) {
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
        group_walker<L, BR>(a, tb, xs, run, k, live, iter, lx);
        // every lane executes the atomic (lane 0 adds G, the others zero) and
        // lane 0's result is broadcast, so no lane leaves the wave's path
        const uint32_t got = atomicAdd(&a.queue[0], lane == 0 ? (uint32_t)G : 0u);
        q0 = gridDim.x * (blockDim.x >> 6) * (uint32_t)G + (uint32_t)__shfl((int)got, 0, 64);
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

// Tables in LDS when they take at most GROUP_LDS_TABLES bytes (every
// reaction's descriptor and changes are then one LDS read away instead of a
// cache round trip in the event chain).
#define GROUP_LDS_TABLES (48 * 1024)

bool group_tables_in_lds(const SimArgs &a) { return group_tables_bytes(a.R, a.n_chg) <= GROUP_LDS_TABLES; }

// Blocks of at most 8 reactions per lane (with the tables in LDS) keep their
// descriptors and propensities in registers: 4 register slots for blocks of
// up to 4 (more would cost them occupancy), 8 for blocks of 5 to 8.
int group_regs(const SimArgs &a, int32_t lanes) {
    if (!group_tables_in_lds(a)) return 0;
    const int32_t B = (a.R + lanes - 1) / lanes;
    return B <= 4 ? 4 : B <= 8 ? 8 : 0;
}

template <int L, bool LT, int BR>
hipError_t launch_group(const SimArgs &a, int32_t *xs, hipStream_t st) {
    constexpr int G = 64 / L;
    const size_t shmem =
        (LT ? group_tables_bytes(a.R, a.n_chg) : 0) + sizeof(int32_t) * (size_t)GROUP_WAVES * G * a.S;
    static size_t last_shmem = 0;
    static int per_cu = 0;
    if (per_cu == 0 || shmem != last_shmem) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ssa_group_kernel<L, LT, BR>, 64 * GROUP_WAVES,
                                                         shmem) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        last_shmem = shmem;
    }
    const int64_t walkers = (int64_t)a.n_runs * a.cap;
    const int64_t need = (walkers + (int64_t)GROUP_WAVES * G - 1) / ((int64_t)GROUP_WAVES * G);
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)per_cu * group_cus()));
    hipLaunchKernelGGL((ssa_group_kernel<L, LT, BR>), dim3(blocks), dim3(64 * GROUP_WAVES), shmem, st, a, xs);
    return hipGetLastError();
}

template <int L>
hipError_t launch_group(const SimArgs &a, int32_t *xs, hipStream_t st) {
    const int br = group_regs(a, L);
    if (br == 4) return launch_group<L, true, 4>(a, xs, st);
    if (br == 8) return launch_group<L, true, 8>(a, xs, st);
    return group_tables_in_lds(a) ? launch_group<L, true, 0>(a, xs, st) : launch_group<L, false, 0>(a, xs, st);
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

const char *ssa_group_name(const SimArgs &a, int32_t lanes) {
    // 5 lane counts x (4 or 8 register slots, tables in LDS, through the cache)
    static const char *const names[5][4] = {
        {"ssa_group_kernel<2, true, 4>", "ssa_group_kernel<2, true, 8>", "ssa_group_kernel<2, true, 0>",
         "ssa_group_kernel<2, false, 0>"},
        {"ssa_group_kernel<4, true, 4>", "ssa_group_kernel<4, true, 8>", "ssa_group_kernel<4, true, 0>",
         "ssa_group_kernel<4, false, 0>"},
        {"ssa_group_kernel<8, true, 4>", "ssa_group_kernel<8, true, 8>", "ssa_group_kernel<8, true, 0>",
         "ssa_group_kernel<8, false, 0>"},
        {"ssa_group_kernel<16, true, 4>", "ssa_group_kernel<16, true, 8>", "ssa_group_kernel<16, true, 0>",
         "ssa_group_kernel<16, false, 0>"},
        {"ssa_group_kernel<32, true, 4>", "ssa_group_kernel<32, true, 8>", "ssa_group_kernel<32, true, 0>",
         "ssa_group_kernel<32, false, 0>"}};
    const int li = lanes == 2 ? 0 : lanes == 4 ? 1 : lanes == 8 ? 2 : lanes == 16 ? 3 : 4;
    const int br = group_regs(a, lanes);
    const int vi = br == 4 ? 0 : br == 8 ? 1 : group_tables_in_lds(a) ? 2 : 3;
    return names[li][vi];
}
