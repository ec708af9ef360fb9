// ssa_lane.hip -- Gillespie direct-method SSA, one lane per walker (gfx950).
//
// Each lane carries one walker through one WE interval tau (Sec. II.A, the
// propagation step of the WE procedure in Sec. II.B):
//   1. all propensities a_j = c_j * prod_s C(x_s, nu_js) (divided by
//      1 + (x_r / K)^n for a Hill-type rate, Sec. III.C) and their total a0,
//      summed in reaction order;
//   2. waiting time dt = -log(1 - u1) / a0; stop when t + dt > tau (the
//      exponential is memoryless, so the overshoot is simply discarded);
//   3. reaction j = first index whose running sum exceeds u2 * a0;
//   4. x += nu_j, t += dt.
// u1, u2 come from one Philox4x32-10 block at counter (event, slot, iter, 0).
//
// Design for CDNA4: walker state and propensities live in VGPRs, the
// reaction table is wave-uniform (scalar loads), and the state change of the
// chosen reaction is an int8 delta row picked by register selects (up to 8
// reactions) or read from the wave's LDS copy of the rows, so nothing in the
// event loop waits on global memory.  HBM traffic is one read and one write
// of the state per interval.  Walkers are laid out bin-major, so neighbouring
// lanes have similar total propensity and the wave diverges little.
#include "ssa_lane_body.h"

#include <algorithm>

// Resident blocks per CU of the persistent grid, at most.
#ifndef LANE_POOL_PER_CU
#define LANE_POOL_PER_CU 5
#endif
// Idle lanes refill once at least this many of the wave's lanes are idle.
#ifndef LANE_REFILL_MIN
#define LANE_REFILL_MIN 12
#endif

// Persistent lane kernel: every lane runs walkers from the work queue (see
// work_queue.hip) until it is empty; the wave takes as many queue entries as
// it has idle lanes with one atomic and hands them out in lane order.  Walkers
// differ a lot in how many events one interval takes (the total propensity
// grows steeply along the progress coordinate), so a fixed walker-per-lane
// assignment would leave most lanes of a wave idle while its slowest walker
// finishes.
template <int SMAX, int RMAX, bool HILL, bool LEAP>
__device__ __forceinline__ void lane_pool(const SimArgs &a, int32_t *__restrict__ xs, int32_t *wrows) {
    constexpr bool REG = RMAX <= LANE_REG_RMAX;
    if constexpr (!REG) lane_stage_rows<SMAX>(a, wrows);
    LaneNet<SMAX, RMAX, HILL> net;
    net.load(a, wrows);
    uint32_t hor[LEAP ? SMAX : 1], hnu[LEAP ? SMAX : 1];
    if constexpr (LEAP) leap_orders(net, hor, hnu);
    LeapRng lr;
    lr.reset();
    const int lane = threadIdx.x & 63;
    const uint32_t iter = *a.iter_dev;
    const double tau = a.tau;
    const uint32_t M = (uint32_t)a.m_targ;
    const uint32_t total = a.queue[1] * M;
    const unsigned long long below = lane ? ((1ull << lane) - 1ull) : 0ull;
    LaneWalker w;
    int32_t x[SMAX];
    w.bad = false;
    bool active = false, exhausted = false;
    size_t gslot = 0;
    int32_t *xr = xs;
    for (;;) {
        const unsigned long long need = __ballot(!active);
        const int nneed = __popcll(need);
        if (!exhausted && (nneed >= LANE_REFILL_MIN || nneed == 64)) {
            // every lane executes the atomic (only the leader adds), so no
            // lane takes a path of its own around the wave-wide steps
            const int leader = __ffsll((long long)need) - 1;
            const uint32_t got = atomicAdd(&a.queue[0], lane == leader ? (uint32_t)nneed : 0u);
            const uint32_t base = (uint32_t)__shfl((int)got, leader, 64);
            if ((uint64_t)base + (uint64_t)nneed >= total) exhausted = true;
            if (!active) {
                const uint32_t q = base + (uint32_t)__popcll(need & below);
                if (q < total) {
                    const uint32_t sg = q / M, o = q - sg * M;
                    const int2 seg = a.seg[sg];
                    if ((int32_t)o < seg.y) {
                        const uint32_t g = (uint32_t)seg.x + o;   // below 2^30
                        const uint32_t run = g / (uint32_t)a.cap;
                        const uint32_t k = g - run * (uint32_t)a.cap;
                        gslot = g;
                        xr = xs + gslot * a.S;
                        w.begin(x, xr, a.S, k, a.seeds[run], iter);
                        if constexpr (LEAP) lr.reset();
                        active = true;
                    }
                }
            }
        }
        if (!__ballot(active) && exhausted) break;
        if constexpr (LEAP) {
            if (active && !lane_leap_step(net, w, lr, x, hor, hnu, iter, tau, a.leap_eps)) {
                lane_finish(a, w, x, xr, gslot);
                active = false;
            }
        } else {
            if (active && !lane_event(net, w, x, iter, tau)) {
                lane_finish(a, w, x, xr, gslot);
                active = false;
            }
        }
    }
}

template <int SMAX, int RMAX>
__global__ __launch_bounds__(256) void ssa_lane_pool_kernel(SimArgs a, int32_t *__restrict__ xs) {
    constexpr int ROWS = RMAX <= LANE_REG_RMAX ? 1 : RMAX * LaneRow<SMAX>::W;
    __shared__ int32_t rows[4 * ROWS];
    lane_pool<SMAX, RMAX, false, false>(a, xs, rows + (threadIdx.x >> 6) * ROWS);
}

// The same for networks with Hill-type rates (Sec. III.C).
template <int SMAX, int RMAX>
__global__ __launch_bounds__(256) void ssa_lane_hill_kernel(SimArgs a, int32_t *__restrict__ xs) {
    constexpr int ROWS = RMAX <= LANE_REG_RMAX ? 1 : RMAX * LaneRow<SMAX>::W;
    __shared__ int32_t rows[4 * ROWS];
    lane_pool<SMAX, RMAX, true, false>(a, xs, rows + (threadIdx.x >> 6) * ROWS);
}

// The same with tau-leaping instead of the exact direct method.
template <int SMAX, int RMAX>
__global__ __launch_bounds__(256) void ssa_lane_leap_kernel(SimArgs a, int32_t *__restrict__ xs) {
    constexpr int ROWS = RMAX <= LANE_REG_RMAX ? 1 : RMAX * LaneRow<SMAX>::W;
    __shared__ int32_t rows[4 * ROWS];
    lane_pool<SMAX, RMAX, false, true>(a, xs, rows + (threadIdx.x >> 6) * ROWS);
}

// Fixed assignment, one walker per lane: used for the two largest variants,
// whose register footprint leaves no room for the queue state.
template <int SMAX, int RMAX>
__global__ __launch_bounds__(256) void ssa_lane_kernel(SimArgs a, int32_t *__restrict__ xs) {
    constexpr bool REG = RMAX <= LANE_REG_RMAX;
    constexpr int ROWS = REG ? 1 : RMAX * LaneRow<SMAX>::W;
    __shared__ int32_t rows[4 * ROWS];
    int32_t *wrows = rows + (threadIdx.x >> 6) * ROWS;
    if constexpr (!REG) lane_stage_rows<SMAX>(a, wrows);
    const int32_t gid = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    const int32_t run = gid / a.cap;
    const int32_t k = gid - run * a.cap;
    if (run >= a.n_runs) return;
    if (k >= a.n_walk[run]) return;
    lane_walker<SMAX, RMAX>(a, xs, run, k, *a.iter_dev, wrows);
}


namespace {
// Persistent grid: as many blocks as stay resident on the device, capped at
// LANE_POOL_PER_CU per CU.
template <int SMAX, int RMAX, int VARIANT>   // 0: exact, 1: Hill-type rates, 2: tau-leaping
unsigned pool_blocks(const SimArgs &a) {
    static int per_cu = -1, n_cu = 0;   // one cache per kernel
    void (*kernel)(SimArgs, int32_t *);
    if constexpr (VARIANT == 1) kernel = ssa_lane_hill_kernel<SMAX, RMAX>;
    else if constexpr (VARIANT == 2) kernel = ssa_lane_leap_kernel<SMAX, RMAX>;
    else kernel = ssa_lane_pool_kernel<SMAX, RMAX>;
    if (per_cu < 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess || per_cu < 1) {
            per_cu = 1;
            n_cu = std::max(n_cu, 1);
        }
        // More resident blocks are not faster: on Schloegl at 2048 x 60 x 8
        // walkers, when <1,4> could hold 7 per CU, a launch took 1.188 ms at 5
        // per CU against 1.215 at 4, 1.268 at 3, 1.243 at 6 and 1.230 at 7.
        if (per_cu > LANE_POOL_PER_CU) per_cu = LANE_POOL_PER_CU;
    }
    const int64_t need = ((int64_t)a.n_runs * a.cap + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)per_cu * n_cu));
}

template <int SMAX, int RMAX>
hipError_t launch_fixed(const SimArgs &a, int32_t *xs, hipStream_t st) {
    const int64_t total = (int64_t)a.n_runs * a.cap;
    hipLaunchKernelGGL((ssa_lane_kernel<SMAX, RMAX>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a,
                       xs);
    return hipGetLastError();
}

template <int SMAX, int RMAX>
hipError_t launch_pool(const SimArgs &a, int32_t *xs, hipStream_t st) {
    hipLaunchKernelGGL((ssa_lane_pool_kernel<SMAX, RMAX>), dim3(pool_blocks<SMAX, RMAX, 0>(a)),
                       dim3(256), 0, st, a, xs);
    return hipGetLastError();
}

template <int SMAX, int RMAX>
hipError_t launch_hill(const SimArgs &a, int32_t *xs, hipStream_t st) {
    hipLaunchKernelGGL((ssa_lane_hill_kernel<SMAX, RMAX>), dim3(pool_blocks<SMAX, RMAX, 1>(a)),
                       dim3(256), 0, st, a, xs);
    return hipGetLastError();
}
template <int SMAX, int RMAX>
hipError_t launch_leap(const SimArgs &a, int32_t *xs, hipStream_t st) {
    hipLaunchKernelGGL((ssa_lane_leap_kernel<SMAX, RMAX>), dim3(pool_blocks<SMAX, RMAX, 2>(a)),
                       dim3(256), 0, st, a, xs);
    return hipGetLastError();
}
}  // namespace

// Launch helper: picks the smallest register footprint that holds the
// network.  The queue variants need the queue built by launch_work_queue.
hipError_t launch_ssa_lane(const SimArgs &a, int32_t *xs, hipStream_t st) {
    if (a.engine == 1) {
        if (a.hill) return hipErrorInvalidValue;
        if (a.S <= 1 && a.R <= 4) return launch_leap<1, 4>(a, xs, st);
        if (a.S <= 2 && a.R <= 8) return launch_leap<2, 8>(a, xs, st);
        if (a.S <= 8 && a.R <= 16) return launch_leap<8, 16>(a, xs, st);
        return hipErrorInvalidValue;
    }
    if (a.hill) {
        if (a.S <= 2 && a.R <= 8) return launch_hill<2, 8>(a, xs, st);
        if (a.S <= 8 && a.R <= 16) return launch_hill<8, 16>(a, xs, st);
        return hipErrorInvalidValue;
    }
    if (a.S <= 1 && a.R <= 4) return launch_pool<1, 4>(a, xs, st);
    if (a.S <= 2 && a.R <= 8) return launch_pool<2, 8>(a, xs, st);
    if (a.S <= 8 && a.R <= 16) return launch_pool<8, 16>(a, xs, st);
    if (a.S <= 16 && a.R <= 32) return launch_fixed<16, 32>(a, xs, st);
    if (a.S <= 32 && a.R <= 64) return launch_fixed<32, 64>(a, xs, st);
    return hipErrorInvalidValue;
}

// The name of the kernel launch_ssa_lane runs for these arguments.
const char *ssa_lane_name(const SimArgs &a) {
    if (a.engine == 1)
        return a.S <= 1 && a.R <= 4 ? "ssa_lane_leap_kernel<1,4>"
               : a.S <= 2 && a.R <= 8 ? "ssa_lane_leap_kernel<2,8>" : "ssa_lane_leap_kernel<8,16>";
    if (a.hill) return a.S <= 2 && a.R <= 8 ? "ssa_lane_hill_kernel<2,8>" : "ssa_lane_hill_kernel<8,16>";
    if (a.S <= 1 && a.R <= 4) return "ssa_lane_pool_kernel<1,4>";
    if (a.S <= 2 && a.R <= 8) return "ssa_lane_pool_kernel<2,8>";
    if (a.S <= 8 && a.R <= 16) return "ssa_lane_pool_kernel<8,16>";
    if (a.S <= 16 && a.R <= 32) return "ssa_lane_kernel<16,32>";
    return "ssa_lane_kernel<32,64>";
}

// Deltas travel as int8, so every change must lie in [-128, 127].
bool lane_kernel_fits(int32_t S, int32_t R, int32_t max_delta) {
    return S <= 32 && R <= 64 && max_delta <= 127;
}
