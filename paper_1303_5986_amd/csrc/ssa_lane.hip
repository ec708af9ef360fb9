// ssa_lane.hip -- Gillespie direct-method SSA, one lane per walker (gfx950).
//
// Each lane carries one walker through one WE interval tau (Sec. II.A, the
// propagation step of the WE procedure in Sec. II.B):
//   1. all propensities a_j = c_j * prod_s C(x_s, nu_js) and their total a0,
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

// ------------------------------------------------------------ work queue
// Walkers differ a lot in how many events one interval takes (the total
// propensity grows steeply along the progress coordinate), so a fixed
// walker-per-lane assignment leaves most lanes of a wave idle while its
// slowest walker finishes.  The lanes instead pull walkers from a queue:
// segments of up to m_targ consecutive slots (one occupied bin after
// resampling), ordered by the mean events per walker seen in their bin in
// the last interval, busiest first -- longest-first scheduling.  The order
// is a hint only: every result depends on (seed, iteration, slot, event),
// never on which lane runs a walker.

// Segments per bin: one thread per (run, segment).
__global__ __launch_bounds__(256) void lane_seg_count_kernel(SimArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t run = (int32_t)(gid / a.n_bins), j = (int32_t)(gid - (int64_t)run * a.n_bins);
    if (run >= a.n_runs) return;
    const int64_t first = (int64_t)j * a.m_targ;
    if (first >= a.n_walk[run]) return;
    const int32_t b = min(max(a.bin[(size_t)run * a.cap + first], 0), a.n_bins - 1);
    atomicAdd(&a.occ_bin[b * a.seg_rep + run % a.seg_rep], 1);
}

// Bin order and queue offsets: one block.  Sorts the bins by mean events
// per walker (descending; ties: higher bin first), lays out their segments
// in that order, and clears the statistics and the queue.
#define LANE_SCHED_MAX 8192
__global__ __launch_bounds__(1024) void lane_seg_order_kernel(SimArgs a) {
    __shared__ float key[LANE_SCHED_MAX];
    __shared__ int16_t idx[LANE_SCHED_MAX];
    __shared__ int32_t part[1024];
    const int32_t NB = a.n_bins, tid = threadIdx.x, nthr = blockDim.x;
    int32_t P = 1;
    while (P < NB) P <<= 1;
    for (int32_t b = tid; b < P; b += nthr) {
        float kv = -1.0f;
        if (b < NB) {
            const int32_t nw = a.n_bin[b];
            kv = nw > 0 ? a.ev_bin[b] / (float)nw : 0.0f;
        }
        key[b] = kv;
        idx[b] = (int16_t)b;
    }
    __syncthreads();
    // bitonic sort, descending by (key, bin)
    for (int32_t size = 2; size <= P; size <<= 1)
        for (int32_t d = size >> 1; d > 0; d >>= 1) {
            for (int32_t i = tid; i < P; i += nthr) {
                const int32_t j = i ^ d;
                if (j > i) {
                    const bool desc = (i & size) == 0;
                    const float ki = key[i], kj = key[j];
                    const int32_t bi = idx[i], bj = idx[j];
                    const bool i_first = ki > kj || (ki == kj && bi > bj);
                    if (i_first != desc) {
                        key[i] = kj; key[j] = ki;
                        idx[i] = (int16_t)bj; idx[j] = (int16_t)bi;
                    }
                }
            }
            __syncthreads();
        }
    // exclusive prefix of the segment counters in sorted bin order (the
    // replicas of a bin consecutive): per-thread chunks of that sequence
    const int32_t rep = a.seg_rep, NC = NB * rep;
    const int32_t per = (NC + nthr - 1) / nthr;
    const int32_t lo = min(tid * per, NC), hi = min(lo + per, NC);
    auto counter = [&](int32_t i) { return (int32_t)idx[i / rep] * rep + i % rep; };
    int32_t acc = 0;
    for (int32_t i = lo; i < hi; ++i) acc += a.occ_bin[counter(i)];
    // block-wide exclusive scan of the chunk sums: within waves, then over
    // the wave totals
    const int lane = tid & 63, wv = tid >> 6;
    int32_t incl = acc;
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
    }
    if (lane == 63) part[wv] = incl;
    __syncthreads();
    if (tid == 0) {
        int32_t run = 0;
        for (int32_t t = 0; t < nthr / 64; ++t) {
            const int32_t v = part[t];
            part[t] = run;
            run += v;
        }
        a.queue[0] = 0u;
        a.queue[1] = (uint32_t)run;
    }
    __syncthreads();
    acc = part[wv] + incl - acc;
    for (int32_t i = lo; i < hi; ++i) {
        const int32_t c = counter(i);
        a.seg_off[c] = acc;
        acc += a.occ_bin[c];
    }
    __syncthreads();
    for (int32_t c = tid; c < NC; c += nthr) {
        a.occ_bin[c] = 0;
        a.seg_cur[c] = 0;
    }
    for (int32_t b = tid; b < NB; b += nthr) {
        a.ev_bin[b] = 0.0f;
        a.n_bin[b] = 0;
    }
}

// Segment list: one thread per (run, segment), same grid as the count.
__global__ __launch_bounds__(256) void lane_seg_fill_kernel(SimArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t run = (int32_t)(gid / a.n_bins), j = (int32_t)(gid - (int64_t)run * a.n_bins);
    if (run >= a.n_runs) return;
    const int32_t n = a.n_walk[run];
    const int64_t first = (int64_t)j * a.m_targ;
    if (first >= n) return;
    const size_t g = (size_t)run * a.cap + first;
    const int32_t b = min(max(a.bin[g], 0), a.n_bins - 1);
    const int32_t c = b * a.seg_rep + run % a.seg_rep;
    const int32_t pos = a.seg_off[c] + atomicAdd(&a.seg_cur[c], 1);
    a.seg[pos] = make_int2((int32_t)g, (int32_t)min((int64_t)a.m_targ, n - first));
}

// Idle lanes refill once at least this many of the wave's lanes are idle.
#ifndef LANE_REFILL_MIN
#define LANE_REFILL_MIN 4
#endif

// Persistent lane kernel: every lane runs walkers from the queue until it is
// empty; the wave takes as many queue entries as it has idle lanes with one
// atomic and hands them out in lane order.
template <int SMAX, int RMAX>
__global__ __launch_bounds__(256) void ssa_lane_pool_kernel(SimArgs a, int32_t *__restrict__ xs) {
    constexpr bool REG = RMAX <= LANE_REG_RMAX;
    constexpr int ROWS = REG ? 1 : RMAX * LaneRow<SMAX>::W;
    __shared__ int32_t rows[4 * ROWS];
    int32_t *wrows = rows + (threadIdx.x >> 6) * ROWS;
    if constexpr (!REG) lane_stage_rows<SMAX>(a, wrows);
    LaneNet<SMAX, RMAX> net;
    net.load(a, wrows);
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
            const int leader = __ffsll((long long)need) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(&a.queue[0], (uint32_t)nneed);
            base = __shfl(base, leader, 64);
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
                        w.begin(x, xr, a.S, k, a.seeds[run]);
                        active = true;
                    }
                }
            }
        }
        if (!__ballot(active)) {
            if (exhausted) break;
            continue;
        }
        if (active && !lane_event(net, w, x, iter, tau)) {
            lane_finish(a, w, x, xr, gslot);
            active = false;
        }
    }
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

hipError_t launch_lane_schedule(const SimArgs &a, hipStream_t st) {
    const int64_t total = (int64_t)a.n_runs * a.n_bins;
    const unsigned g = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(lane_seg_count_kernel, dim3(g), dim3(256), 0, st, a);
    hipLaunchKernelGGL(lane_seg_order_kernel, dim3(1), dim3(1024), 0, st, a);
    hipLaunchKernelGGL(lane_seg_fill_kernel, dim3(g), dim3(256), 0, st, a);
    return hipGetLastError();
}

namespace {
// Persistent grid: as many blocks as stay resident on the device.
template <int SMAX, int RMAX>
unsigned pool_blocks(const SimArgs &a) {
    static int per_cu = -1, n_cu = 0;
    if (per_cu < 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ssa_lane_pool_kernel<SMAX, RMAX>, 256, 0) !=
                hipSuccess || per_cu < 1) {
            per_cu = 1;
            n_cu = std::max(n_cu, 1);
        }
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
    hipLaunchKernelGGL((ssa_lane_pool_kernel<SMAX, RMAX>), dim3(pool_blocks<SMAX, RMAX>(a)), dim3(256), 0, st, a,
                       xs);
    return hipGetLastError();
}
}  // namespace

// Launch helper: picks the smallest register footprint that holds the
// network.  The queue variants need the queue built by launch_lane_schedule.
hipError_t launch_ssa_lane(const SimArgs &a, int32_t *xs, hipStream_t st) {
    if (a.S <= 1 && a.R <= 4) return launch_pool<1, 4>(a, xs, st);
    if (a.S <= 2 && a.R <= 8) return launch_pool<2, 8>(a, xs, st);
    if (a.S <= 8 && a.R <= 16) return launch_pool<8, 16>(a, xs, st);
    if (a.S <= 16 && a.R <= 32) return launch_fixed<16, 32>(a, xs, st);
    if (a.S <= 32 && a.R <= 64) return launch_fixed<32, 64>(a, xs, st);
    return hipErrorInvalidValue;
}

// Deltas travel as int8, so every change must lie in [-128, 127].
bool lane_kernel_fits(int32_t S, int32_t R, int32_t max_delta) {
    return S <= 32 && R <= 64 && max_delta <= 127;
}
