// work_queue.hip -- the walker work queue of the persistent propagation
// kernels (gfx950).
//
// Before each propagation step three small kernels (one, for few runs) list
// the walkers as segments of up to m_targ consecutive slots (one occupied
// bin after resampling) and order the segments by the mean events per walker
// seen in their bin during the last interval, busiest first -- longest-
// processing-time-first scheduling, so the long walkers start early and the
// short ones fill the tail.  The propagation kernels then take walkers from the front
// of the queue with one atomic per request.  The order is a scheduling hint
// only: every result depends on (seed, iteration, slot, event), never on
// which lane or wave runs a walker.
#include "we_common.h"

// Segments per bin: one thread per (run, segment).
__global__ __launch_bounds__(256) void queue_count_kernel(SimArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t run = (int32_t)(gid / a.n_bins), j = (int32_t)(gid - (int64_t)run * a.n_bins);
    if (run >= a.n_runs) return;
    const int64_t first = (int64_t)j * a.m_targ;
    if (first >= a.n_walk[run]) return;
    const int32_t b = min(max(a.bin[(size_t)run * a.cap + first], 0), a.n_bins - 1);
    atomicAdd(&a.occ_bin[b * a.seg_rep + run % a.seg_rep], 1);
}

// Bitonic sort of 64 (key, bin) pairs held one per lane, descending by key
// and, for equal keys, by bin: the comparator of the block sort below, with
// shuffles in place of LDS and barriers.
__device__ __forceinline__ void wave_sort_desc(float &key, int32_t &idx, int lane) {
    for (int size = 2; size <= 64; size <<= 1)
        for (int d = size >> 1; d > 0; d >>= 1) {
            const float ko = __shfl_xor(key, d, 64);
            const int32_t io = __shfl_xor(idx, d, 64);
            const bool lower = (lane & d) == 0;
            const float ki = lower ? key : ko, kj = lower ? ko : key;
            const int32_t bi = lower ? idx : io, bj = lower ? io : idx;
            const bool i_first = ki > kj || (ki == kj && bi > bj);
            const bool desc = (lane & size) == 0;
            if (i_first != desc) {
                key = ko;
                idx = io;
            }
        }
}

// Bin order and queue offsets: one block.  Sorts the bins by mean events
// per walker (descending; ties: higher bin first), lays out their segments
// in that order, and clears the statistics and the queue.  SMALL (few runs,
// queue_small below): the same block first counts the segments into LDS
// and afterwards lists them itself, so the three steps are one launch.
#define QUEUE_MAX_BINS 8192
#define QUEUE_CHUNK 16   // counters per thread: NB * seg_rep <= 16384 over 1024 threads
#define QUEUE_SMALL_SEGS 4096
#define QUEUE_SMALL_BINS 1024
template <bool SMALL>
__global__ __launch_bounds__(1024) void queue_order_kernel(SimArgs a) {
    constexpr int32_t KB = SMALL ? QUEUE_SMALL_BINS : QUEUE_MAX_BINS;
    __shared__ float key[KB];
    __shared__ int16_t idx[KB];
    __shared__ int32_t part[1024];
    // SMALL only: per counter, segments / first position / fill cursor, and
    // each (run, segment)'s bin (-1: no walkers)
    __shared__ int32_t s_occ[SMALL ? QUEUE_SMALL_BINS : 1];
    __shared__ int32_t s_off[SMALL ? QUEUE_SMALL_BINS : 1];
    __shared__ int32_t s_cur[SMALL ? QUEUE_SMALL_BINS : 1];
    __shared__ int16_t s_bin[SMALL ? QUEUE_SMALL_SEGS : 1];
    const int32_t NB = a.n_bins, tid = threadIdx.x, nthr = blockDim.x;
    int32_t P = 1;
    while (P < NB) P <<= 1;
    const int32_t rep = a.seg_rep, NC = NB * rep;
    const int lane = tid & 63, wv = tid >> 6, nwv = nthr >> 6;
    const int32_t n_seg = a.n_runs * NB;
    if constexpr (SMALL) {
        for (int32_t c = tid; c < NC; c += nthr) {
            s_occ[c] = 0;
            s_cur[c] = 0;
        }
        __syncthreads();
        for (int32_t sg = tid; sg < n_seg; sg += nthr) {
            const int32_t run = sg / NB, j = sg - run * NB;
            const int64_t first = (int64_t)j * a.m_targ;
            int32_t b = -1;
            if (first < a.n_walk[run]) {
                b = min(max(a.bin[(size_t)run * a.cap + first], 0), NB - 1);
                atomicAdd(&s_occ[b * rep + run % rep], 1);
            }
            s_bin[sg] = (int16_t)b;
        }
    }
    // key of each bin: its replicas' event and walker counts summed by one
    // wave (rep <= 128: two entries per lane at most); four bins per wave at
    // a time, so that their loads are in flight together
    for (int32_t b0 = wv; b0 < P; b0 += 4 * nwv) {
        float ev[4];
        int32_t nw[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int32_t b = b0 + u * nwv;
            ev[u] = 0.0f;
            nw[u] = 0;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int32_t r = lane + 64 * q;
                if (b < NB && r < rep) {
                    ev[u] += a.ev_bin[b * rep + r];
                    nw[u] += a.n_bin[b * rep + r];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            for (int d = 32; d > 0; d >>= 1) {
                ev[u] += __shfl_xor(ev[u], d, 64);
                nw[u] += __shfl_xor(nw[u], d, 64);
            }
            const int32_t b = b0 + u * nwv;
            if (lane == 0 && b < P) {
                key[b] = b < NB ? (nw[u] > 0 ? ev[u] / (float)nw[u] : 0.0f) : -1.0f;
                idx[b] = (int16_t)b;
            }
        }
    }
    __syncthreads();
    if (P <= 64) {
        // at most 64 keys: wave 0 sorts them in registers (slots past P hold
        // a key below every real and padding key, so they sort last)
        if (wv == 0) {
            float k = lane < P ? key[lane] : -2.0f;
            int32_t b = lane < P ? (int32_t)idx[lane] : 64 + lane;
            wave_sort_desc(k, b, lane);
            if (lane < P) {
                key[lane] = k;
                idx[lane] = (int16_t)b;
            }
        }
        __syncthreads();
    } else {
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
    }
    // exclusive prefix of the segment counters in sorted bin order (the
    // replicas of a bin consecutive): per-thread chunks of that sequence,
    // at most QUEUE_CHUNK long (NB * rep <= 16384), held in registers
    const int32_t per = (NC + nthr - 1) / nthr;
    const int32_t lo = min(tid * per, NC), hi = min(lo + per, NC);
    auto counter = [&](int32_t i) { return (int32_t)idx[i / rep] * rep + i % rep; };
    int32_t cnt[QUEUE_CHUNK];
    int32_t acc = 0;
#pragma unroll
    for (int q = 0; q < QUEUE_CHUNK; ++q) {
        cnt[q] = lo + q < hi ? (SMALL ? s_occ[counter(lo + q)] : a.occ_bin[counter(lo + q)]) : 0;
        acc += cnt[q];
    }
    // block-wide exclusive scan of the chunk sums: within waves, then over
    // the wave totals
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
#pragma unroll
    for (int q = 0; q < QUEUE_CHUNK; ++q)
        if (lo + q < hi) {
            if (SMALL)
                s_off[counter(lo + q)] = acc;
            else
                a.seg_off[counter(lo + q)] = acc;
            acc += cnt[q];
        }
    __syncthreads();
    if constexpr (SMALL) {
        // the segment list, as queue_fill_kernel lays it out
        for (int32_t sg = tid; sg < n_seg; sg += nthr) {
            const int32_t b = s_bin[sg];
            if (b < 0) continue;
            const int32_t run = sg / NB, j = sg - run * NB;
            const int32_t n = a.n_walk[run];
            const int64_t first = (int64_t)j * a.m_targ;
            const int32_t c = b * rep + run % rep;
            const int32_t pos = s_off[c] + atomicAdd(&s_cur[c], 1);
            a.seg[pos] = make_int2((int32_t)((size_t)run * a.cap + first), (int32_t)min((int64_t)a.m_targ, n - first));
        }
    }
    for (int32_t c = tid; c < NC; c += nthr) {
        if (!SMALL) {
            a.occ_bin[c] = 0;
            a.seg_cur[c] = 0;
        }
        a.ev_bin[c] = 0.0f;
        a.n_bin[c] = 0;
    }
}

// Tiny case (queue_tiny: at most 64 segments and 64 counters, e.g. one run of
// up to 64 bins): the same three steps in one wave, with no block barrier
// in the sort -- lane b holds bin b's key, a bitonic sort over the 64 lanes
// by shuffles (the same comparator as above, padding keys -1 last), then a
// wave prefix over the counters in sorted order.  Gives the same segment
// order per counter as queue_order_kernel<true>.
__global__ __launch_bounds__(64) void queue_order_wave_kernel(SimArgs a) {
    __shared__ int32_t s_occ[64], s_off[64], s_cur[64];
    const int lane = threadIdx.x & 63;
    const int32_t NB = a.n_bins, rep = a.seg_rep, NC = NB * rep, n_seg = a.n_runs * NB;
    s_occ[lane] = 0;
    s_cur[lane] = 0;
    __syncthreads();
    // each segment's bin (lane = run * NB + segment)
    int32_t b = -1, run = 0, j = 0;
    if (lane < n_seg) {
        run = lane / NB;
        j = lane - run * NB;
        if ((int64_t)j * a.m_targ < a.n_walk[run]) {
            b = min(max(a.bin[(size_t)run * a.cap + (size_t)j * a.m_targ], 0), NB - 1);
            atomicAdd(&s_occ[b * rep + run % rep], 1);
        }
    }
    // bin keys: mean events per walker over the bin's replica counters
    float key = -1.0f;
    int32_t idx = lane;
    if (lane < NB) {
        float ev = 0.0f;
        int32_t nw = 0;
        for (int32_t r = 0; r < rep; ++r) {
            ev += a.ev_bin[lane * rep + r];
            nw += a.n_bin[lane * rep + r];
        }
        key = nw > 0 ? ev / (float)nw : 0.0f;
    }
    wave_sort_desc(key, idx, lane);
    __syncthreads();
    // exclusive prefix of the counters in sorted bin order (replicas of a
    // bin consecutive): lane i holds counter i of that sequence
    const int32_t bin_at = __shfl(idx, rep > 0 ? lane / rep : 0, 64);
    const int32_t c = bin_at * rep + lane % rep;
    const int32_t cnt = lane < NC ? s_occ[c] : 0;
    int32_t incl = cnt;
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
    }
    if (lane < NC) s_off[c] = incl - cnt;
    const int32_t total = __shfl(incl, 63, 64);
    if (lane == 0) {
        a.queue[0] = 0u;
        a.queue[1] = (uint32_t)total;
    }
    __syncthreads();
    // the segment list, as queue_fill_kernel lays it out
    if (b >= 0) {
        const int32_t n = a.n_walk[run];
        const int64_t first = (int64_t)j * a.m_targ;
        const int32_t cc = b * rep + run % rep;
        const int32_t pos = s_off[cc] + atomicAdd(&s_cur[cc], 1);
        a.seg[pos] = make_int2((int32_t)((size_t)run * a.cap + first), (int32_t)min((int64_t)a.m_targ, n - first));
    }
    if (lane < NC) {
        a.ev_bin[lane] = 0.0f;
        a.n_bin[lane] = 0;
    }
}

// Segment list: one thread per (run, segment), same grid as the count.
__global__ __launch_bounds__(256) void queue_fill_kernel(SimArgs a) {
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

// Few runs (at most QUEUE_SMALL_SEGS segments, QUEUE_SMALL_BINS counters):
// one block does all three steps; else three launches.
bool queue_small(const SimArgs &a) {
    return (int64_t)a.n_runs * a.n_bins <= QUEUE_SMALL_SEGS && a.n_bins <= QUEUE_SMALL_BINS &&
           (int64_t)a.n_bins * a.seg_rep <= QUEUE_SMALL_BINS;
}

// At most 64 segments and 64 counters: one wave does everything.
bool queue_tiny(const SimArgs &a) {
    return (int64_t)a.n_runs * a.n_bins <= 64 && a.n_bins <= 64 && (int64_t)a.n_bins * a.seg_rep <= 64;
}

hipError_t launch_work_queue(const SimArgs &a, hipStream_t st) {
    if (queue_tiny(a)) {
        hipLaunchKernelGGL(queue_order_wave_kernel, dim3(1), dim3(64), 0, st, a);
        return hipGetLastError();
    }
    if (queue_small(a)) {
        hipLaunchKernelGGL(queue_order_kernel<true>, dim3(1), dim3(1024), 0, st, a);
        return hipGetLastError();
    }
    const int64_t total = (int64_t)a.n_runs * a.n_bins;
    const unsigned g = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(queue_count_kernel, dim3(g), dim3(256), 0, st, a);
    hipLaunchKernelGGL(queue_order_kernel<false>, dim3(1), dim3(1024), 0, st, a);
    hipLaunchKernelGGL(queue_fill_kernel, dim3(g), dim3(256), 0, st, a);
    return hipGetLastError();
}
