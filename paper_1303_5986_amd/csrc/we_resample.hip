// we_resample.hip -- the WE bookkeeping between two propagation steps:
// recycling, binning, per-bin split/merge, the state gather and the
// observables (gfx950).  Per iteration, after the SSA kernel:
//
//   recycle_bin (one lane per walker, whole grid)
//      recycling (Sec. II.B.2): a walker whose state lies in
//      B = { x : sum_s coef_s x_s >= thr } is flagged and restarts from the
//      state A, keeping its weight; checked once, at the end of the interval
//      (the paper checks walkers only every tau);
//      bin of every walker on the progress coordinate (or, with learned
//      bins, the bin is written afterwards by the committor kernel);
//   resample (one workgroup per run)
//      the run's recycled weight (summed in slot order) and reactions fired;
//      per-bin split/merge (Sec. II.B):
//        n == M: unchanged;
//        n <  M: replicate to M copies; one more copy is given, repeatedly,
//                to the parent with the largest per-copy weight w/c (ties:
//                lowest slot); each copy carries w/c, so the bin's weight is
//                conserved (a lone walker gets the paper's w/M exactly);
//        n >  M: merge the two lowest-weight walkers (ties: lowest slot): the
//                first survives with probability w_i/(w_i+w_j), else the
//                second, and the survivor carries w_i + w_j; repeat;
//      output order: bins ascending, parents by ascending slot, copies of a
//      parent consecutive -- neighbouring lanes then hold walkers of similar
//      state for the next SSA step;
//      per-walker bin, weight and list arrays are staged in LDS;
//   gather_rows (one lane per count, whole grid): new state rows copied
//      from their parents;
//   observe: P(x_s = k, t) accumulated per run with FP64 atomics.
// All weight arithmetic is sequential per bin, so weights are reproducible
// bit for bit.
#include "we_common.h"

#define RESAMPLE_LDS_CAP 8192

__device__ __forceinline__ double coord_of(const double *__restrict__ coef,
                                           const int32_t *__restrict__ xr, int32_t S) {
    double q = 0.0;
    for (int32_t s = 0; s < S; ++s) q = q + coef[s] * (double)xr[s];
    return q;
}

__device__ __forceinline__ void recycle_bin_one(const SimArgs &a, int32_t *__restrict__ x_cur, int32_t grid_bins,
                                                int64_t gid) {
    const int32_t run = (int32_t)(gid / a.cap);
    const int32_t k = (int32_t)(gid - (int64_t)run * a.cap);
    if (run >= a.n_runs) return;
    if (k >= a.n_walk[run]) return;
    const int32_t S = a.S;
    const size_t idx = (size_t)run * a.cap + k;
    int32_t *row = x_cur + idx * S;
    int32_t rec = 0;
    if (a.recycle && coord_of(a.tgt_coef, row, S) >= a.tgt_thr) {
        rec = 1;
        for (int32_t s = 0; s < S; ++s) row[s] = a.x_rec[s];
    }
    a.s_rec[idx] = rec;
    if (grid_bins) a.s_bin[idx] = bin_index(a.edges, a.n_bins, coord_of(a.bin_coef, row, S));
}

__global__ __launch_bounds__(256) void we_recycle_bin_kernel(SimArgs a, int32_t *__restrict__ x_cur,
                                                             int32_t grid_bins) {
    recycle_bin_one(a, x_cur, grid_bins, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Per-walker working arrays of one run: LDS when the run fits, else global.
struct RunWork {
    double *w;          // weights in bin-major order
    int32_t *list;      // slots in bin-major order
    uint16_t *bin;      // bin of every slot
    uint16_t *cnt;      // copies / alive flags in bin-major order
};

__device__ __forceinline__ void resample_run(const SimArgs &a, const double *__restrict__ w_cur,
                                             double *__restrict__ w_nxt, int32_t use_lds, int32_t run,
                                             unsigned char *lds) {
    const int32_t tid = threadIdx.x, nthr = blockDim.x;
    const int32_t NB = a.n_bins, M = a.m_targ, cap = a.cap;
    __shared__ int64_t ev_part[256];
    int32_t *cnt = reinterpret_cast<int32_t *>(lds);   // [NB]
    int32_t *start = cnt + NB;                          // [NB+1]
    int32_t *ostart = start + NB + 1;                   // [NB+1]
    int32_t *cursor = ostart + NB + 1;                  // [NB]
    unsigned char *tail = reinterpret_cast<unsigned char *>(cursor + NB);
    tail += (16 - ((uintptr_t)tail & 15)) & 15;

    const uint32_t iter = *a.iter_dev;
    const int32_t rec_slot = (int32_t)iter;
    const int32_t n = a.n_walk[run];
    const size_t base = (size_t)run * cap;
    const double *wr = w_cur + base;
    const int32_t *sbin = a.s_bin + base;
    const int32_t *srec = a.s_rec + base;
    RunWork wk;
    if (use_lds) {
        wk.w = reinterpret_cast<double *>(tail);
        wk.list = reinterpret_cast<int32_t *>(wk.w + cap);
        wk.bin = reinterpret_cast<uint16_t *>(wk.list + cap);
        wk.cnt = wk.bin + cap;
    } else {
        wk.w = a.s_w + base;
        wk.list = a.s_list + base;
        wk.bin = reinterpret_cast<uint16_t *>(a.s_cnt + base);
        wk.cnt = wk.bin + cap;
    }

    for (int32_t b = tid; b < NB; b += nthr) cnt[b] = 0;
    __syncthreads();
    int64_t my_ev = 0;
    for (int32_t k = tid; k < n; k += nthr) {
        const int32_t b = sbin[k];
        wk.bin[k] = (uint16_t)b;
        atomicAdd(&cnt[b], 1);
        my_ev += a.ev_walker[base + k];
    }
    ev_part[tid] = my_ev;
    __syncthreads();

    // recycled weight (slot order), reactions fired, bin offsets
    if (tid == 0) {
        double f = 0.0;
        for (int32_t k = 0; k < n; ++k)
            if (srec[k]) f = f + wr[k];
        int64_t ev = 0;
        for (int32_t t = 0; t < nthr; ++t) ev += ev_part[t];
        if (rec_slot < a.max_iters) {
            a.flux[(size_t)run * a.max_iters + rec_slot] = f;
            a.ev_iter[(size_t)run * a.max_iters + rec_slot] = ev;
            a.seg_iter[(size_t)run * a.max_iters + rec_slot] = n;
        }
        int32_t acc = 0, oacc = 0;
        for (int32_t b = 0; b < NB; ++b) {
            start[b] = acc;
            cursor[b] = acc;
            ostart[b] = oacc;
            acc += cnt[b];
            oacc += (cnt[b] > 0) ? M : 0;
        }
        start[NB] = acc;
        ostart[NB] = oacc;
    }
    __syncthreads();

    // stable placement of every walker into its bin's segment (slot order
    // kept): one wave walks the slots 64 at a time; lanes with the same bin
    // are ranked by a ballot, and the bin's cursor advances by the group size
    if (tid < 64) {
        const int lane = tid;
        for (int32_t c0 = 0; c0 < n; c0 += 64) {
            const int32_t k = c0 + lane;
            const bool valid = k < n;
            const int32_t b = valid ? (int32_t)wk.bin[k] : -1;
            unsigned long long todo = __ballot(valid);
            while (todo) {
                const int leader = __ffsll((long long)todo) - 1;
                const int32_t lb = __shfl(b, leader, 64);
                const unsigned long long grp = __ballot(valid && b == lb);
                if (valid && b == lb) {
                    const unsigned long long below = lane ? (grp & ((1ull << lane) - 1ull)) : 0ull;
                    const int32_t p = cursor[lb] + __popcll(below);
                    wk.list[p] = k;
                    wk.w[p] = wr[k];
                }
                __builtin_amdgcn_wave_barrier();
                if (lane == leader) cursor[lb] += __popcll(grp);
                __builtin_amdgcn_wave_barrier();
                todo &= ~grp;
            }
        }
    }
    __syncthreads();

    // split / merge, one thread per bin
    const uint64_t seed = a.seeds[run];
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    int32_t *orig = a.origin + base;
    int32_t *obin = a.bin + base;
    double *wn = w_nxt + base;
    for (int32_t b = tid; b < NB; b += nthr) {
        const int32_t nb = cnt[b], p0 = start[b];
        int32_t o = ostart[b];
        if (nb == 0) continue;
        if (nb == M) {
            for (int32_t q = 0; q < nb; ++q) {
                orig[o] = wk.list[p0 + q];
                wn[o] = wk.w[p0 + q];
                obin[o] = b;
                ++o;
            }
        } else if (nb < M) {
            for (int32_t q = 0; q < nb; ++q) wk.cnt[p0 + q] = 1;
            for (int32_t extra = nb; extra < M; ++extra) {
                int32_t best = 0;
                double best_share = wk.w[p0] / (double)wk.cnt[p0];
                for (int32_t q = 1; q < nb; ++q) {
                    const double share = wk.w[p0 + q] / (double)wk.cnt[p0 + q];
                    if (share > best_share) { best = q; best_share = share; }
                }
                wk.cnt[p0 + best] += 1;
            }
            for (int32_t q = 0; q < nb; ++q) {
                const int32_t c = wk.cnt[p0 + q];
                const double share = wk.w[p0 + q] / (double)c;
                for (int32_t r = 0; r < c; ++r) {
                    orig[o] = wk.list[p0 + q];
                    wn[o] = share;
                    obin[o] = b;
                    ++o;
                }
            }
        } else {
            for (int32_t q = 0; q < nb; ++q) wk.cnt[p0 + q] = 1;   // alive flags
            int32_t alive = nb;
            uint32_t m = 0;
            while (alive > M) {
                int32_t i = -1, j = -1;
                double wi_min = 0.0, wj_min = 0.0;
                for (int32_t q = 0; q < nb; ++q) {
                    if (!wk.cnt[p0 + q]) continue;
                    const double v = wk.w[p0 + q];
                    if (i < 0 || v < wi_min) { j = i; wj_min = wi_min; i = q; wi_min = v; }
                    else if (j < 0 || v < wj_min) { j = q; wj_min = v; }
                }
                const U4 r = philox4x32_10(m, (uint32_t)b, iter, 1u, k0, k1);
                m += 1;
                const double u = uniform53(r.x, r.y);
                const double sum = wi_min + wj_min;
                const double p_i = wi_min / sum;
                const int32_t keep = (u < p_i) ? i : j;
                const int32_t drop = (keep == i) ? j : i;
                wk.w[p0 + keep] = sum;
                wk.cnt[p0 + drop] = 0;
                alive -= 1;
            }
            for (int32_t q = 0; q < nb; ++q) {
                if (!wk.cnt[p0 + q]) continue;
                orig[o] = wk.list[p0 + q];
                wn[o] = wk.w[p0 + q];
                obin[o] = b;
                ++o;
            }
        }
    }
    __syncthreads();
    if (tid == 0) a.n_walk[run] = ostart[NB];
}

__global__ __launch_bounds__(256) void we_resample_kernel(SimArgs a, const double *__restrict__ w_cur,
                                                          double *__restrict__ w_nxt, int32_t use_lds) {
    extern __shared__ __align__(16) unsigned char lds[];
    resample_run(a, w_cur, w_nxt, use_lds, blockIdx.x, lds);
}

// New state rows from their parents: one lane per copy number.
__device__ __forceinline__ void gather_one(const SimArgs &a, const int32_t *__restrict__ x_cur,
                                           int32_t *__restrict__ x_nxt, int64_t gid) {
    const int64_t per_run = (int64_t)a.cap * a.S;
    const int32_t run = (int32_t)(gid / per_run);
    if (run >= a.n_runs) return;
    const int64_t rem = gid - (int64_t)run * per_run;
    const int32_t dst = (int32_t)(rem / a.S);
    const int32_t s = (int32_t)(rem - (int64_t)dst * a.S);
    if (dst >= a.n_walk[run]) return;
    const size_t base = (size_t)run * a.cap;
    const int32_t src = a.origin[base + dst];
    x_nxt[(base + dst) * a.S + s] = x_cur[(base + src) * a.S + s];
}

__global__ __launch_bounds__(256) void we_gather_rows_kernel(SimArgs a, const int32_t *__restrict__ x_cur,
                                                             int32_t *__restrict__ x_nxt) {
    gather_one(a, x_cur, x_nxt, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// P(x_s = k, t) accumulated over iterations: one lane per walker, FP64 atomics.
__device__ __forceinline__ void observe_one(const SimArgs &a, const int32_t *__restrict__ xs,
                                            const double *__restrict__ ws, int64_t gid64) {
    const int32_t gid = (int32_t)gid64;
    const int32_t run = gid / a.cap;
    const int32_t k = gid - run * a.cap;
    if (run >= a.n_runs) return;
    if (k >= a.n_walk[run]) return;
    const size_t idx = (size_t)run * a.cap + k;
    const double wv = ws[idx];
    if (a.nh > 0) {
        const int32_t v = xs[idx * a.S + a.hist_species] - a.hist_lo;
        if (v >= 0 && v < a.nh) atomicAdd(&a.hist[(size_t)run * a.nh + v], wv);
    }
    if (a.n_joint > 0) {
        int32_t cell = 0, mul = 1;
        for (int d = 0; d < a.n_joint; ++d) {
            const int32_t c = min(xs[idx * a.S + a.joint_species[d]] / a.joint_width, a.joint_bins - 1);
            cell += c * mul;
            mul *= a.joint_bins;
        }
        atomicAdd(&a.jhist[(size_t)run * a.jcells + cell], wv);
    }
}

__global__ __launch_bounds__(256) void we_observe_kernel(SimArgs a, const int32_t *__restrict__ xs,
                                                         const double *__restrict__ ws) {
    observe_one(a, xs, ws, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------- batched
// The same steps for many sims in one launch each: grid y = sim, per-sim
// arguments and buffer pointers read from device memory.
struct BatchPtrs {
    const SimArgs *args;
    int32_t *const *x_cur;
    int32_t *const *x_nxt;
    const double *const *w_cur;
    double *const *w_nxt;
    const int32_t *use_lds;
    const int32_t *grid_bins;
};

__global__ __launch_bounds__(256) void we_batch_recycle_bin_kernel(BatchPtrs b) {
    const int32_t i = blockIdx.y;
    recycle_bin_one(b.args[i], b.x_cur[i], b.grid_bins[i], (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(256) void we_batch_resample_kernel(BatchPtrs b) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int32_t i = blockIdx.y;
    const SimArgs &a = b.args[i];
    if ((int32_t)blockIdx.x >= a.n_runs) return;
    resample_run(a, b.w_cur[i], b.w_nxt[i], b.use_lds[i], blockIdx.x, lds);
}

__global__ __launch_bounds__(256) void we_batch_gather_kernel(BatchPtrs b) {
    const int32_t i = blockIdx.y;
    gather_one(b.args[i], b.x_cur[i], b.x_nxt[i], (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(256) void we_batch_observe_kernel(BatchPtrs b) {
    const int32_t i = blockIdx.y;
    const SimArgs &a = b.args[i];
    if (a.nh <= 0 && a.n_joint <= 0) return;
    observe_one(a, b.x_nxt[i], b.w_nxt[i], (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void we_batch_advance_kernel(BatchPtrs b, int32_t n) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) *b.args[i].iter_dev += 1u;
}

hipError_t launch_batch_bookkeeping(const BatchPtrs &b, int32_t n_sims, int64_t max_slots, int32_t max_runs,
                                    int64_t max_cells, size_t shmem, bool observe, hipStream_t st) {
    const unsigned gs = (unsigned)((max_slots + 255) / 256);
    hipLaunchKernelGGL(we_batch_recycle_bin_kernel, dim3(gs, n_sims), dim3(256), 0, st, b);
    hipLaunchKernelGGL(we_batch_resample_kernel, dim3(max_runs, n_sims), dim3(256), shmem, st, b);
    hipLaunchKernelGGL(we_batch_gather_kernel, dim3((unsigned)((max_cells + 255) / 256), n_sims), dim3(256), 0, st, b);
    if (observe) hipLaunchKernelGGL(we_batch_observe_kernel, dim3(gs, n_sims), dim3(256), 0, st, b);
    hipLaunchKernelGGL(we_batch_advance_kernel, dim3((n_sims + 63) / 64), dim3(64), 0, st, b, n_sims);
    return hipGetLastError();
}

hipError_t launch_recycle_bin(const SimArgs &a, int32_t *x_cur, bool grid_bins, hipStream_t st) {
    const int64_t total = (int64_t)a.n_runs * a.cap;
    hipLaunchKernelGGL(we_recycle_bin_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       a, x_cur, grid_bins ? 1 : 0);
    return hipGetLastError();
}

bool resample_uses_lds(const SimArgs &a);
size_t resample_lds_bytes(const SimArgs &a, bool use_lds) {
    size_t b = sizeof(int32_t) * (4 * (size_t)a.n_bins + 2) + 16;
    if (use_lds) b += (size_t)a.cap * (sizeof(double) + sizeof(int32_t) + 2 * sizeof(uint16_t));
    return b;
}

bool resample_uses_lds(const SimArgs &a) {
    return a.cap <= RESAMPLE_LDS_CAP && resample_lds_bytes(a, true) <= 150 * 1024;
}

hipError_t launch_resample(const SimArgs &a, int32_t *x_cur, const double *w_cur, int32_t *x_nxt,
                           double *w_nxt, hipStream_t st) {
    const bool use_lds = resample_uses_lds(a);
    const size_t shmem = resample_lds_bytes(a, use_lds);
    hipLaunchKernelGGL(we_resample_kernel, dim3(a.n_runs), dim3(256), shmem, st, a, w_cur, w_nxt,
                       use_lds ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t total = (int64_t)a.n_runs * a.cap * a.S;
    hipLaunchKernelGGL(we_gather_rows_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       a, x_cur, x_nxt);
    return hipGetLastError();
}

hipError_t launch_observe(const SimArgs &a, const int32_t *xs, const double *ws, hipStream_t st) {
    const int64_t total = (int64_t)a.n_runs * a.cap;
    hipLaunchKernelGGL(we_observe_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       a, xs, ws);
    return hipGetLastError();
}

// End of an iteration: advance the device-side iteration counter.
__global__ void we_advance_kernel(SimArgs a) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *a.iter_dev += 1u;
}

hipError_t launch_advance(const SimArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(we_advance_kernel, dim3(1), dim3(64), 0, st, a);
    return hipGetLastError();
}
