// we_resample.hip -- the WE bookkeeping between two propagation steps:
// recycling, binning, per-bin split/merge and the observables (gfx950).
//
// One workgroup per run (runs are independent, Sec. II.B).  Per iteration:
//   A. recycling (Sec. II.B.2): a walker whose state is in
//      B = { x : sum_s coef_s x_s >= thr } adds its weight to the run's flux
//      and restarts from the state A, keeping its weight; checked once, at
//      the end of the interval;
//   B. bin of every walker on the progress coordinate;
//   C. per-bin split/merge (Sec. II.B):
//        n == M: unchanged;
//        n <  M: replicate to M copies; one more copy is given, repeatedly,
//                to the parent with the largest per-copy weight w/c (ties:
//                lowest slot); each copy carries w/c, so the bin's weight is
//                conserved (a lone walker gets the paper's w/M exactly);
//        n >  M: merge the two lowest-weight walkers (ties: lowest slot): the
//                first survives with probability w_i/(w_i+w_j), else the
//                second, and the survivor carries w_i + w_j; repeat;
//      output layout: bins ascending, parents by ascending slot, copies of a
//      parent consecutive -- the "canonical" layout, which also keeps
//      walkers of similar state in neighbouring lanes for the next SSA step;
//   D. copy each new walker's state row from its parent.
// All weight arithmetic is sequential per bin, so the resulting weights are
// reproducible bit for bit.
#include "we_common.h"

__device__ __forceinline__ double coord_of(const double *__restrict__ coef,
                                           const int32_t *__restrict__ xr, int32_t S) {
    double q = 0.0;
    for (int32_t s = 0; s < S; ++s) q = q + coef[s] * (double)xr[s];
    return q;
}

__global__ __launch_bounds__(256) void we_resample_kernel(SimArgs a, int32_t *__restrict__ x_cur,
                                                          const double *__restrict__ w_cur,
                                                          int32_t *__restrict__ x_nxt,
                                                          double *__restrict__ w_nxt,
                                                          uint32_t iter, int32_t rec_slot) {
    extern __shared__ int32_t lds[];
    const int32_t run = blockIdx.x;
    const int32_t tid = threadIdx.x, nthr = blockDim.x;
    const int32_t S = a.S, NB = a.n_bins, M = a.m_targ, cap = a.cap;
    int32_t *cnt = lds;                // [NB]
    int32_t *start = cnt + NB;         // [NB+1]
    int32_t *ostart = start + NB + 1;  // [NB+1]
    __shared__ int64_t ev_part[256];

    const int32_t n = a.n_walk[run];
    const size_t base = (size_t)run * cap;
    int32_t *xr = x_cur + base * S;
    const double *wr = w_cur + base;
    int32_t *sbin = a.s_bin + base;
    int32_t *srec = a.s_rec + base;
    int32_t *slist = a.s_list + base;
    double *sw = a.s_w + base;
    int32_t *scnt = a.s_cnt + base;

    // A + B: recycling and bin of every walker
    int64_t my_ev = 0;
    for (int32_t k = tid; k < n; k += nthr) {
        int32_t *row = xr + (size_t)k * S;
        int32_t rec = 0;
        if (a.recycle) {
            if (coord_of(a.tgt_coef, row, S) >= a.tgt_thr) {
                rec = 1;
                for (int32_t s = 0; s < S; ++s) row[s] = a.x_rec[s];
            }
        }
        srec[k] = rec;
        sbin[k] = bin_index(a.edges, NB, coord_of(a.bin_coef, row, S));
        my_ev += a.ev_walker[base + k];
    }
    ev_part[tid] = my_ev;
    for (int32_t b = tid; b < NB; b += nthr) cnt[b] = 0;
    __syncthreads();

    // flux (sequential in slot order) and events (integer, any order)
    if (tid == 0) {
        double f = 0.0;
        for (int32_t k = 0; k < n; ++k)
            if (srec[k]) f = f + wr[k];
        int64_t ev = 0;
        for (int32_t t = 0; t < nthr; ++t) ev += ev_part[t];
        if (rec_slot >= 0) {
            a.flux[(size_t)run * a.max_iters + rec_slot] = f;
            a.ev_iter[(size_t)run * a.max_iters + rec_slot] = ev;
            a.seg_iter[(size_t)run * a.max_iters + rec_slot] = n;
        }
    }

    // C1: members of each bin, in slot order
    for (int32_t b = tid; b < NB; b += nthr) {
        int32_t c = 0;
        for (int32_t k = 0; k < n; ++k) c += (sbin[k] == b);
        cnt[b] = c;
    }
    __syncthreads();
    if (tid == 0) {
        int32_t acc = 0, oacc = 0;
        for (int32_t b = 0; b < NB; ++b) {
            start[b] = acc;
            ostart[b] = oacc;
            acc += cnt[b];
            oacc += (cnt[b] > 0) ? M : 0;
        }
        start[NB] = acc;
        ostart[NB] = oacc;
        if (oacc > cap) atomicOr(a.err, WE_DERR_CAPACITY);
    }
    __syncthreads();
    for (int32_t b = tid; b < NB; b += nthr) {
        int32_t p = start[b];
        for (int32_t k = 0; k < n; ++k)
            if (sbin[k] == b) {
                slist[p] = k;
                sw[p] = wr[k];
                ++p;
            }
    }
    __syncthreads();

    // C2: split / merge, one thread per bin
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
                orig[o] = slist[p0 + q];
                wn[o] = sw[p0 + q];
                obin[o] = b;
                ++o;
            }
        } else if (nb < M) {
            for (int32_t q = 0; q < nb; ++q) scnt[p0 + q] = 1;
            for (int32_t extra = nb; extra < M; ++extra) {
                int32_t best = 0;
                double best_share = sw[p0] / (double)scnt[p0];
                for (int32_t q = 1; q < nb; ++q) {
                    const double share = sw[p0 + q] / (double)scnt[p0 + q];
                    if (share > best_share) { best = q; best_share = share; }
                }
                scnt[p0 + best] += 1;
            }
            for (int32_t q = 0; q < nb; ++q) {
                const int32_t c = scnt[p0 + q];
                const double share = sw[p0 + q] / (double)c;
                for (int32_t r = 0; r < c; ++r) {
                    orig[o] = slist[p0 + q];
                    wn[o] = share;
                    obin[o] = b;
                    ++o;
                }
            }
        } else {
            for (int32_t q = 0; q < nb; ++q) scnt[p0 + q] = 1;   // alive flags
            int32_t alive = nb;
            uint32_t m = 0;
            while (alive > M) {
                int32_t i = -1, j = -1;
                for (int32_t q = 0; q < nb; ++q) {
                    if (!scnt[p0 + q]) continue;
                    const double v = sw[p0 + q];
                    if (i < 0 || v < sw[p0 + i]) { j = i; i = q; }
                    else if (j < 0 || v < sw[p0 + j]) { j = q; }
                }
                const U4 r = philox4x32_10(m, (uint32_t)b, iter, 1u, k0, k1);
                m += 1;
                const double u = uniform53(r.x, r.y);
                const double wi = sw[p0 + i], wj = sw[p0 + j];
                const double sum = wi + wj;
                const double p_i = wi / sum;
                const int32_t keep = (u < p_i) ? i : j;
                const int32_t drop = (keep == i) ? j : i;
                sw[p0 + keep] = sum;
                scnt[p0 + drop] = 0;
                alive -= 1;
            }
            for (int32_t q = 0; q < nb; ++q) {
                if (!scnt[p0 + q]) continue;
                orig[o] = slist[p0 + q];
                wn[o] = sw[p0 + q];
                obin[o] = b;
                ++o;
            }
        }
    }
    __syncthreads();

    // D: state rows of the new ensemble
    const int32_t n_out = ostart[NB];
    int32_t *xn = x_nxt + base * S;
    const int64_t total = (int64_t)n_out * S;
    for (int64_t idx = tid; idx < total; idx += nthr) {
        const int32_t dst = (int32_t)(idx / S);
        const int32_t s = (int32_t)(idx - (int64_t)dst * S);
        xn[idx] = xr[(size_t)orig[dst] * S + s];
    }
    if (tid == 0) a.n_walk[run] = n_out;
}

// P(x_s = k, t) accumulated over iterations: one lane per walker, FP64 atomics.
__global__ __launch_bounds__(256) void we_observe_kernel(SimArgs a, const int32_t *__restrict__ xs,
                                                         const double *__restrict__ ws) {
    const int32_t gid = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    const int32_t run = gid / a.cap;
    const int32_t k = gid - run * a.cap;
    if (run >= a.n_runs) return;
    if (k >= a.n_walk[run]) return;
    const size_t idx = (size_t)run * a.cap + k;
    const int32_t v = xs[idx * a.S + a.hist_species] - a.hist_lo;
    if (v >= 0 && v < a.nh) atomicAdd(&a.hist[(size_t)run * a.nh + v], ws[idx]);
}

hipError_t launch_resample(const SimArgs &a, int32_t *x_cur, const double *w_cur, int32_t *x_nxt,
                           double *w_nxt, uint32_t iter, int32_t rec_slot, hipStream_t st) {
    const size_t shmem = sizeof(int32_t) * (3 * (size_t)a.n_bins + 2);
    hipLaunchKernelGGL(we_resample_kernel, dim3(a.n_runs), dim3(256), shmem, st, a, x_cur, w_cur,
                       x_nxt, w_nxt, iter, rec_slot);
    return hipGetLastError();
}

hipError_t launch_observe(const SimArgs &a, const int32_t *xs, const double *ws, hipStream_t st) {
    const int64_t total = (int64_t)a.n_runs * a.cap;
    hipLaunchKernelGGL(we_observe_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       a, xs, ws);
    return hipGetLastError();
}
