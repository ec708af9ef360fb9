// reweight.hip -- steady-state reweighting (Sec. II.B.2, Eq. ss), gfx950.
//
// One workgroup per run, launched after the resampling of every iteration;
// it returns at once unless (iteration + 1) is a multiple of the period.
// The flux matrix F[i][j] (weight moved from bin j into bin i, summed from
// the second interval on) is accumulated by the resampling kernel.
//
//   1. W_j = sum_i F[i][j] (ascending i), the weight that started intervals
//      in bin j; the current weight w_i of every bin (its walkers in slot
//      order; the resampled ensemble is bin-major).
//   2. Candidates: bins that are occupied, weigh more than zero and have
//      W_j > 0, in ascending order; the pivot is the one holding the most
//      weight (ties: the lowest bin).
//   3. The pivot's strongly connected component among the candidates, edge
//      j -> i where F[i][j] > 0: forward and backward reachability over
//      64-bit adjacency masks, run by one wave (OR-reductions, no barriers).
//   4. Eq. ss on the component, with rates r(a -> b) = F[b][a] / W_a, by
//      state reduction (Grassmann, Taksar and Heyman 1985): states are
//      removed from the highest index down, each time with
//          s_m = sum_{j<m} r(m -> j),  r(i -> j) += r(i -> m) r(m -> j) / s_m,
//      then pi_0 = 1, pi_m = sum_{i<m} pi_i r(i -> m) / s_m.  Every term is
//      non-negative, so there is no cancellation; on a strongly connected
//      set every s_m and pi_m is positive.
//   5. Bin a's walkers are scaled by (pi_a / Z * W_A) / w_a, Z = sum pi,
//      W_A the component's current weight, which it keeps; every other bin
//      is scaled by 1 (exactly unchanged).  Optionally F is cleared, so that
//      the next event sees only the intervals after this one.
// The rate matrix lives in LDS when it fits, else in a per-run global
// scratch.  Sums over lanes use fixed shuffle trees, so the result is
// deterministic (graph replays equal eager runs bit for bit).
#include "we_internal.h"

#define RW_THREADS 256
#define RW_LDS_LIMIT (128 * 1024)

namespace {

__host__ __device__ inline size_t rw_align8(size_t b) { return (b + 7) & ~(size_t)7; }

// Bytes of the small per-run tables: W, w, pi, s, factor (double), candidate
// and component lists and a bin -> candidate map (int32), the two adjacency
// bit matrices (uint64), 4 ints of scalars and the forward and backward
// reach masks (8 words each; n_bins <= 512).
#define RW_MISC_BYTES (16 + 2 * 8 * 8)
__host__ __device__ inline size_t rw_small_bytes(int32_t NB) {
    const size_t nw = (size_t)(NB + 63) / 64;
    return rw_align8(40 * (size_t)NB + 12 * (size_t)NB) + 16 * (size_t)NB * nw + RW_MISC_BYTES;
}

__device__ __forceinline__ double rw_wave_sum(double v) {
    for (int d = 32; d > 0; d >>= 1) v = v + __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ unsigned long long rw_wave_or(unsigned long long v) {
    for (int d = 32; d > 0; d >>= 1) v |= __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ void rw_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave 0: grows `reach` (nw words over candidate indices) along the rows of
// `adj` (adj[c * nw + word]: the candidates one step from c) until nothing
// changes.  Inlined, so that every access stays an LDS access: a generic
// pointer would turn them into flat accesses, which the wave-level sync does
// not order against the caller's LDS reads.
__device__ __forceinline__ void rw_reach(unsigned long long *reach, const unsigned long long *adj, int32_t nc, int32_t nw,
                         int lane) {
    for (;;) {
        unsigned long long acc[8];
#pragma unroll
        for (int w = 0; w < 8; ++w) acc[w] = 0ull;
        for (int32_t c = lane; c < nc; c += 64) {
            if ((reach[c >> 6] >> (c & 63)) & 1ull) {
#pragma unroll
                for (int w = 0; w < 8; ++w)
                    if (w < nw) acc[w] |= adj[(size_t)c * nw + w];
            }
        }
        int changed = 0;
#pragma unroll
        for (int w = 0; w < 8; ++w) {
            if (w < nw) {
                const unsigned long long r = reach[w];
                const unsigned long long nr = r | rw_wave_or(acc[w]);
                changed |= nr != r;
                rw_wave_sync();
                if (lane == 0) reach[w] = nr;
                rw_wave_sync();
            }
        }
        if (!changed) break;
    }
}

}  // namespace

// RL: the rate matrix in LDS (else in the run's global scratch); a template
// parameter so that the compiler knows the address space of every access.
template <bool RL>
__global__ __launch_bounds__(RW_THREADS) void we_reweight_kernel(SimArgs a, double *__restrict__ w_nxt) {
    extern __shared__ __align__(16) unsigned char lds[];
    const uint32_t iter = *a.iter_dev;
    if ((iter + 1u) % (uint32_t)a.rw_period != 0u) return;
    const int32_t run = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int32_t NB = a.n_bins, NW = (NB + 63) >> 6;
    const size_t base = (size_t)run * a.cap;
    const int32_t n = a.n_walk[run];
    const double *__restrict__ F = a.rw_F + (size_t)run * NB * NB;
    const int32_t *__restrict__ bins = a.bin + base;
    double *__restrict__ w = w_nxt + base;

    double *Wc = reinterpret_cast<double *>(lds);   // [NB]
    double *wb = Wc + NB;                             // [NB]
    double *pi = wb + NB;                             // [NB] over the component
    double *sm = pi + NB;                             // [NB] over the component
    double *fac = sm + NB;                            // [NB]
    int32_t *cand = reinterpret_cast<int32_t *>(fac + NB);  // [NB] candidate -> bin
    int32_t *act = cand + NB;                               // [NB] component -> bin
    int32_t *pos = act + NB;                                // [NB] per bin
    unsigned long long *succ =
        reinterpret_cast<unsigned long long *>(lds + rw_align8(40 * (size_t)NB + 12 * (size_t)NB));
    unsigned long long *pred = succ + (size_t)NB * NW;
    int32_t *misc = reinterpret_cast<int32_t *>(pred + (size_t)NB * NW);   // 4 ints
    unsigned long long *fw = reinterpret_cast<unsigned long long *>(misc + 4);   // 8 words
    unsigned long long *bw = fw + 8;                                              // 8 words
    double *R = RL ? reinterpret_cast<double *>(lds + rw_small_bytes(NB)) : a.rw_R + (size_t)run * NB * NB;

    // 1. W_j, and where each bin's walkers start (act doubles as that table)
    for (int32_t j = tid; j < NB; j += nthr) {
        double acc = 0.0;
        for (int32_t i = 0; i < NB; ++i) acc = acc + F[(size_t)i * NB + j];
        Wc[j] = acc;
        act[j] = -1;
        fac[j] = 1.0;
    }
    __syncthreads();
    for (int32_t k = tid; k < n; k += nthr)
        if (k == 0 || bins[k] != bins[k - 1]) act[bins[k]] = k;
    __syncthreads();
    for (int32_t i = tid; i < NB; i += nthr) {
        double acc = 0.0;
        int32_t c = 0;
        for (int32_t k = act[i]; k >= 0 && k < n && bins[k] == i; ++k) {
            acc = acc + w[k];
            ++c;
        }
        wb[i] = acc;
        pos[i] = c;
    }
    __syncthreads();

    // 2. candidates (ascending) and the pivot
    if (wave == 0) {
        int32_t nc = 0;
        for (int32_t c0 = 0; c0 < NB; c0 += 64) {
            const int32_t i = c0 + lane;
            const bool is = i < NB && pos[i] > 0 && wb[i] > 0.0 && Wc[i] > 0.0;
            const unsigned long long m = __ballot(is);
            const int32_t idx = nc + __popcll(m & ((1ull << lane) - 1ull));
            rw_wave_sync();
            if (i < NB) pos[i] = is ? idx : -1;
            if (is) cand[idx] = i;
            nc += __popcll(m);
        }
        double bv = -1.0;
        int32_t bc = INT32_MAX;
        for (int32_t c = lane; c < nc; c += 64) {
            const double v = wb[cand[c]];
            if (v > bv) { bv = v; bc = c; }
        }
        for (int d = 32; d > 0; d >>= 1) {
            const double ov = __shfl_xor(bv, d, 64);
            const int32_t oc = __shfl_xor(bc, d, 64);
            if (ov > bv || (ov == bv && oc < bc)) { bv = ov; bc = oc; }
        }
        if (lane == 0) {
            misc[0] = nc;
            misc[2] = bc;
            misc[3] = 0;
        }
    }
    __syncthreads();
    const int32_t nc = misc[0];
    bool ok = false;
    if (nc >= 2) {
        // 3. adjacency among the candidates, then the pivot's component
        for (size_t t = tid; t < (size_t)nc * NW; t += nthr) {
            succ[t] = 0ull;
            pred[t] = 0ull;
        }
        __syncthreads();
        for (size_t t = tid; t < (size_t)nc * nc; t += nthr) {
            const int32_t to = (int32_t)(t / nc), from = (int32_t)(t - (size_t)to * nc);
            if (to != from && F[(size_t)cand[to] * NB + cand[from]] > 0.0) {
                atomicOr(&succ[(size_t)from * NW + (to >> 6)], 1ull << (to & 63));
                atomicOr(&pred[(size_t)to * NW + (from >> 6)], 1ull << (from & 63));
            }
        }
        __syncthreads();
        if (wave == 0) {
            const int32_t pv = misc[2];
            for (int32_t q = lane; q < NW; q += 64) {
                fw[q] = q == (pv >> 6) ? 1ull << (pv & 63) : 0ull;
                bw[q] = fw[q];
            }
            rw_wave_sync();
            rw_reach(fw, succ, nc, NW, lane);
            rw_reach(bw, pred, nc, NW, lane);
            int32_t na = 0;
            for (int32_t c0 = 0; c0 < nc; c0 += 64) {
                const int32_t c = c0 + lane;
                const bool in = c < nc && ((fw[c >> 6] & bw[c >> 6]) >> (c & 63)) & 1ull;
                const unsigned long long m = __ballot(in);
                if (in) act[na + __popcll(m & ((1ull << lane) - 1ull))] = cand[c];
                na += __popcll(m);
            }
            if (lane == 0) misc[1] = na;
        }
        __syncthreads();
        const int32_t na = misc[1];
        if (na >= 2) {
            // 4. rates on the component, state reduction, back substitution
            for (size_t t = tid; t < (size_t)na * na; t += nthr) {
                const int32_t to = (int32_t)(t / na), from = (int32_t)(t - (size_t)to * na);
                R[(size_t)from * na + to] =
                    from == to ? 0.0 : F[(size_t)act[to] * NB + act[from]] / Wc[act[from]];
            }
            __syncthreads();
            for (int32_t m = na - 1; m >= 1; --m) {
                if (wave == 0) {
                    double p = 0.0;
                    for (int32_t j = lane; j < m; j += 64) p = p + R[(size_t)m * na + j];
                    const double s = rw_wave_sum(p);
                    if (s > 0.0)
                        for (int32_t j = lane; j < m; j += 64) R[(size_t)m * na + j] = R[(size_t)m * na + j] / s;
                    if (lane == 0) {
                        sm[m] = s;
                        if (!(s > 0.0)) misc[3] = 1;
                    }
                }
                __syncthreads();
                if (misc[3]) break;
                // one row per wave: rows with r(i -> m) = 0 are skipped whole
                // (the rates join neighbouring bins only, so most rows are, and
                // the elimination keeps that band); each entry gets the same
                // single update as before, so the result is unchanged
                const int32_t n_waves = nthr >> 6;
                for (int32_t i = wave; i < m; i += n_waves) {
                    const double rim = R[(size_t)i * na + m];
                    if (rim == 0.0) continue;
                    for (int32_t j = lane; j < m; j += 64)
                        if (j != i) R[(size_t)i * na + j] = R[(size_t)i * na + j] + rim * R[(size_t)m * na + j];
                }
                __syncthreads();
            }
            if (wave == 0 && !misc[3]) {
                if (lane == 0) pi[0] = 1.0;
                rw_wave_sync();
                bool pos_ok = true;
                for (int32_t m = 1; m < na; ++m) {
                    double p = 0.0;
                    for (int32_t i = lane; i < m; i += 64) p = p + pi[i] * R[(size_t)i * na + m];
                    const double v = rw_wave_sum(p) / sm[m];
                    pos_ok = pos_ok && v > 0.0;
                    if (lane == 0) pi[m] = v;
                    rw_wave_sync();
                }
                if (pos_ok) {
                    double zp = 0.0, wp = 0.0;
                    for (int32_t q = lane; q < na; q += 64) {
                        zp = zp + pi[q];
                        wp = wp + wb[act[q]];
                    }
                    const double Z = rw_wave_sum(zp), WA = rw_wave_sum(wp);
                    for (int32_t q = lane; q < na; q += 64) fac[act[q]] = (pi[q] / Z * WA) / wb[act[q]];
                    if (lane == 0) misc[3] = 2;
                }
            }
            __syncthreads();
            ok = misc[3] == 2;
        }
    }

    // 5. rescale; with rw_reset the flux matrix starts over (every read of
    // it lies before the last barrier)
    if (ok)
        for (int32_t k = tid; k < n; k += nthr) w[k] = w[k] * fac[bins[k]];
    if (a.rw_reset) {
        double *Fw = a.rw_F + (size_t)run * NB * NB;
        for (size_t t = tid; t < (size_t)NB * NB; t += nthr) Fw[t] = 0.0;
    }
    if (tid == 0) a.rw_stat[2 * (size_t)run + (ok ? 0 : 1)] += 1;
}

bool rw_solve_in_lds(int32_t NB) {
    return rw_small_bytes(NB) + 8 * (size_t)NB * NB <= RW_LDS_LIMIT;
}

hipError_t launch_reweight(const SimArgs &a, double *w_nxt, hipStream_t st) {
    const size_t shmem = rw_small_bytes(a.n_bins) + (a.rw_R ? 0 : 8 * (size_t)a.n_bins * a.n_bins);
    if (a.rw_R) hipLaunchKernelGGL(we_reweight_kernel<false>, dim3(a.n_runs), dim3(RW_THREADS), shmem, st, a, w_nxt);
    else hipLaunchKernelGGL(we_reweight_kernel<true>, dim3(a.n_runs), dim3(RW_THREADS), shmem, st, a, w_nxt);
    return hipGetLastError();
}
