// we_resample.hip -- the WE bookkeeping between two propagation steps:
// recycling, binning, per-bin split/merge, the state gather and the
// observables (gfx950).  Per iteration, after the SSA kernel:
//
//   recycle_bin (one lane per walker, whole grid)
//      recycling (Sec. II.B.2): a walker whose state lies in
//      B = { x : sum_s coef_s x_s >= thr } is flagged and restarts from the
//      state A, keeping its weight; checked once, at the end of the interval
//      (the paper checks walkers only every tau);
//      bin of every walker on the progress coordinate, or on a grid over two
//      coordinates, bin = b1 + n1 * b2 (or, with learned bins, the bin is
//      written afterwards by the committor kernel);
//   resample (one workgroup per run)
//      stable placement of the walkers by bin: per-wave cursor rows let
//      several waves place their own runs of slots at once;
//      the run's recycled weight (summed in slot order) and reactions fired;
//      per-bin split/merge (Sec. II.B), one wave per bin:
//        n == M: unchanged;
//        n <  M: replicate to M copies; one more copy is given, repeatedly,
//                to the parent with the largest per-copy weight w/c (ties:
//                lowest slot); each copy carries w/c, so the bin's weight is
//                conserved (a lone walker gets the paper's w/M exactly); the
//                wave finds the largest share with DPP max steps;
//        n >  M: merge the two lowest-weight walkers (ties: lowest slot): the
//                first survives with probability w_i/(w_i+w_j), else the
//                second, and the survivor carries w_i + w_j; repeat.
//        With the weight-equalizing rule (rs_rule 1), whatever n: W is the
//        bin's weight summed in slot order and w* = W/M; the two lowest are
//        merged as above while their sum is <= w* or the bin has no room to
//        split its heavy walkers (sum_k max(1, ceil(w_k/(2w*))) > M, which
//        includes n > M); the survivors are then replicated up to M as above.
//        Up to 64 walkers a bin is held one walker per lane in registers and
//        each merge takes two DPP wave minima.  Larger bins are sorted once
//        by (weight, slot); merged walkers queue up in the order they are
//        made, which is also non-decreasing in weight, so each merge only
//        compares the heads of the two queues (ties of equal sums ordered by
//        a small heap): the same pairs as a full search, in O(n log n)
//        instead of O(n^2);
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
#include "we_internal.h"

#include <algorithm>

#define RESAMPLE_LDS_CAP 8192
#define RESAMPLE_LDS_MAX (150 * 1024)
// Cursor rows for placing walkers in parallel: one row of n_bins per wave, as
// long as the rows hold at most this many counters.
#define RESAMPLE_PLACE_INTS 4096
// Bin-parallel resampling: runs fewer than this, bins at least this many.
#define RESAMPLE_GROUP_COUNT_M 32
#define RESAMPLE_BIN_PARALLEL_RUNS 256
#define RESAMPLE_BIN_PARALLEL_BINS 32
// Threads per run: up to 16 waves, so up to 16 bins are split/merged at
// once.  With many runs the grid fills the chip anyway and smaller blocks
// cost less to start, so launches with at least RESAMPLE_MANY_RUNS blocks use
// 4 waves per run.
#define RESAMPLE_THREADS 1024
#define RESAMPLE_MANY_RUNS 512
__host__ inline unsigned resample_threads(int64_t blocks) {
    return blocks >= RESAMPLE_MANY_RUNS ? 256u : (unsigned)RESAMPLE_THREADS;
}

// sum_s coef_s x_s in ascending species order over the nonzero
// coefficients only: a zero coefficient adds +0 or -0, which leaves a sum
// that started at +0 unchanged, so the result is the full sum bit for bit.
__device__ __forceinline__ double coord_of(const double *__restrict__ coef, const int32_t *__restrict__ nz,
                                           int32_t n_nz, const int32_t *__restrict__ xr) {
    double q = 0.0;
    for (int32_t i = 0; i < n_nz; ++i) {
        const int32_t s = nz[i];
        q = q + coef[s] * (double)xr[s];
    }
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
    if (a.recycle && coord_of(a.tgt_coef, a.tgt_nz, a.n_tgt_nz, row) >= a.tgt_thr) {
        rec = 1;
        for (int32_t s = 0; s < S; ++s) row[s] = a.x_rec[s];
    }
    a.s_rec[idx] = rec;
    if (grid_bins) {
        int32_t b = bin_index(a.edges, a.n_bins1, coord_of(a.bin_coef, a.bin_nz, a.n_bin_nz, row));
        if (a.n_bins2 > 1)
            b += a.n_bins1 * bin_index(a.edges2, a.n_bins2, coord_of(a.bin_coef2, a.bin_nz2, a.n_bin_nz2, row));
        a.s_bin[idx] = b;
    }
}

__global__ __launch_bounds__(256) void we_recycle_bin_kernel(SimArgs a, int32_t *__restrict__ x_cur,
                                                             int32_t grid_bins) {
    recycle_bin_one(a, x_cur, grid_bins, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Per-walker working arrays of one run (LDS when the run fits, else global);
// Idx is the type of an index inside one bin (uint16 in LDS, int32 in global).
template <class Idx>
struct RunWork {
    double *w;          // weights in bin-major order (-1 marks a merged-away walker)
    int32_t *list;      // slots in bin-major order
    uint16_t *tag;      // per slot: bin | 0x8000 if recycled (until placement)
    Idx *aux;           // per position: split copy counts, or the merge sort order
    Idx *qa;            // per position: queue of merged walkers (aliases tag)
};

namespace {

union RsBits {
    double d;
    int32_t w[2];
};

template <int CTRL>
__device__ __forceinline__ double rs_dpp(double v) {
    RsBits in, out;
    in.d = v;
    out.w[0] = __builtin_amdgcn_update_dpp(0, in.w[0], CTRL, 0xF, 0xF, false);
    out.w[1] = __builtin_amdgcn_update_dpp(0, in.w[1], CTRL, 0xF, 0xF, false);
    return out.d;
}

__device__ __forceinline__ double rs_readlane(double v, int l) {
    RsBits in, out;
    in.d = v;
    out.w[0] = __builtin_amdgcn_readlane(in.w[0], l);
    out.w[1] = __builtin_amdgcn_readlane(in.w[1], l);
    return out.d;
}

// Largest value over the 64 lanes (every lane gets it): quad swaps, half-row
// and row mirrors give each 16-lane row its maximum; four readlanes finish.
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, rs_dpp<0xB1>(v));    // quad_perm [1,0,3,2]
    v = fmax(v, rs_dpp<0x4E>(v));    // quad_perm [2,3,0,1]
    v = fmax(v, rs_dpp<0x141>(v));   // row_half_mirror
    v = fmax(v, rs_dpp<0x140>(v));   // row_mirror
    return fmax(fmax(rs_readlane(v, 0), rs_readlane(v, 16)), fmax(rs_readlane(v, 32), rs_readlane(v, 48)));
}

// Smallest value over the 64 lanes, by the same steps as wave_max.
__device__ __forceinline__ double wave_min(double v) {
    v = fmin(v, rs_dpp<0xB1>(v));
    v = fmin(v, rs_dpp<0x4E>(v));
    v = fmin(v, rs_dpp<0x141>(v));
    v = fmin(v, rs_dpp<0x140>(v));
    return fmin(fmin(rs_readlane(v, 0), rs_readlane(v, 16)), fmin(rs_readlane(v, 32), rs_readlane(v, 48)));
}

// Sum over the 64 lanes (every lane gets it), by the steps of wave_max.
template <int CTRL>
__device__ __forceinline__ float rs_dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float wave_sum_f32(float v) {
    v += rs_dpp_f32<0xB1>(v);
    v += rs_dpp_f32<0x4E>(v);
    v += rs_dpp_f32<0x141>(v);
    v += rs_dpp_f32<0x140>(v);
    const int32_t bits = __float_as_int(v);
    return (__int_as_float(__builtin_amdgcn_readlane(bits, 0)) + __int_as_float(__builtin_amdgcn_readlane(bits, 16))) +
           (__int_as_float(__builtin_amdgcn_readlane(bits, 32)) + __int_as_float(__builtin_amdgcn_readlane(bits, 48)));
}

__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
    for (int d = 32; d > 0; d >>= 1) v = min(v, __shfl_xor(v, d, 64));
    return v;
}

__device__ __forceinline__ int32_t wave_excl_scan(int32_t v, int lane, int32_t *total) {
    int32_t x = v;
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    *total = __shfl(x, 63, 64);
    return x - v;
}

// Orders the LDS/global accesses of the lanes of one wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int32_t wave_sum_i32(int32_t v) {
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Copies a walker of weight v needs so that none carries more than twice the
// bin's ideal weight (at least one: every walker holds a place).
__device__ __forceinline__ int32_t need_copies(double v, double two_ideal) {
    const double q = ceil(v / two_ideal);
    return q < 1.0 ? 1 : (int32_t)q;
}

struct BinOut {
    int32_t *orig;
    double *wn;
    int32_t *obin;
};

// n < M: M - n extra copies handed out one at a time to the parent with the
// largest per-copy weight w/c, ties to the lowest slot.  Lane L owns the
// contiguous parents [L*kq, (L+1)*kq), so the lowest lane holding the wave's
// largest share holds the lowest tied slot.
template <class Idx>
__device__ void split_bin(const RunWork<Idx> &wk, int32_t p0, int32_t nb, int32_t M, int32_t b, int32_t o0,
                          const BinOut &out, int lane) {
    const int32_t kq = (nb + 63) >> 6;
    const int32_t q_lo = min(lane * kq, nb), q_hi = min(q_lo + kq, nb);
    const double *w = wk.w + p0;
    Idx *c = wk.aux + p0;
    double bs = -1.0;
    int32_t bq = -1;
    for (int32_t q = q_lo; q < q_hi; ++q) {
        c[q] = 1;
        const double s = w[q] / 1.0;
        if (s > bs) { bs = s; bq = q; }
    }
    for (int32_t e = nb; e < M; ++e) {
        const double mx = wave_max(bs);
        const unsigned long long win = __ballot(bs == mx);
        const int wl = __ffsll((long long)win) - 1;
        if (lane == wl) {
            c[bq] = (Idx)(c[bq] + 1);
            bs = -1.0;
            bq = -1;
            for (int32_t q = q_lo; q < q_hi; ++q) {
                const double s = w[q] / (double)c[q];
                if (s > bs) { bs = s; bq = q; }
            }
        }
    }
    int32_t cl = 0;
    for (int32_t q = q_lo; q < q_hi; ++q) cl += (int32_t)c[q];
    int32_t tot;
    int32_t o = o0 + wave_excl_scan(cl, lane, &tot);
    for (int32_t q = q_lo; q < q_hi; ++q) {
        const int32_t cc = (int32_t)c[q];
        const double share = w[q] / (double)cc;
        const int32_t k = wk.list[p0 + q];
        for (int32_t r = 0; r < cc; ++r) {
            out.orig[o] = k;
            out.wn[o] = share;
            out.obin[o] = b;
            ++o;
        }
    }
}

// Steady-state reweighting's flux matrix (Sec. II.B.2): row `Frow` (end bin
// b) gains, walker by walker in slot order, the weight of each of the bin's
// walkers in the column of its start bin (held in aux).  One start bin at a
// time, ascending; each column is read, added to in slot order and written
// back by this wave alone.
template <class Idx>
__device__ void rw_flux_bin(double *__restrict__ Frow, const RunWork<Idx> &wk, int32_t p0, int32_t nb,
                            int lane) {
    int32_t jprev = -1;
    for (;;) {
        int32_t jm = INT32_MAX;
        for (int32_t q = lane; q < nb; q += 64) {
            const int32_t j = (int32_t)wk.aux[p0 + q];
            if (j > jprev) jm = min(jm, j);
        }
        jm = wave_min_i32(jm);
        if (jm == INT32_MAX) break;
        double acc = Frow[jm];
        for (int32_t c0 = 0; c0 < nb; c0 += 64) {
            const int32_t q = c0 + lane;
            const bool m = q < nb && (int32_t)wk.aux[p0 + q] == jm;
            const double wv = m ? wk.w[p0 + q] : 0.0;
            unsigned long long mk = __ballot(m);
            while (mk) {
                const int l = __ffsll((long long)mk) - 1;
                acc = acc + rs_readlane(wv, l);
                mk &= mk - 1ull;
            }
        }
        if (lane == 0) Frow[jm] = acc;
        jprev = jm;
    }
}

// n < M with at most 64 K parents: lane L owns the contiguous parents
// [K L, K L + K) (as split_bin's lanes do), their weights, copy counts and
// per-copy shares in registers; the same hand-out as split_bin: the lowest
// lane holding the wave's largest share holds the lowest tied slot, and
// within a lane the lowest slot wins a tie.
template <int K, class Idx>
__device__ void split_bin_lanes(const RunWork<Idx> &wk, int32_t p0, int32_t nb, int32_t M, int32_t b, int32_t o0,
                                const BinOut &out, int lane) {
    double wq[K];
    int32_t c[K];
    double bs = -1.0;
    int32_t bk = -1;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int32_t q = K * lane + k;
        wq[k] = q < nb ? wk.w[p0 + q] : 0.0;
        c[k] = 1;
        if (q < nb) {
            const double sh = wq[k] / 1.0;
            if (sh > bs) { bs = sh; bk = k; }
        }
    }
    for (int32_t e = nb; e < M; ++e) {
        const double mx = wave_max(bs);
        const int wl = __ffsll((long long)__ballot(bs == mx)) - 1;
        if (lane == wl) {
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (k == bk) c[k] += 1;
            bs = -1.0;
            bk = -1;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (K * lane + k < nb) {
                    const double sh = wq[k] / (double)c[k];
                    if (sh > bs) { bs = sh; bk = k; }
                }
        }
    }
    int32_t cl = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) cl += K * lane + k < nb ? c[k] : 0;
    int32_t tot;
    int32_t o = o0 + wave_excl_scan(cl, lane, &tot);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int32_t q = K * lane + k;
        if (q >= nb) continue;
        const double share = wq[k] / (double)c[k];
        const int32_t kk = wk.list[p0 + q];
        for (int32_t r = 0; r < c[k]; ++r) {
            out.orig[o] = kk;
            out.wn[o] = share;
            out.obin[o] = b;
            ++o;
        }
    }
}

// The merge queues of one bin.  Q1: the bin's walkers sorted by (weight,
// slot).  Q2: merged walkers in the order they were made; their weights never
// decrease (each merge takes the two lightest, so every later pair sums to at
// least as much), so only equal-weight runs of Q2 need ordering by slot: the
// run at the front of Q2 is kept as a min-heap on the slot in A[hs, he);
// A[he, re) are spent entries and A[re, t) is the rest of Q2 in order.
// Every lane runs the same steps; lane 0 does the stores.
template <class Idx>
struct MergeQueues {
    const Idx *perm;
    Idx *A;
    double *W;
    int32_t nb, h1, q1;
    double w1;
    int32_t hs, he, re, t;
    double hw;
    int lane;

    __device__ void put(int32_t i, int32_t v) {
        if (lane == 0) A[i] = (Idx)v;
        wave_sync();
    }

    __device__ void sift_down(int32_t pos, int32_t size, int32_t x) {
        for (;;) {
            int32_t ch = 2 * pos + 1;
            if (ch >= size) break;
            int32_t cv = uni((int32_t)A[hs + ch]);
            if (ch + 1 < size) {
                const int32_t cv2 = uni((int32_t)A[hs + ch + 1]);
                if (cv2 < cv) { ch += 1; cv = cv2; }
            }
            if (cv >= x) break;
            put(hs + pos, cv);
            pos = ch;
        }
        put(hs + pos, x);
    }

    __device__ void refill() {
        hs = re;
        hw = W[uni((int32_t)A[re])];
        int32_t e = re + 1;
        while (e < t && W[uni((int32_t)A[e])] == hw) ++e;
        he = e;
        re = e;
        for (int32_t i = (e - hs) / 2 - 1; i >= 0; --i) sift_down(i, e - hs, uni((int32_t)A[hs + i]));
    }

    // remove and return the lightest walker (ties: lowest slot)
    __device__ void pop(double *wo, int32_t *qo) {
        if (he == hs && re < t) refill();
        const bool has1 = h1 < nb, has2 = he > hs;
        int32_t q2 = has2 ? uni((int32_t)A[hs]) : 0;
        const bool take1 = has1 && (!has2 || w1 < hw || (w1 == hw && q1 < q2));
        if (take1) {
            *wo = w1;
            *qo = q1;
            ++h1;
            if (h1 < nb) {
                q1 = uni((int32_t)perm[h1]);
                w1 = W[q1];
            }
        } else {
            *wo = hw;
            *qo = q2;
            --he;
            if (he > hs) sift_down(0, he - hs, uni((int32_t)A[he]));
        }
    }

    __device__ void push(double s, int32_t q) {
        if (he > hs && re == t && s == hw) {
            int32_t pos = he - hs;
            if (he == t) { ++t; ++re; }
            ++he;
            while (pos > 0) {
                const int32_t par = (pos - 1) >> 1;
                const int32_t pv = uni((int32_t)A[hs + par]);
                if (pv <= q) break;
                put(hs + pos, pv);
                pos = par;
            }
            put(hs + pos, q);
        } else {
            put(t, q);
            ++t;
        }
    }
};

// n > M with at most 64 K walkers: walker q lives in lane q % 64, register
// q / 64.  Each merge finds the lightest live walker by a wave minimum (ties:
// the lowest register, then the lowest lane, i.e. the lowest slot), then the
// lightest of the rest; the merged-away walker holds +inf from then on.  The
// same pairs, draws and sums as merge_bin, without its sort of the bin.
template <int K, class Idx>
__device__ void merge_bin_lanes(const RunWork<Idx> &wk, int32_t p0, int32_t nb, int32_t M, int32_t b, int32_t o0,
                                const BinOut &out, uint32_t iter, uint32_t k0, uint32_t k1, int lane) {
    const double inf = __builtin_huge_val();
    double wv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) wv[k] = 64 * k + lane < nb ? wk.w[p0 + 64 * k + lane] : inf;
    // the lowest slot among the walkers of weight w, given each register's ballot
    auto lowest = [&](const double *v, double w) {
        int32_t q = -1;
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
            const unsigned long long m = __ballot(v[k] == w);
            if (m) q = 64 * k + __ffsll((long long)m) - 1;
        }
        return q;
    };
    double ul = 0.0;
    for (int32_t m = 0; m < nb - M; ++m) {
        if ((m & 63) == 0) {   // the next 64 merge draws, one per lane
            const U4 rr = philox4x32_10((uint32_t)(m + lane), (uint32_t)b, iter, 1u, k0, k1);
            ul = uniform53(rr.x, rr.y);
        }
        double lm = wv[0];
#pragma unroll
        for (int k = 1; k < K; ++k) lm = fmin(lm, wv[k]);
        const double wi = wave_min(lm);
        const int32_t qi = lowest(wv, wi);
        double wr[K];
#pragma unroll
        for (int k = 0; k < K; ++k) wr[k] = (64 * k + lane == qi) ? inf : wv[k];
        double lr = wr[0];
#pragma unroll
        for (int k = 1; k < K; ++k) lr = fmin(lr, wr[k]);
        const double wj = wave_min(lr);
        const int32_t qj = lowest(wr, wj);
        const double u = rs_readlane(ul, m & 63);
        const double sum = wi + wj;
        const double p_i = wi / sum;
        const int32_t keep = (u < p_i) ? qi : qj;
        const int32_t drop = (keep == qi) ? qj : qi;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (64 * k + lane == keep) wv[k] = sum;
            if (64 * k + lane == drop) wv[k] = inf;
        }
    }
    int32_t o = o0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const bool live = 64 * k + lane < nb && wv[k] != inf;
        int32_t tot;
        const int32_t ok = o + wave_excl_scan(live ? 1 : 0, lane, &tot);
        if (live) {
            out.orig[ok] = wk.list[p0 + 64 * k + lane];
            out.wn[ok] = wv[k];
            out.obin[ok] = b;
        }
        o += tot;
    }
}

// After merging with the weight-equalizing rule: the n_live survivors of a
// bin (positions whose weight is >= 0; merged-away ones hold -1) replicated
// up to M copies as in split_bin, the counts in aux.
template <class Idx>
__device__ void split_survivors(const RunWork<Idx> &wk, int32_t p0, int32_t nb, int32_t n_live, int32_t M,
                                int32_t b, int32_t o0, const BinOut &out, int lane) {
    const int32_t kq = (nb + 63) >> 6;
    const int32_t q_lo = min(lane * kq, nb), q_hi = min(q_lo + kq, nb);
    const double *w = wk.w + p0;
    Idx *c = wk.aux + p0;
    double bs = -1.0;
    int32_t bq = -1;
    for (int32_t q = q_lo; q < q_hi; ++q) {
        const bool live = w[q] >= 0.0;
        c[q] = (Idx)(live ? 1 : 0);
        if (live) {
            const double sh = w[q] / 1.0;
            if (sh > bs) { bs = sh; bq = q; }
        }
    }
    for (int32_t e = n_live; e < M; ++e) {
        const double mx = wave_max(bs);
        const int wl = __ffsll((long long)__ballot(bs == mx)) - 1;
        if (lane == wl) {
            c[bq] = (Idx)(c[bq] + 1);
            bs = -1.0;
            bq = -1;
            for (int32_t q = q_lo; q < q_hi; ++q) {
                if (!(w[q] >= 0.0)) continue;
                const double sh = w[q] / (double)c[q];
                if (sh > bs) { bs = sh; bq = q; }
            }
        }
    }
    int32_t cl = 0;
    for (int32_t q = q_lo; q < q_hi; ++q) cl += (int32_t)c[q];
    int32_t tot;
    int32_t o = o0 + wave_excl_scan(cl, lane, &tot);
    for (int32_t q = q_lo; q < q_hi; ++q) {
        const int32_t cc = (int32_t)c[q];
        if (cc == 0) continue;
        const double share = w[q] / (double)cc;
        const int32_t k = wk.list[p0 + q];
        for (int32_t r = 0; r < cc; ++r) {
            out.orig[o] = k;
            out.wn[o] = share;
            out.obin[o] = b;
            ++o;
        }
    }
}

// Weight-equalizing rule with at most 64 walkers: walker q lives in lane q.
// The merges are merge_bin_lanes' (same pairs, draws and sums) under the
// rule's condition; the survivors are then replicated as in split_bin_lanes
// (merged-away lanes hold +inf and get no copy).
template <class Idx>
__device__ void equalize_bin_lanes(const RunWork<Idx> &wk, int32_t p0, int32_t nb, int32_t M, int32_t b,
                                   int32_t o0, const BinOut &out, uint32_t iter, uint32_t k0, uint32_t k1,
                                   int lane) {
    const double inf = __builtin_huge_val();
    const bool own = lane < nb;
    double wv = own ? wk.w[p0 + lane] : inf;
    double Wb = 0.0;                      // the bin's weight, in slot order
    for (int32_t q = 0; q < nb; ++q) Wb = Wb + wk.w[p0 + q];
    const bool eq = Wb > 0.0;
    const double ideal = Wb / (double)M;
    const double two_ideal = ideal + ideal;
    int32_t need = eq ? wave_sum_i32(own ? need_copies(wv, two_ideal) : 0) : 0;
    int32_t n = nb;
    double ul = 0.0;
    for (int32_t m = 0; n > 1; ++m) {
        const double wi = wave_min(wv);
        const int qi = __ffsll((long long)__ballot(wv == wi)) - 1;
        const double wrest = lane == qi ? inf : wv;
        const double wj = wave_min(wrest);
        const int qj = __ffsll((long long)__ballot(wrest == wj)) - 1;
        const double sum = wi + wj;
        const bool go = eq ? (sum <= ideal || need > M) : (n > M);
        if (!go) break;
        if ((m & 63) == 0) {   // the next 64 merge draws, one per lane
            const U4 rr = philox4x32_10((uint32_t)(m + lane), (uint32_t)b, iter, 1u, k0, k1);
            ul = uniform53(rr.x, rr.y);
        }
        const double u = rs_readlane(ul, m & 63);
        const double p_i = wi / sum;
        const int keep = (u < p_i) ? qi : qj;
        const int drop = (keep == qi) ? qj : qi;
        if (eq) need = need - need_copies(wi, two_ideal) - need_copies(wj, two_ideal) + need_copies(sum, two_ideal);
        if (lane == keep) wv = sum;
        if (lane == drop) wv = inf;
        n -= 1;
    }
    const bool live = own && wv != inf;
    int32_t c = live ? 1 : 0;
    double bs = live ? wv / 1.0 : -1.0;
    for (int32_t e = n; e < M; ++e) {
        const double mx = wave_max(bs);
        const int wl = __ffsll((long long)__ballot(bs == mx)) - 1;
        if (lane == wl) {
            c += 1;
            bs = wv / (double)c;
        }
    }
    int32_t tot;
    int32_t o = o0 + wave_excl_scan(c, lane, &tot);
    if (live) {
        const double share = wv / (double)c;
        const int32_t k = wk.list[p0 + lane];
        for (int32_t r = 0; r < c; ++r) {
            out.orig[o] = k;
            out.wn[o] = share;
            out.obin[o] = b;
            ++o;
        }
    }
}

// n > M: merge the two lightest walkers (ties: lowest slot) until M remain.
// EQ: the weight-equalizing rule's merges, then the survivors' split.
template <class Idx, bool EQ>
__device__ void merge_bin(const RunWork<Idx> &wk, int32_t p0, int32_t nb, int32_t M, int32_t b, int32_t o0,
                          const BinOut &out, uint32_t iter, uint32_t k0, uint32_t k1, int lane) {
    double *W = wk.w + p0;
    Idx *perm = wk.aux + p0;
    bool eq = false;
    double ideal = 0.0, two_ideal = 0.0;
    int32_t need = 0;
    if (EQ) {
        double Wb = 0.0;                  // the bin's weight, in slot order
        for (int32_t q = 0; q < nb; ++q) Wb = Wb + W[q];
        eq = Wb > 0.0;
        ideal = Wb / (double)M;
        two_ideal = ideal + ideal;
        if (eq) {
            int32_t nl = 0;
            for (int32_t q = lane; q < nb; q += 64) nl += need_copies(W[q], two_ideal);
            need = wave_sum_i32(nl);
        }
        wave_sync();
    }
    // sort order of the bin by (weight, slot): bitonic network whose first
    // step of every merge compares mirrored pairs, so positions past nb act as
    // +inf and never move
    for (int32_t q = lane; q < nb; q += 64) perm[q] = (Idx)q;
    wave_sync();
    int32_t P = 1;
    while (P < nb) P <<= 1;
    for (int32_t size = 2; size <= P; size <<= 1) {
        for (int32_t d = size >> 1; d > 0; d >>= 1) {
            const bool mirror = d == (size >> 1);
            for (int32_t cidx = lane; cidx < (P >> 1); cidx += 64) {
                const int32_t blk = cidx / d, r = cidx - blk * d;
                int32_t i, j;
                if (mirror) {
                    i = blk * size + r;
                    j = blk * size + size - 1 - r;
                } else {
                    i = blk * 2 * d + r;
                    j = i + d;
                }
                if (j < nb) {
                    const int32_t qi = (int32_t)perm[i], qj = (int32_t)perm[j];
                    const double wi = W[qi], wj = W[qj];
                    if (wj < wi || (wj == wi && qj < qi)) {
                        perm[i] = (Idx)qj;
                        perm[j] = (Idx)qi;
                    }
                }
            }
            wave_sync();
        }
    }

    MergeQueues<Idx> Q;
    Q.perm = perm;
    Q.A = wk.qa + p0;
    Q.W = W;
    Q.nb = nb;
    Q.h1 = 0;
    Q.q1 = uni((int32_t)perm[0]);
    Q.w1 = W[Q.q1];
    Q.hs = Q.he = Q.re = Q.t = 0;
    Q.hw = 0.0;
    Q.lane = lane;
    double ul = 0.0;
    int32_t n = nb;
    for (int32_t m = 0; EQ ? (n > 1) : (m < nb - M); ++m) {
        double wi, wj;
        int32_t qi, qj;
        Q.pop(&wi, &qi);
        Q.pop(&wj, &qj);
        const double sum = wi + wj;
        if (EQ) {
            // the two just taken stay live (their weights are untouched)
            const bool go = eq ? (sum <= ideal || need > M) : (n > M);
            if (!go) break;
            if (eq)
                need = need - need_copies(wi, two_ideal) - need_copies(wj, two_ideal) +
                       need_copies(sum, two_ideal);
        }
        if ((m & 63) == 0) {   // the next 64 merge draws, one per lane
            const U4 rr = philox4x32_10((uint32_t)(m + lane), (uint32_t)b, iter, 1u, k0, k1);
            ul = uniform53(rr.x, rr.y);
        }
        const double u = rs_readlane(ul, m & 63);
        const double p_i = wi / sum;
        const int32_t keep = (u < p_i) ? qi : qj;
        const int32_t drop = (keep == qi) ? qj : qi;
        if (lane == 0) {
            W[keep] = sum;
            W[drop] = -1.0;
        }
        wave_sync();
        Q.push(sum, keep);
        n -= 1;
    }
    wave_sync();
    if (EQ) {
        split_survivors(wk, p0, nb, n, M, b, o0, out, lane);
        return;
    }

    const int32_t kq = (nb + 63) >> 6;
    const int32_t q_lo = min(lane * kq, nb), q_hi = min(q_lo + kq, nb);
    int32_t cl = 0;
    for (int32_t q = q_lo; q < q_hi; ++q) cl += (W[q] >= 0.0) ? 1 : 0;
    int32_t tot;
    int32_t o = o0 + wave_excl_scan(cl, lane, &tot);
    for (int32_t q = q_lo; q < q_hi; ++q) {
        const double wq = W[q];
        if (!(wq >= 0.0)) continue;
        out.orig[o] = wk.list[p0 + q];
        out.wn[o] = wq;
        out.obin[o] = b;
        ++o;
    }
}

}  // namespace

// One bin's split/merge (and its row of the reweighting flux matrix) on the
// calling wave: the walkers at positions [p0, p0 + nb) of wk, the output at
// slots [o0, o0 + M).
template <class Idx>
__device__ void resample_bin(const SimArgs &a, const RunWork<Idx> &wk, const BinOut &out, int32_t run, int32_t b,
                             int32_t nb, int32_t p0, int32_t o0, uint32_t iter, uint32_t k0, uint32_t k1,
                             bool rw_acc, int lane) {
    const int32_t NB = a.n_bins, M = a.m_targ;
    if (rw_acc) rw_flux_bin(a.rw_F + ((size_t)run * NB + b) * NB, wk, p0, nb, lane);
    if (a.rs_rule == 1) {
        if (nb <= 64) equalize_bin_lanes(wk, p0, nb, M, b, o0, out, iter, k0, k1, lane);
        else merge_bin<Idx, true>(wk, p0, nb, M, b, o0, out, iter, k0, k1, lane);
    } else if (nb == M) {
        for (int32_t q = lane; q < nb; q += 64) {
            out.orig[o0 + q] = wk.list[p0 + q];
            out.wn[o0 + q] = wk.w[p0 + q];
            out.obin[o0 + q] = b;
        }
    } else if (nb < M) {
        if (nb <= 64) split_bin_lanes<1>(wk, p0, nb, M, b, o0, out, lane);
        else if (nb <= 128) split_bin_lanes<2>(wk, p0, nb, M, b, o0, out, lane);
        else split_bin(wk, p0, nb, M, b, o0, out, lane);
    } else {
        if (nb <= 64) merge_bin_lanes<1>(wk, p0, nb, M, b, o0, out, iter, k0, k1, lane);
        else if (nb <= 128) merge_bin_lanes<2>(wk, p0, nb, M, b, o0, out, iter, k0, k1, lane);
        else if (nb <= 256) merge_bin_lanes<4>(wk, p0, nb, M, b, o0, out, iter, k0, k1, lane);
        else merge_bin<Idx, false>(wk, p0, nb, M, b, o0, out, iter, k0, k1, lane);
    }
}

// The run's working arrays in device memory (see resample_run_t).
__device__ __forceinline__ RunWork<int32_t> global_work(const SimArgs &a, size_t base) {
    RunWork<int32_t> wk;
    wk.w = a.s_w + base;
    wk.list = a.s_list + base;
    wk.tag = reinterpret_cast<uint16_t *>(a.s_cnt + base);
    wk.qa = a.s_bin + base;
    wk.aux = a.s_cnt + base;
    return wk;
}

// binfo != NULL (device arrays only, use_lds 0): stop after placement and
// staging, and leave each bin's count, first position and first output slot
// in binfo[run][3][n_bins] for we_resample_bins_kernel.
template <class Idx>
__device__ void resample_run_t(const SimArgs &a, const double *__restrict__ w_cur, double *__restrict__ w_nxt,
                               int32_t use_lds, int32_t run, unsigned char *lds, int32_t *__restrict__ binfo) {
    const int32_t tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, n_waves = nthr >> 6;
    const int32_t NB = a.n_bins, M = a.m_targ, cap = a.cap;
    __shared__ int64_t ev_part[RESAMPLE_THREADS];
    __shared__ int32_t any_rec;   // 1 when some walker was recycled this interval
    int32_t *cnt = reinterpret_cast<int32_t *>(lds);   // [NB]
    int32_t *start = cnt + NB;                          // [NB+1]
    int32_t *ostart = start + NB + 1;                   // [NB+1]
    // walkers are placed by P waves at once, wave r over its own contiguous
    // run of 64-slot chunks; row r of the cursor table first counts, per bin,
    // the walkers of those chunks, then holds where the next one goes
    const int32_t P = max(1, min(n_waves, a.place_rows));
    int32_t *cursor = ostart + NB + 1;                  // [a.place_rows][NB]
    float *evb = reinterpret_cast<float *>(cursor + (size_t)max(1, a.place_rows) * NB); // [NB] events per bin
    unsigned char *tail = reinterpret_cast<unsigned char *>(evb + NB);
    tail += (16 - ((uintptr_t)tail & 15)) & 15;

    const uint32_t iter = *a.iter_dev;
    const int32_t rec_slot = (int32_t)iter;
    const int32_t n = a.n_walk[run];
    const size_t base = (size_t)run * cap;
    const double *wr = w_cur + base;
    const int32_t *sbin = a.s_bin + base;
    const int32_t *srec = a.s_rec + base;
    RunWork<Idx> wk;
    if (use_lds) {
        wk.w = reinterpret_cast<double *>(tail);
        wk.list = reinterpret_cast<int32_t *>(wk.w + cap);
        wk.tag = reinterpret_cast<uint16_t *>(wk.list + cap);
        wk.qa = reinterpret_cast<Idx *>(wk.tag);
        wk.aux = reinterpret_cast<Idx *>(wk.tag + cap);
    } else {
        // global: the tag array in the first half of the s_cnt rows, the
        // queue over s_bin (read only before the first barrier), the aux
        // array over s_cnt once placement is done
        const RunWork<int32_t> g = global_work(a, base);
        wk.w = g.w;
        wk.list = g.list;
        wk.tag = g.tag;
        wk.qa = reinterpret_cast<Idx *>(g.qa);
        wk.aux = reinterpret_cast<Idx *>(g.aux);
    }

    const int32_t n_chunks = (n + 63) >> 6;
    const int32_t per_row = max(1, (n_chunks + P - 1) / P) * 64;   // slots per row
    for (int32_t b = tid; b < NB; b += nthr) {
        cnt[b] = 0;
        evb[b] = 0.0f;
    }
    for (int32_t i = tid; i < P * NB; i += nthr) cursor[i] = 0;
    if (tid == 0) any_rec = 0;
    __syncthreads();
    // counts per bin and per cursor row: each wave takes 64 consecutive slots
    // (one cursor row: per_row is a multiple of 64); with at least
    // RESAMPLE_GROUP_COUNT_M walkers per bin it adds each bin's group of lanes
    // with one LDS atomic (walkers sit in slot order by their previous bin, so
    // a chunk holds few bins, and LDS atomics on one address serialize), with
    // smaller bins one atomic per walker (many bins per chunk, few collisions)
    int64_t my_ev = 0;
    for (int32_t c0 = wave * 64; c0 < n; c0 += nthr) {
        const int32_t k = c0 + lane;
        const bool valid = k < n;
        int32_t b = -1;
        uint32_t ev = 0u;
        bool rc = false;
        if (valid) {
            b = sbin[k];
            ev = a.ev_walker[base + k];
            rc = srec[k] != 0;
            wk.tag[k] = (uint16_t)(b | (rc ? 0x8000 : 0));
            my_ev += ev;
        }
        if (__ballot(rc) && lane == 0) any_rec = 1;
        const int32_t row = c0 / per_row;
        if (M < RESAMPLE_GROUP_COUNT_M) {   // small bins: many per chunk, little contention
            if (valid) {
                atomicAdd(&cnt[b], 1);
                atomicAdd(&cursor[row * NB + b], 1);
                if (a.queue_stats) atomicAdd(&evb[b], (float)ev);
            }
            continue;
        }
        unsigned long long todo = __ballot(valid);
        while (todo) {
            const int leader = __ffsll((long long)todo) - 1;
            const int32_t lb = __shfl(b, leader, 64);
            const bool mine = valid && b == lb;
            const unsigned long long grp = __ballot(mine);
            const float gev = a.queue_stats ? wave_sum_f32(mine ? (float)ev : 0.0f) : 0.0f;
            if (lane == leader) {
                const int32_t g = (int32_t)__popcll(grp);
                atomicAdd(&cnt[lb], g);
                atomicAdd(&cursor[row * NB + lb], g);
                if (a.queue_stats) atomicAdd(&evb[lb], gev);
            }
            todo &= ~grp;
        }
    }
    ev_part[tid] = my_ev;
    __syncthreads();
    // per-bin event statistics for the propagation kernels' work queue (a
    // scheduling hint only: no result depends on it)
    if (a.queue_stats)
        for (int32_t b = tid; b < NB; b += nthr)
            if (cnt[b] > 0) {
                const int32_t c = b * a.seg_rep + run % a.seg_rep;
                atomicAdd(&a.ev_bin[c], evb[b]);
                atomicAdd(&a.n_bin[c], cnt[b]);
            }

    // wave 0: bin offsets (walkers ordered by bin, then slot)
    if (wave == 0) {
        const int32_t kb = (NB + 63) >> 6;
        const int32_t b_lo = min(lane * kb, NB), b_hi = min(b_lo + kb, NB);
        int32_t acc = 0, oacc = 0;
        for (int32_t b = b_lo; b < b_hi; ++b) {
            acc += cnt[b];
            oacc += cnt[b] > 0 ? M : 0;
        }
        int32_t tot, otot;
        acc = wave_excl_scan(acc, lane, &tot);
        oacc = wave_excl_scan(oacc, lane, &otot);
        for (int32_t b = b_lo; b < b_hi; ++b) {
            start[b] = acc;
            ostart[b] = oacc;
            acc += cnt[b];
            oacc += cnt[b] > 0 ? M : 0;
        }
        if (lane == 63) {
            start[NB] = tot;
            ostart[NB] = otot;
        }
    }
    __syncthreads();
    // row r's count of bin b becomes the position of its first walker of b
    for (int32_t b = tid; b < NB; b += nthr) {
        int32_t c = start[b];
        for (int32_t r = 0; r < P; ++r) {
            const int32_t t = cursor[r * NB + b];
            cursor[r * NB + b] = c;
            c += t;
        }
    }
    __syncthreads();

    // stable placement: waves r < P, each over its chunks in slot order;
    // lanes with the same bin are ranked by a ballot and the bin's cursor
    // advances by the group size
    if (wave < P) {
        int32_t *cur = cursor + wave * NB;
        const int32_t k_hi = min(n, (wave + 1) * per_row);
        for (int32_t c0 = wave * per_row; c0 < k_hi; c0 += 64) {
            const int32_t k = c0 + lane;
            const bool valid = k < k_hi;
            const int32_t b = valid ? (int32_t)(wk.tag[k] & 0x7FFF) : -1;
            unsigned long long todo = __ballot(valid);
            while (todo) {
                const int leader = __ffsll((long long)todo) - 1;
                const int32_t lb = __shfl(b, leader, 64);
                const unsigned long long grp = __ballot(valid && b == lb);
                if (valid && b == lb) {
                    const unsigned long long below = lane ? (grp & ((1ull << lane) - 1ull)) : 0ull;
                    wk.list[cur[lb] + __popcll(below)] = k;
                }
                wave_sync();
                if (lane == leader) cur[lb] += __popcll(grp);
                wave_sync();
                todo &= ~grp;
            }
        }
    }
    // the last wave: reactions fired and the recycled weight, summed in slot
    // order
    if (wave == n_waves - 1) {
        int64_t ev = 0;
        for (int32_t t = lane; t < nthr; t += 64) ev += ev_part[t];
        for (int d = 32; d > 0; d >>= 1) ev += __shfl_xor(ev, d, 64);
        double f = 0.0;
        for (int32_t c0 = 0; any_rec && c0 < n; c0 += 64) {   // no recycled walker: f stays 0
            const int32_t k = c0 + lane;
            const bool rec = k < n && (wk.tag[k] & 0x8000);
            unsigned long long rm = __ballot(rec);
            if (rm) {
                const double wv = rec ? wr[k] : 0.0;
                while (rm) {
                    const int l = __ffsll((long long)rm) - 1;
                    f = f + rs_readlane(wv, l);
                    rm &= rm - 1ull;
                }
            }
        }
        if (lane == 0 && rec_slot < a.max_iters) {
            a.flux[(size_t)run * a.max_iters + rec_slot] = f;
            a.ev_iter[(size_t)run * a.max_iters + rec_slot] = ev;
            a.seg_iter[(size_t)run * a.max_iters + rec_slot] = n;
        }
    }
    __syncthreads();
    // flux matrix of reweighting: from the second interval on (the first
    // one's walkers carry no bin yet); the start bins go to aux, which only
    // the split/merge of the same bin uses afterwards
    const bool rw_acc = a.rw_F != nullptr && iter >= 1u;
    for (int32_t p = tid; p < n; p += nthr) {
        const int32_t k = wk.list[p];
        wk.w[p] = wr[k];
        if (rw_acc) wk.aux[p] = (Idx)a.bin[base + k];
    }
    __syncthreads();

    if (binfo) {
        // bin-parallel mode: leave the bins to we_resample_bins_kernel
        int32_t *bi = binfo + (size_t)run * 3 * NB;
        for (int32_t b = tid; b < NB; b += nthr) {
            bi[b] = cnt[b];
            bi[NB + b] = start[b];
            bi[2 * NB + b] = ostart[b];
        }
        if (tid == 0) a.n_walk[run] = ostart[NB];
        return;
    }

    // split / merge: one wave per bin
    const uint64_t seed = a.seeds[run];
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    BinOut out;
    out.orig = a.origin + base;
    out.obin = a.bin + base;
    out.wn = w_nxt + base;
    for (int32_t b = wave; b < NB; b += n_waves) {
        const int32_t nb = uni(cnt[b]);
        if (nb == 0) continue;
        resample_bin(a, wk, out, run, b, nb, uni(start[b]), uni(ostart[b]), iter, k0, k1, rw_acc, lane);
    }
    __syncthreads();
    if (tid == 0) a.n_walk[run] = ostart[NB];
}

__device__ __forceinline__ void resample_run(const SimArgs &a, const double *__restrict__ w_cur,
                                             double *__restrict__ w_nxt, int32_t use_lds, int32_t run,
                                             unsigned char *lds, int32_t *binfo = nullptr) {
    if (use_lds) resample_run_t<uint16_t>(a, w_cur, w_nxt, 1, run, lds, nullptr);
    else resample_run_t<int32_t>(a, w_cur, w_nxt, 0, run, lds, binfo);
}

__global__ __launch_bounds__(RESAMPLE_THREADS) void we_resample_kernel(SimArgs a, const double *__restrict__ w_cur,
                                                          double *__restrict__ w_nxt, int32_t use_lds,
                                                          int32_t *__restrict__ binfo) {
    extern __shared__ __align__(16) unsigned char lds[];
    resample_run(a, w_cur, w_nxt, use_lds, blockIdx.x, lds, binfo);
}

// Bin-parallel split/merge after we_resample_kernel's placement: grid
// (ceil(n_bins / 4), runs), one wave per bin, the same per-bin steps on the
// run's arrays in device memory; bins of one run write disjoint ranges.
__global__ __launch_bounds__(256) void we_resample_bins_kernel(SimArgs a, double *__restrict__ w_nxt,
                                                               const int32_t *__restrict__ binfo) {
    const int lane = threadIdx.x & 63;
    const int32_t run = blockIdx.y, NB = a.n_bins;
    const int32_t b = (int32_t)blockIdx.x * 4 + (int32_t)(threadIdx.x >> 6);
    if (b >= NB) return;                       // uniform over the wave
    const int32_t *bi = binfo + (size_t)run * 3 * NB;
    const int32_t nb = uni(bi[b]);
    if (nb == 0) return;
    const size_t base = (size_t)run * a.cap;
    const RunWork<int32_t> wk = global_work(a, base);
    BinOut out;
    out.orig = a.origin + base;
    out.obin = a.bin + base;
    out.wn = w_nxt + base;
    const uint32_t iter = *a.iter_dev;
    const uint64_t seed = a.seeds[run];
    resample_bin(a, wk, out, run, b, nb, uni(bi[NB + b]), uni(bi[2 * NB + b]), iter, (uint32_t)seed,
                 (uint32_t)(seed >> 32), a.rw_F != nullptr && iter >= 1u, lane);
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

// The same with 32-bit index arithmetic, for sims whose n_runs * cap * S
// copy numbers stay below 2^31: a 64-bit division by a runtime divisor is a
// long instruction sequence, a 32-bit one a short one.
__device__ __forceinline__ void gather_one32(const SimArgs &a, const int32_t *__restrict__ x_cur,
                                             int32_t *__restrict__ x_nxt, uint32_t gid) {
    const uint32_t S = (uint32_t)a.S, per_run = (uint32_t)a.cap * S;
    const uint32_t run = gid / per_run;
    if (run >= (uint32_t)a.n_runs) return;
    const uint32_t rem = gid - run * per_run;
    const uint32_t dst = rem / S;
    const uint32_t s = rem - dst * S;
    if ((int32_t)dst >= a.n_walk[run]) return;
    const uint32_t base = run * (uint32_t)a.cap;
    const uint32_t src = (uint32_t)a.origin[base + dst];
    x_nxt[(base + dst) * S + s] = x_cur[(base + src) * S + s];
}

__global__ __launch_bounds__(256) void we_gather_rows_kernel(SimArgs a, const int32_t *__restrict__ x_cur,
                                                             int32_t *__restrict__ x_nxt, int32_t narrow) {
    if (narrow)
        gather_one32(a, x_cur, x_nxt, blockIdx.x * blockDim.x + threadIdx.x);
    else
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

__global__ __launch_bounds__(RESAMPLE_THREADS) void we_batch_resample_kernel(BatchPtrs b) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int32_t i = blockIdx.y;
    const SimArgs &a = b.args[i];
    if ((int32_t)blockIdx.x >= a.n_runs) return;
    resample_run(a, b.w_cur[i], b.w_nxt[i], b.use_lds[i], blockIdx.x, lds);
}

// Grid-strided over each member's own cells: a grid sized for the largest
// member would spend most of its workgroups on members that have no cells
// left for them.
__global__ __launch_bounds__(256) void we_batch_gather_kernel(BatchPtrs b) {
    const int32_t i = blockIdx.y;
    const SimArgs &a = b.args[i];
    const int64_t cells = (int64_t)a.n_runs * a.cap * a.S;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < cells; gid += stride)
        gather_one(a, b.x_cur[i], b.x_nxt[i], gid);
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

// Workgroups per member in the batched gather (each strides over its member's
// cells): 64 members then give 32768 workgroups, 128 per CU.
#define BATCH_GATHER_BLOCKS 512

hipError_t launch_batch_bookkeeping(const BatchPtrs &b, int32_t n_sims, int64_t max_slots, int32_t max_runs,
                                    int64_t max_cells, size_t shmem, bool observe, const CmBatchModel *models,
                                    int32_t s_max_cm, hipStream_t st) {
    const unsigned gs = (unsigned)((max_slots + 255) / 256);
    hipLaunchKernelGGL(we_batch_recycle_bin_kernel, dim3(gs, n_sims), dim3(256), 0, st, b);
    if (models) {
        const hipError_t e = committor_bin_batch(b.args, b.x_cur, models, n_sims, max_slots, s_max_cm, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(we_batch_resample_kernel, dim3(max_runs, n_sims),
                       dim3(resample_threads((int64_t)max_runs * n_sims)), shmem, st, b);
    const unsigned gg = (unsigned)std::max<int64_t>(1, std::min<int64_t>((max_cells + 255) / 256, BATCH_GATHER_BLOCKS));
    hipLaunchKernelGGL(we_batch_gather_kernel, dim3(gg, n_sims), dim3(256), 0, st, b);
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
static size_t lds_bytes_rows(const SimArgs &a, bool use_lds, int32_t rows) {
    size_t b = sizeof(int32_t) * ((4 + (size_t)rows) * a.n_bins + 2) + 16;
    if (use_lds) b += (size_t)a.cap * (sizeof(double) + sizeof(int32_t) + 2 * sizeof(uint16_t));
    return b;
}

size_t resample_lds_bytes(const SimArgs &a, bool use_lds) {
    return lds_bytes_rows(a, use_lds, a.place_rows > 0 ? a.place_rows : 1);
}

// The per-walker arrays go to LDS when they fit beside a single cursor row.
bool resample_uses_lds(const SimArgs &a) {
    return a.cap <= RESAMPLE_LDS_CAP && lds_bytes_rows(a, true, 1) <= RESAMPLE_LDS_MAX;
}

int32_t resample_place_rows(const SimArgs &a, int64_t blocks) {
    const bool ul = resample_uses_lds(a);
    int32_t rows = (int32_t)(resample_threads(blocks) / 64);
    rows = std::min<int32_t>(rows, std::max<int32_t>(1, RESAMPLE_PLACE_INTS / std::max(1, a.n_bins)));
    while (rows > 1 && lds_bytes_rows(a, ul, rows) > RESAMPLE_LDS_MAX) --rows;
    return rows;
}

// Bin-parallel resampling pays when the runs alone leave most of the chip idle
// and a run's waves would otherwise take more than one bin each in turn
// (measured, one MI355X: 16 toggle runs x 64 bins 0.045 -> 0.033 ms, 64
// switch runs x 465 bins 0.211 -> 0.202 ms; one run of 50 bins on 16 waves
// 35.1 -> 33.3 us and eight such runs 57.2 -> 56.4 us per step, with the
// bins of up to 256 walkers merged in registers -- before those, one run
// of 50 bins went 0.063 -> 0.067 ms, its staging being in device memory).
bool resample_bins_parallel(const SimArgs &a) {
    const int64_t waves = resample_threads(a.n_runs) / 64;
    return a.n_runs < RESAMPLE_BIN_PARALLEL_RUNS && a.n_bins >= RESAMPLE_BIN_PARALLEL_BINS &&
           a.n_bins >= waves;
}

hipError_t launch_resample(const SimArgs &a, int32_t *x_cur, const double *w_cur, int32_t *x_nxt,
                           double *w_nxt, int32_t *binfo, hipStream_t st) {
    const bool split = binfo && resample_bins_parallel(a);
    const bool use_lds = !split && resample_uses_lds(a);
    const size_t shmem = resample_lds_bytes(a, use_lds);
    hipLaunchKernelGGL(we_resample_kernel, dim3(a.n_runs), dim3(resample_threads(a.n_runs)), shmem, st, a, w_cur, w_nxt,
                       use_lds ? 1 : 0, split ? binfo : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (split) {
        hipLaunchKernelGGL(we_resample_bins_kernel, dim3((unsigned)((a.n_bins + 3) / 4), (unsigned)a.n_runs), dim3(256),
                           0, st, a, w_nxt, binfo);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t total = (int64_t)a.n_runs * a.cap * a.S;
    const int32_t narrow = total + 256 < ((int64_t)1 << 31) ? 1 : 0;
    hipLaunchKernelGGL(we_gather_rows_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       a, x_cur, x_nxt, narrow);
    return hipGetLastError();
}

// The same with the one-species histogram summed per block in LDS first:
// block (run, i) takes walkers i*per ... (i+1)*per - 1 of one run, adds their
// weights into an LDS copy of the run's histogram row, then adds the nonzero
// entries to the row in device memory (one atomic per distinct count per
// block instead of one per walker, and none on a shared address within a
// run); the joint histogram likewise, per distinct cell.  Thread 0 of
// block (0, 0) also advances the iteration counter, which no step of this
// kernel reads, in place of the separate advance launch.  per = 1024
// walkers (four per thread) when the runs alone give enough blocks, else 256
// (one per thread: few runs, where the blocks' walkers are the whole grid).
#define OBS_WALKERS 1024
#define OBS_WALKERS_FEW 256
#define OBS_FEW_RUNS 64
#define OBS_LDS_BINS 6144
#define OBS_JOINT_LOG2 9
#define OBS_JOINT_SLOTS (1 << OBS_JOINT_LOG2)
#define OBS_JOINT_PROBES 16
__global__ __launch_bounds__(256) void we_observe_lds_kernel(SimArgs a, const int32_t *__restrict__ xs,
                                                             const double *__restrict__ ws, int32_t per) {
    extern __shared__ __align__(16) unsigned char obs_lds[];
    double *h = reinterpret_cast<double *>(obs_lds);
    // joint-histogram cells of this block's walkers, summed per distinct cell
    // in an open-addressing table before one device atomic per cell (walkers
    // of one bin tend to share a cell, and device atomics on one address
    // serialize)
    __shared__ int32_t jkey[OBS_JOINT_SLOTS];
    __shared__ double jval[OBS_JOINT_SLOTS];
    const int32_t run = blockIdx.x, tid = threadIdx.x;
    if (run == 0 && blockIdx.y == 0 && tid == 0) *a.iter_dev += 1u;
    const int32_t n = a.n_walk[run];
    const int32_t k0 = (int32_t)blockIdx.y * per, k1 = min(n, k0 + per);
    if (k0 >= n) return;   // uniform over the block
    for (int32_t v = tid; v < a.nh; v += blockDim.x) h[v] = 0.0;
    for (int32_t v = tid; v < OBS_JOINT_SLOTS; v += blockDim.x) {
        jkey[v] = -1;
        jval[v] = 0.0;
    }
    __syncthreads();
    const size_t base = (size_t)run * a.cap;
    double *jrow = a.jhist + (size_t)run * a.jcells;
    for (int32_t k = k0 + tid; k < k1; k += blockDim.x) {
        const size_t idx = base + k;
        const double wv = ws[idx];
        const int32_t v = xs[idx * a.S + a.hist_species] - a.hist_lo;
        if (v >= 0 && v < a.nh) atomicAdd(&h[v], wv);
        if (a.n_joint > 0) {
            int32_t cell = 0, mul = 1;
            for (int d = 0; d < a.n_joint; ++d) {
                const int32_t c = min(xs[idx * a.S + a.joint_species[d]] / a.joint_width, a.joint_bins - 1);
                cell += c * mul;
                mul *= a.joint_bins;
            }
            const uint32_t h0 = ((uint32_t)cell * 2654435761u) >> (32 - OBS_JOINT_LOG2);
            bool done = false;
            for (int32_t p = 0; p < OBS_JOINT_PROBES && !done; ++p) {
                const int32_t slot = (int32_t)((h0 + (uint32_t)p) & (OBS_JOINT_SLOTS - 1));
                const int32_t prev = atomicCAS(&jkey[slot], -1, cell);
                if (prev == -1 || prev == cell) {
                    atomicAdd(&jval[slot], wv);
                    done = true;
                }
            }
            if (!done) atomicAdd(&jrow[cell], wv);   // table crowded: straight to the device row
        }
    }
    __syncthreads();
    double *row = a.hist + (size_t)run * a.nh;
    for (int32_t v = tid; v < a.nh; v += blockDim.x)
        if (h[v] != 0.0) atomicAdd(&row[v], h[v]);
    for (int32_t v = tid; v < OBS_JOINT_SLOTS; v += blockDim.x)
        if (jkey[v] >= 0) atomicAdd(&jrow[jkey[v]], jval[v]);
}

// Histograms and the end of the iteration; *advanced tells whether the iteration
// counter was advanced (else the caller launches the advance kernel).
hipError_t launch_observe(const SimArgs &a, const int32_t *xs, const double *ws, hipStream_t st, bool *advanced) {
    *advanced = false;
    if (a.nh > 0 && a.nh <= OBS_LDS_BINS) {
        const int32_t per = a.n_runs < OBS_FEW_RUNS ? OBS_WALKERS_FEW : OBS_WALKERS;
        const dim3 grid((unsigned)a.n_runs, (unsigned)((a.cap + per - 1) / per));
        hipLaunchKernelGGL(we_observe_lds_kernel, grid, dim3(256), (size_t)a.nh * sizeof(double), st, a, xs, ws,
                           per);
        *advanced = true;
        return hipGetLastError();
    }
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
