// we_common.h -- device-side building blocks and the argument block shared by
// the WE kernels (gfx950).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten
// rounds of two 32x32->64 multiplies with the round key, key bumped by the
// Weyl constants between rounds.  Counter layout used throughout:
//   SSA event e of the walker in slot k, iteration i:  (e, k, i, 0)
//   merge number m in bin b, iteration i:              (m, b, i, 1)
// keyed by the run's 64-bit seed.  Every result therefore depends only on
// (seed, iteration, slot, event), never on scheduling.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define WE_COUNT_MAX_DEV 131071
#define WE_DPACK_WORDS 8

// Error bits latched in device memory.
enum : int32_t {
    WE_DERR_OVERFLOW = 1,   // a count left [0, WE_COUNT_MAX]
    WE_DERR_SELECT = 2,     // no reaction with positive propensity at selection
    WE_DERR_CAPACITY = 4,   // resampling would exceed the slot reservation
};

// One reaction's reactants and rate, packed for wave-uniform (scalar) loads.
struct __align__(16) RxnDesc {
    double c;        // stochastic rate constant c_j
    uint16_t s1, s2; // reactant species (unused entries: 0)
    uint8_t nu1, nu2;// multiplicities (0 = absent)
    uint8_t nchg;    // number of species changed
    uint8_t order;   // nu1 + nu2
};

// A reaction's Hill-type repression (Sec. III.C): its propensity is divided
// by 1 + (x_species / K)^n; n = 0: none.
struct __align__(16) HillDesc {
    double K;
    int32_t species;
    int32_t n;
};

// Where a reaction's dependency entries and changes start, in one load.
struct __align__(16) RxnInfo {
    int32_t dep_begin, dep_count, chg_begin, chg_count;
};

// One reaction whose propensity changes when a given reaction fires, with
// its own descriptor inline (so no second lookup is needed).
struct __align__(16) DepEntry {
    double c;
    uint16_t s1, s2;
    uint8_t nu1, nu2;
    uint16_t r;
};

// Species change of a reaction, packed as (species << 16) | (delta & 0xffff).
__host__ __device__ inline int32_t pack_change(int32_t s, int32_t d) {
    return (int32_t)(((uint32_t)s << 16) | ((uint32_t)d & 0xffffu));
}
__host__ __device__ inline int32_t change_species(int32_t p) { return (int32_t)((uint32_t)p >> 16); }
__host__ __device__ inline int32_t change_delta(int32_t p) { return (int32_t)(int16_t)(p & 0xffff); }

// Factored dependency graph of the LDS-resident wave kernel.  Per reaction
// an 8-byte change header: up to 4 changed species, one 16-bit code each
// (bits 0-8 species < 512, bits 9-12 delta + 8, delta in [-8, 7]), code k at
// bits 16k.  Per species one 32-bit word: where the ids of the reactions
// taking it as a reactant start in the incidence list (bits 0-15) and how
// many there are (bits 16-31); each species' ids ascend.  The reactions whose
// propensity a firing changes are the union of its changed species' lists.
#define FACT_MAX_SPECIES 512
#define FACT_MAX_INC 65535
#define FACT_MAX_CHANGES 4
__host__ __device__ inline uint32_t fact_code(int32_t s, int32_t delta) {
    return (uint32_t)s | ((uint32_t)(delta + 8) << 9);
}
__host__ __device__ inline int32_t fact_species(uint32_t code) { return (int32_t)(code & 0x1FFu); }
__host__ __device__ inline int32_t fact_delta(uint32_t code) { return (int32_t)((code >> 9) & 0xFu) - 8; }
__host__ __device__ inline uint32_t fact_inc_word(int32_t begin, int32_t count) {
    return (uint32_t)begin | ((uint32_t)count << 16);
}
// LDS byte offsets of the tables: descriptors, headers, per-species words,
// incidence ids, then the waves' slices; 16-byte aligned pieces.
__host__ __device__ inline size_t fact_align16(size_t v) { return (v + 15) & ~(size_t)15; }
__host__ __device__ inline size_t fact_off_hdr(int32_t R) { return 16 * (size_t)R; }
__host__ __device__ inline size_t fact_off_tab(int32_t R) { return fact_align16(24 * (size_t)R); }
__host__ __device__ inline size_t fact_off_inc(int32_t R, int32_t S) {
    return fact_align16(fact_off_tab(R) + 4 * (size_t)S);
}
__host__ __device__ inline size_t fact_tables_bytes(int32_t R, int32_t S, int32_t n_inc) {
    return fact_align16(fact_off_inc(R, S) + 2 * (size_t)n_inc);
}

// Everything a WE kernel needs, passed by value.
struct SimArgs {
    // network
    const RxnDesc *__restrict__ desc;    // [R]
    const int32_t *__restrict__ chg_ptr; // [R+1]
    const int32_t *__restrict__ chg;     // packed changes
    const int32_t *__restrict__ dpack;   // [R][WE_DPACK_WORDS]: the change of species s (< 32) in
                                         //   byte s%4 of word s/4, as int8 (lane kernel)
    const int32_t *__restrict__ dep_ptr; // [R+1] reactions whose propensity a reaction changes
    const uint16_t *__restrict__ dep;    //       (sorted, unique)
    const RxnInfo *__restrict__ rinfo;   // [R]
    const DepEntry *__restrict__ deps;   // dependency entries with descriptors
    const HillDesc *__restrict__ hill;   // [R padded] Hill-type rates (null: none)
    const uint2 *__restrict__ fhdr;      // [R] factored change headers (null: network too large)
    const uint32_t *__restrict__ inc_tab;// [S] incidence start | count << 16
    const uint16_t *__restrict__ inc;    // [n_inc] species -> reactions taking it as a reactant
    int32_t n_inc;
    int32_t n_chg;                       // entries of chg (chg_ptr[R])
    int32_t S, R;
    int32_t engine;                      // 0: exact SSA, 1: tau-leaping (lane kernel)
    double leap_eps;                     // tau-leaping error control
    // runs
    int32_t n_runs, cap, n_bins, m_targ, max_iters;
    int32_t rs_rule;                     // split/merge: 0 count-only, 1 weight-equalizing
    double tau;
    const uint64_t *__restrict__ seeds;  // [n_runs]
    // bins and target
    const double *__restrict__ bin_coef; // [S]
    const double *__restrict__ edges;    // [n_bins+1]
    int32_t recycle;
    double tgt_thr;
    const double *__restrict__ tgt_coef; // [S]
    const int32_t *__restrict__ bin_nz;  // species with a nonzero bin_coef, ascending
    // second grid axis (n_bins2 > 1): bin = b1 + n_bins1 * b2, n_bins = n_bins1 * n_bins2
    int32_t n_bins1, n_bins2, n_bin_nz2;
    const double *__restrict__ bin_coef2;
    const double *__restrict__ edges2;
    const int32_t *__restrict__ bin_nz2;
    const int32_t *__restrict__ tgt_nz;  // species with a nonzero tgt_coef, ascending
    int32_t n_bin_nz, n_tgt_nz;
    const int32_t *__restrict__ x_rec;   // [S]
    // ensemble (current and next buffers are passed per launch)
    int32_t *n_walk;                     // [n_runs]
    int32_t *bin;                        // [n_runs*cap] bin of each walker (after resample)
    int32_t *origin;                     // [n_runs*cap] parent slot (after resample)
    uint32_t *ev_walker;                 // [n_runs*cap] reactions fired this interval
    // series
    double *flux;                        // [n_runs*max_iters]
    int64_t *ev_iter;                    // [n_runs*max_iters]
    int32_t *seg_iter;                   // [n_runs*max_iters] walkers propagated
    // resample scratch
    int32_t *s_bin;                      // [n_runs*cap]
    int32_t *s_rec;                      // [n_runs*cap]
    int32_t *s_list;                     // [n_runs*cap]
    double *s_w;                         // [n_runs*cap]
    int32_t *s_cnt;                      // [n_runs*cap]
    // observables
    double *hist;                        // [n_runs*nh]
    int32_t hist_species, hist_lo, nh;
    double *jhist;                       // [n_runs * jcells]
    int32_t n_joint, joint_bins, joint_width, jcells;
    int32_t joint_species[5];
    int32_t *err;
    uint32_t *iter_dev;                  // current WE iteration (advanced on the device)
    // work queue of the propagation kernels: segments of up to m_targ
    // consecutive walkers, ordered by the mean events per walker of their bin
    int32_t queue_stats;                 // 1: resampling gathers the per-bin event statistics
    int32_t place_rows;                  // resampling: rows of per-bin cursors in LDS, one per
                                         //   wave that places walkers (at least 1)
    // steady-state reweighting (off when rw_period == 0)
    int32_t rw_period;
    int32_t rw_reset;                    // 1: F restarts after every event
    double *rw_F;                        // [n_runs][n_bins][n_bins] flux matrix F[i][j]
    double *rw_R;                        // [n_runs][n_bins][n_bins] solve scratch (null: in LDS)
    int32_t *rw_stat;                    // [n_runs][2] events applied, skipped
    float *ev_bin;                       // [n_bins][seg_rep] events of the walkers that ended in each bin
    int32_t *n_bin;                      // [n_bins][seg_rep] walkers that ended in each bin
    int32_t seg_rep;                     // counters per bin (spread over replicas, picked by run,
                                         //   against atomic contention): min(128, 16384/n_bins, n_runs/16), >= 1
    int32_t *occ_bin;                    // [n_bins][seg_rep] queue segments per counter
    int32_t *seg_off;                    // [n_bins][seg_rep] first queue segment of each counter
    int32_t *seg_cur;                    // [n_bins][seg_rep]
    int2 *seg;                           // [n_runs * n_bins] (first slot run*cap + j*m_targ, walkers)
    uint32_t *queue;                     // [2] next walker index, number of segments
};

// ---------------------------------------------------------------- Philox
struct U4 { uint32_t x, y, z, w; };

// Round multipliers and Weyl key increments of Philox4x32.
constexpr uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u;
constexpr uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u;

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                             uint32_t k0, uint32_t k1) {
    const uint32_t M0 = PHILOX_M0, M1 = PHILOX_M1;
    const uint32_t W0 = PHILOX_W0, W1 = PHILOX_W1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;   // one 32x32->64 multiply each
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    return U4{c0, c1, c2, c3};
}

// Uniform on [0,1) with 53 random bits: ((a >> 5) * 2^26 + (b >> 6)) * 2^-53,
// formed as (a >> 5) 2^-27 + (b >> 6) 2^-53 in one FMA: both terms are exact
// and so is their sum (below 1 with 53 significant bits), so the value is the
// same as converting the 53-bit integer, in fewer instructions.
__device__ __forceinline__ double uniform53(uint32_t a, uint32_t b) {
    return fma((double)(a >> 5), 0x1.0p-27, (double)(b >> 6) * 0x1.0p-53);
}

// 1/d for a positive normal double: the hardware reciprocal estimate and two
// Newton steps r <- r + r (1 - d r); within an ulp or so of the quotient.
__device__ __forceinline__ double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

// The same with one Newton step: the estimate is good to about 2^-25, so one
// step leaves about 2^-50 (up to ~10 ulp), which is enough where the quotient
// only scales a small correction term.
__device__ __forceinline__ double recip_1step(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

// -log(1 - u) for u in [0, 1) a 53-bit uniform, in FP64, within about one
// ulp: the exponential waiting-time variate of the direct method (Sec. II.A).
// With y = 1 - u (exact) = 2^k m, m in [sqrt(1/2), sqrt(2)):
//   log m = 2 atanh(s), s = f / (2 + f), f = m - 1 (exact),
//         = f - (f^2/2 - s (f^2/2 + R)),  R = sum_{i=1..10} 2 s^(2i) / (2i + 1)
// (the atanh series; |s| <= 0.1716, so the first omitted term is below
// 1e-18 relative), and k ln 2 is added as k ln2_hi (exact: ln2_hi has 42
// significant bits) plus k ln2_lo.  This is the argument reduction of the
// classical fdlibm logarithm with Taylor coefficients; about 35 instructions
// against twice that for the general-purpose log, whose extra precision the
// waiting time does not need.
// d = a b + c as one v_fma_f64.  Written out because in the large event
// loops the compiler otherwise turns each Horner step into a register copy of
// the coefficient followed by the accumulating v_fmac_f64.
__device__ __forceinline__ double fma_vop3(double a, double b, double c) {
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

__device__ __forceinline__ double neg_log1m(double u) {
    constexpr double LN2_HI = 0x1.62e42fefa38p-1, LN2_LO = 0x1.ef35793c7673p-45;
    int k;
    double m = frexp(1.0 - u, &k);                 // 1 - u in (2^-53, 1], m in [0.5, 1)
    if (m < 0x1.6a09e667f3bcdp-1) {                // below sqrt(1/2)
        m = m + m;
        k -= 1;
    }
    const double f = m - 1.0;
    // s enters only through s (f^2/2 + R), at most 4% of the result, so a
    // quotient within ~10 ulp costs nothing measurable (0.76 ulp at most for
    // the whole log, measured, as with the two-step reciprocal)
    const double s = f * recip_1step(2.0 + f);
    const double z = s * s;
    double R = 2.0 / 21.0;
    R = fma_vop3(z, R, 2.0 / 19.0);
    R = fma_vop3(z, R, 2.0 / 17.0);
    R = fma_vop3(z, R, 2.0 / 15.0);
    R = fma_vop3(z, R, 2.0 / 13.0);
    R = fma_vop3(z, R, 2.0 / 11.0);
    R = fma_vop3(z, R, 2.0 / 9.0);
    R = fma_vop3(z, R, 2.0 / 7.0);
    R = fma_vop3(z, R, 2.0 / 5.0);
    R = fma_vop3(z, R, 2.0 / 3.0);
    R = R * z;
    const double hfsq = 0.5 * f * f;
    const double dk = (double)k;
    // -log y = -k ln2_hi - (f - (hfsq - (s (hfsq + R) + k ln2_lo)))
    return -dk * LN2_HI - (f - (hfsq - fma(s, hfsq + R, dk * LN2_LO)));
}

// ---------------------------------------------------------------- propensity
// C(x, nu) for nu in {0,1,2,3}, exactly, as a double (x <= 2^17): x(x-1) and
// x(x-1)(x-2) are integers below 2^53, so every product is exact; C(x,3) is
// x(x-1)(x-2)/2 times the double nearest 1/3, rounded to the nearest integer,
// which is exact because the error is below 2^-3.  No 64-bit integer
// multiply or divide (quarter-rate on CDNA) is needed.
__device__ __forceinline__ double binom_f64(double xd, uint32_t nu) {
    const double p2 = xd * fmax(xd - 1.0, 0.0);
    const double c3 = rint(((p2 * fmax(xd - 2.0, 0.0)) * 0.5) * (1.0 / 3.0));
    const double c2 = p2 * 0.5;
    return nu == 0 ? 1.0 : nu == 1 ? xd : nu == 2 ? c2 : c3;
}

// a_j = c_j * h_j(x): h_j is an exact integer (order <= 3 keeps it below
// 2^53), so the only rounding is the final product, as with an int64 h.
template <class D>
__device__ __forceinline__ double propensity_from(const D &d, uint32_t x1, uint32_t x2) {
    return d.c * (binom_f64((double)x1, d.nu1) * binom_f64((double)x2, d.nu2));
}

// ---------------------------------------------------------------- bins
__device__ __forceinline__ int32_t bin_index(const double *__restrict__ edges, int32_t n_bins,
                                             double q) {
    // largest b in [0, n_bins-1] with edges[b] <= q (b = 0 if q < edges[1]);
    // binary search over the strictly increasing inner edges edges[1..n_bins-1]
    int32_t lo = 0, hi = n_bins - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (q >= edges[mid]) lo = mid; else hi = mid - 1;
    }
    return lo;
}
