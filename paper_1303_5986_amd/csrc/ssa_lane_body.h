// ssa_lane_body.h -- the lane-per-walker event loop (one walker through one
// interval), shared by the per-sim kernel and the batched persistent kernel.
//
// Nothing inside the event loop waits on global memory:
//  * the reaction descriptors are read as whole 16-byte words at uniform
//    addresses (scalar loads, kept in SGPRs where they fit);
//  * h_j(x) = prod_s C(x_s, nu_js) is formed in FP64: every factor and the
//    product are integers below 2^53 (counts <= 2^17, order <= 3), so each
//    is exact -- C(x,3) is x(x-1)(x-2)/2 times the double nearest 1/3,
//    rounded to the nearest integer, which is exact because the error is
//    below 2^-3 -- and no 64-bit integer division is needed;
//  * the state change of the chosen reaction comes from a table of int8
//    deltas per reaction and species: small networks pick their row with
//    register selects while the reaction is chosen, larger ones read it from
//    a per-wave copy in LDS.
#pragma once
#include "we_common.h"

// Networks of up to LANE_REG_RMAX reactions keep their delta rows in registers.
#define LANE_REG_RMAX 8

namespace {

struct LaneRxn {
    double c;
    uint32_t s1, s2, nu1, nu2;
};

__device__ __forceinline__ LaneRxn lane_rxn(const RxnDesc *__restrict__ desc, int j) {
    const uint4 r = reinterpret_cast<const uint4 *>(desc)[j];
    LaneRxn o;
    o.c = __hiloint2double((int)r.y, (int)r.x);
    o.s1 = r.z & 0xFFFFu;
    o.s2 = r.z >> 16;
    o.nu1 = r.w & 0xFFu;
    o.nu2 = (r.w >> 8) & 0xFFu;
    return o;
}

template <int SMAX>
__device__ __forceinline__ double lane_propensity(const LaneRxn &d, const int32_t (&x)[SMAX]) {
    const double h1 = binom_f64((double)x[SMAX == 1 ? 0 : d.s1], d.nu1);
    const double h2 = binom_f64((double)x[SMAX == 1 ? 0 : d.s2], d.nu2);
    return d.c * (h1 * h2);
}

struct LaneHill {
    double K;
    uint32_t s, n;
};

__device__ __forceinline__ LaneHill lane_hill(const HillDesc *__restrict__ hill, int j) {
    const uint4 r = reinterpret_cast<const uint4 *>(hill)[j];
    LaneHill o;
    o.K = __hiloint2double((int)r.y, (int)r.x);
    o.s = r.z;
    o.n = r.w;
    return o;
}

// Hill-type repression (Sec. III.C): a / (1 + t^n), t = x_s / K, the power
// by repeated multiplication, each step one rounding.
template <int SMAX>
__device__ __forceinline__ double lane_repress(double a, const LaneHill &h, const int32_t (&x)[SMAX]) {
    if (h.n == 0) return a;
    const double t = (double)x[SMAX == 1 ? 0 : h.s] / h.K;
    double p = t;
    for (uint32_t i = 1; i < h.n; ++i) p = p * t;
    return a / (1.0 + p);
}

}  // namespace

// Words of the delta row a variant reads (4 species per word).
template <int SMAX>
struct LaneRow {
    static constexpr int W = (SMAX + 3) / 4;
};

// Copies the network's delta rows (R rows of LaneRow<SMAX>::W words) into
// the calling wave's LDS slice; all 64 lanes take part.
template <int SMAX>
__device__ __forceinline__ void lane_stage_rows(const SimArgs &a, int32_t *rows) {
    constexpr int W = LaneRow<SMAX>::W;
    const int lane = threadIdx.x & 63;
    for (int i = lane; i < a.R * W; i += 64) rows[i] = a.dpack[(i / W) * WE_DPACK_WORDS + (i % W)];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The network's uniform tables as one lane kernel sees them.  HILL: some
// reactions carry a Hill-type repression (read with the descriptors).
template <int SMAX, int RMAX, bool HILL = false>
struct LaneNet {
    static constexpr int W = LaneRow<SMAX>::W;
    static constexpr bool REG = RMAX <= LANE_REG_RMAX;
    LaneRxn rx[REG ? RMAX : 1];
    uint32_t drow[REG ? RMAX : 1][W];
    LaneHill hl[HILL && REG ? RMAX : 1];
    const RxnDesc *desc;
    const HillDesc *hill;
    const int32_t *dpack;
    const int32_t *rows;   // this wave's staged delta rows (unused when REG)
    int32_t R;

    // tables padded with zero-rate rows to 64 reactions, so every load is
    // in bounds; small networks keep them in registers for the whole launch
    __device__ __forceinline__ void load(const SimArgs &a, const int32_t *rows_) {
        desc = a.desc;
        hill = a.hill;
        dpack = a.dpack;
        rows = rows_;
        R = a.R;
        if constexpr (REG) {
#pragma unroll
            for (int j = 0; j < RMAX; ++j) {
                rx[j] = lane_rxn(a.desc, j);
#pragma unroll
                for (int w = 0; w < W; ++w) drow[j][w] = (uint32_t)a.dpack[j * WE_DPACK_WORDS + w];
                if constexpr (HILL) hl[j] = lane_hill(a.hill, j);
            }
        }
    }
};

// The walker's SSA stream, Philox4x32-10 at counter (e, slot, iter, 0) under
// key (k0, k1), with everything that does not depend on the event number e
// worked out once per walker.  Round 0 multiplies only c0 = e (c2 = iter is
// the same for every event), so its output word c0 = hi(M1 iter) ^ slot ^ k0
// is fixed; round 1 then multiplies that fixed word, so its M0 product is
// fixed as well and is folded, with the round keys, into a1, b1 and b2.  The
// remaining round keys k + r W are kept rather than recomputed per event.
// draw(e) returns exactly philox4x32_10(e, slot, iter, 0, k0, k1).
struct SsaStream {
    uint32_t k1;        // round 0 key word 1
    uint32_t a1, b1;    // round 1: lo(M1 iter) ^ (k0 + W0); hi(M0 c0') ^ (k1 + W1)
    uint32_t b2;        // round 2: lo(M0 c0') ^ (k1 + 2 W1)
    uint32_t kk0[8];    // k0 + r W0, r = 2..9
    uint32_t kk1[7];    // k1 + r W1, r = 3..9

    __device__ __forceinline__ void init(uint32_t slot, uint32_t iter, uint32_t k0_, uint32_t k1_) {
        const uint64_t p = (uint64_t)PHILOX_M1 * iter;
        const uint32_t c0 = (uint32_t)(p >> 32) ^ slot ^ k0_;   // round 0 output word c0
        const uint64_t q = (uint64_t)PHILOX_M0 * c0;
        k1 = k1_;
        a1 = (uint32_t)p ^ (k0_ + PHILOX_W0);
        b1 = (uint32_t)(q >> 32) ^ (k1_ + PHILOX_W1);
        b2 = (uint32_t)q ^ (k1_ + 2u * PHILOX_W1);
#pragma unroll
        for (int r = 2; r < 10; ++r) kk0[r - 2] = k0_ + (uint32_t)r * PHILOX_W0;
#pragma unroll
        for (int r = 3; r < 10; ++r) kk1[r - 3] = k1_ + (uint32_t)r * PHILOX_W1;
    }

    __device__ __forceinline__ U4 draw(uint32_t e) const {
        // round 0: (e, slot, iter, 0) -> (fixed, lo(M1 iter), hi(M0 e) ^ k1, lo(M0 e))
        uint64_t p0 = (uint64_t)PHILOX_M0 * e;
        uint32_t c2 = (uint32_t)(p0 >> 32) ^ k1;
        uint32_t c3 = (uint32_t)p0;
        // round 1: the M0 product of the fixed word is in b1 (and in b2 for round 2)
        uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t c0 = (uint32_t)(p1 >> 32) ^ a1;
        uint32_t c1 = (uint32_t)p1;
        c2 = b1 ^ c3;
        // round 2: its c3 is the fixed lo(M0 c0'), already in b2
        p0 = (uint64_t)PHILOX_M0 * c0;
        p1 = (uint64_t)PHILOX_M1 * c2;
        c0 = (uint32_t)(p1 >> 32) ^ c1 ^ kk0[0];
        c1 = (uint32_t)p1;
        c2 = (uint32_t)(p0 >> 32) ^ b2;
        c3 = (uint32_t)p0;
#pragma unroll
        for (int r = 3; r < 10; ++r) {
            p0 = (uint64_t)PHILOX_M0 * c0;
            p1 = (uint64_t)PHILOX_M1 * c2;
            c0 = (uint32_t)(p1 >> 32) ^ c1 ^ kk0[r - 2];
            c1 = (uint32_t)p1;
            c2 = (uint32_t)(p0 >> 32) ^ c3 ^ kk1[r - 3];
            c3 = (uint32_t)p0;
        }
        return U4{c0, c1, c2, c3};
    }
};

// One walker's progress through the current interval (its counts live in a
// separate register array, which keeps this struct out of LDS).
struct LaneWalker {
    double t;
    uint32_t e, fired;
    uint32_t slot, k0, k1;
    bool bad;
    SsaStream rs;

    template <int SMAX>
    __device__ __forceinline__ void begin(int32_t (&x)[SMAX], const int32_t *__restrict__ xr, int32_t S, uint32_t k,
                                          uint64_t seed, uint32_t iter) {
#pragma unroll
        for (int s = 0; s < SMAX; ++s) x[s] = (s < S) ? xr[s] : 0;
        t = 0.0;
        e = 0;
        fired = 0;
        slot = k;
        k0 = (uint32_t)seed;
        k1 = (uint32_t)(seed >> 32);
        bad = false;
        rs.init(k, iter, k0, k1);
    }
};

// One event of the direct method (Sec. II.A); false once the walker's
// interval is over (next event beyond tau, no reaction possible, or a count
// out of range -- then w.bad is set).
template <int SMAX, int RMAX, bool HILL>
__device__ __forceinline__ bool lane_event(const LaneNet<SMAX, RMAX, HILL> &net, LaneWalker &w,
                                           int32_t (&x)[SMAX], uint32_t iter, double tau) {
    constexpr int W = LaneRow<SMAX>::W;
    constexpr bool REG = LaneNet<SMAX, RMAX, HILL>::REG;
    double prop[RMAX];
    double a0 = 0.0;
#pragma unroll
    for (int j = 0; j < RMAX; ++j) {
        const LaneRxn d = REG ? net.rx[REG ? j : 0] : lane_rxn(net.desc, j);
        prop[j] = 0.0;
        // register-held tables: rows past R are zero-rate padding, whose
        // propensity is +0 and leaves every sum unchanged, so no row test
        if (REG || j < net.R) {
            prop[j] = lane_propensity<SMAX>(d, x);
            if constexpr (HILL) prop[j] = lane_repress<SMAX>(prop[j], REG ? net.hl[REG ? j : 0] : lane_hill(net.hill, j), x);
            a0 = a0 + prop[j];
        }
    }
    if (!(a0 > 0.0)) return false;
    const U4 r = w.rs.draw(w.e);
    w.e += 1;
    const double u1 = uniform53(r.x, r.y);
    const double u2 = uniform53(r.z, r.w);
    const double dt = neg_log1m(u1) * recip(a0);
    if (w.t + dt > tau) return false;
    w.t = w.t + dt;
    const double target = u2 * a0;
    // The chosen reaction is the first j whose running sum (in reaction order)
    // exceeds the target; if rounding leaves the target above the whole sum,
    // the last reaction with a positive propensity.
    int32_t jsel = -1;
    uint32_t dsel[W];
#pragma unroll
    for (int q = 0; q < W; ++q) dsel[q] = 0u;
    if constexpr (RMAX <= 8) {
        // Small networks: all running sums first, then one pass from the last
        // reaction to the first that takes every hit and so ends on the first
        // (the sums never decrease, every term being >= 0; padding rows repeat
        // the last sum and never come before a real hit).  A select per
        // reaction and no first-hit bookkeeping: 1.067 -> 0.994 ms per launch
        // on Schloegl, measured A/B.  Larger networks keep the forward pass:
        // the stored sums would cost them occupancy.
        double cum[RMAX];
        double c = 0.0;
#pragma unroll
        for (int j = 0; j < RMAX; ++j) {
            if (REG || j < net.R) c = c + prop[j];
            cum[j] = c;
        }
#pragma unroll
        for (int j = RMAX - 1; j >= 0; --j) {
            const bool hit = cum[j] > target;
            if constexpr (REG) {
#pragma unroll
                for (int q = 0; q < W; ++q) dsel[q] = hit ? net.drow[REG ? j : 0][q] : dsel[q];
            } else {
                jsel = hit ? j : jsel;
            }
        }
        if (!(c > target)) {
#pragma unroll
            for (int j = 0; j < RMAX; ++j)
                if ((REG || j < net.R) && prop[j] > 0.0) jsel = j;
            if constexpr (REG) {
#pragma unroll
                for (int q = 0; q < W; ++q) dsel[q] = (uint32_t)net.dpack[jsel * WE_DPACK_WORDS + q];
            }
        }
    } else {
        double cum = 0.0;
        int32_t last_pos = -1;
#pragma unroll
        for (int j = 0; j < RMAX; ++j) {
            if (j < net.R) {
                cum = cum + prop[j];
                if (prop[j] > 0.0) last_pos = j;
                const bool hit = (jsel < 0) && (cum > target);
                if (hit) jsel = j;
                if constexpr (REG) {
#pragma unroll
                    for (int q = 0; q < W; ++q) dsel[q] = hit ? net.drow[REG ? j : 0][q] : dsel[q];
                }
            }
        }
        if (jsel < 0) {
            jsel = last_pos;
            if constexpr (REG) {
#pragma unroll
                for (int q = 0; q < W; ++q) dsel[q] = (uint32_t)net.dpack[jsel * WE_DPACK_WORDS + q];
            }
        }
    }
    if constexpr (!REG) {
#pragma unroll
        for (int q = 0; q < W; ++q) dsel[q] = (uint32_t)net.rows[jsel * W + q];
    }
    w.fired += 1;
    int32_t any = 0;
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
        x[s] += (int32_t)(dsel[s >> 2] << (24 - 8 * (s & 3))) >> 24;
        any |= x[s];
    }
    // a count left [0, 2^17 - 1] iff a bit outside the low 17 is set
    if (any & ~WE_COUNT_MAX_DEV) {
        w.bad = true;
        return false;
    }
    return true;
}

// ---------------------------------------------------------------- tau-leaping
// An engine for the propagation step that WE leaves open (Sec. IV suggests
// tau-leaping): explicit leaps (Gillespie 2001) with the step bound of Cao,
// Gillespie and Petzold (2006), a run of 100 exact events instead of a leap
// where the bound is below 10 / a0, and the leap halved when a count would go
// negative.

// Exact events taken in a row once the step bound is below 10 / a0.
#define LEAP_SSA_RUN 100

// The walker's leap stream: the four words of Philox(n, slot, iter, 4), in
// turn, as uniforms (r + 0.5) 2^-32.
struct LeapRng {
    uint32_t n, idx, b0, b1, b2, b3;
    uint32_t ssa_left;   // exact events still to take before the step bound is tried again
    __device__ __forceinline__ void reset() {
        n = 0;
        idx = 4;
        ssa_left = 0;
    }
    __device__ __forceinline__ double u(uint32_t slot, uint32_t iter, uint32_t k0, uint32_t k1) {
        if (idx == 4) {
            const U4 r = philox4x32_10(n, slot, iter, 4u, k0, k1);
            b0 = r.x;
            b1 = r.y;
            b2 = r.z;
            b3 = r.w;
            n += 1;
            idx = 0;
        }
        const uint32_t v = idx == 0 ? b0 : idx == 1 ? b1 : idx == 2 ? b2 : b3;
        idx += 1;
        return ((double)v + 0.5) * (1.0 / 4294967296.0);
    }
};

// Poisson(lam): inversion by sequential search below 20; above, Hoermann's
// PTRS transformed rejection (1993).
__device__ __forceinline__ int64_t leap_poisson(LeapRng &g, double lam, uint32_t slot, uint32_t iter, uint32_t k0,
                                                uint32_t k1) {
    if (!(lam > 0.0)) return 0;
    if (lam < 20.0) {
        const double u = g.u(slot, iter, k0, k1);
        double p = exp(-lam), F = p;
        int64_t k = 0;
        while (u > F && k < 1000) {
            k += 1;
            p = p * lam / (double)k;
            F = F + p;
        }
        return k;
    }
    const double slam = sqrt(lam), loglam = log(lam);
    const double b = 0.931 + 2.53 * slam, a = -0.059 + 0.02483 * b;
    const double invalpha = 1.1239 + 1.1328 / (b - 3.4), vr = 0.9277 - 3.6224 / (b - 2.0);
    for (;;) {
        const double U = g.u(slot, iter, k0, k1) - 0.5, V = g.u(slot, iter, k0, k1);
        const double us = 0.5 - fabs(U);
        const int64_t k = (int64_t)floor((2.0 * a / us + b) * U + lam + 0.43);
        if (us >= 0.07 && V <= vr) return k;
        if (k < 0 || (us < 0.013 && V > us)) continue;
        if (log(V) + log(invalpha) - log(a / (us * us) + b) <= -lam + (double)k * loglam - lgamma((double)k + 1.0))
            return k;
    }
}

// g_i of the step bound for a species consumed with highest order hor and
// multiplicity nu there, at count x (Cao, Gillespie, Petzold 2006, Eq. 27).
__device__ __forceinline__ double leap_g(uint32_t hor, uint32_t nu, double x) {
    if (hor <= 1) return 1.0;
    if (hor == 2) return nu == 1 ? 2.0 : 2.0 + 1.0 / (x - 1.0);
    if (nu == 1) return 3.0;
    if (nu == 2) return 1.5 * (2.0 + 1.0 / (x - 1.0));
    return 3.0 + 1.0 / (x - 1.0) + 2.0 / (x - 2.0);
}

// The change of species s by reaction j, from the int8 delta rows.
template <int SMAX, int RMAX, bool HILL>
__device__ __forceinline__ int32_t lane_delta(const LaneNet<SMAX, RMAX, HILL> &net, int j, int s) {
    constexpr int W = LaneRow<SMAX>::W;
    const uint32_t word = LaneNet<SMAX, RMAX, HILL>::REG ? net.drow[LaneNet<SMAX, RMAX, HILL>::REG ? j : 0][s >> 2]
                                                        : (uint32_t)net.rows[j * W + (s >> 2)];
    return (int32_t)(word << (24 - 8 * (s & 3))) >> 24;
}

// Highest order of the reactions consuming each species, and the species'
// multiplicity there (the largest, if several), from the descriptors.
template <int SMAX, int RMAX, bool HILL>
__device__ __forceinline__ void leap_orders(const LaneNet<SMAX, RMAX, HILL> &net, uint32_t (&hor)[SMAX],
                                            uint32_t (&hnu)[SMAX]) {
    constexpr bool REG = LaneNet<SMAX, RMAX, HILL>::REG;
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
        hor[s] = 0;
        hnu[s] = 0;
    }
#pragma unroll
    for (int j = 0; j < RMAX; ++j) {
        if (j < net.R) {
            const LaneRxn d = REG ? net.rx[REG ? j : 0] : lane_rxn(net.desc, j);
            const uint32_t order = d.nu1 + d.nu2;
#pragma unroll
            for (int s = 0; s < SMAX; ++s) {
                const uint32_t nu = (d.nu1 && d.s1 == (uint32_t)s) ? d.nu1 : (d.nu2 && d.s2 == (uint32_t)s) ? d.nu2 : 0u;
                if (nu && (order > hor[s] || (order == hor[s] && nu > hnu[s]))) {
                    hor[s] = order;
                    hnu[s] = nu;
                }
            }
        }
    }
}

// One tau-leaping step (a leap or an exact event); false once the walker's
// interval is over.
template <int SMAX, int RMAX, bool HILL>
__device__ __forceinline__ bool lane_leap_step(const LaneNet<SMAX, RMAX, HILL> &net, LaneWalker &w, LeapRng &g,
                                               int32_t (&x)[SMAX], const uint32_t (&hor)[SMAX],
                                               const uint32_t (&hnu)[SMAX], uint32_t iter, double tau, double eps) {
    constexpr bool REG = LaneNet<SMAX, RMAX, HILL>::REG;
    double prop[RMAX];
    double a0 = 0.0;
#pragma unroll
    for (int j = 0; j < RMAX; ++j) {
        const LaneRxn d = REG ? net.rx[REG ? j : 0] : lane_rxn(net.desc, j);
        prop[j] = 0.0;
        if (REG || j < net.R) {   // zero-rate padding adds +0, as in lane_event
            prop[j] = lane_propensity<SMAX>(d, x);
            a0 = a0 + prop[j];
        }
    }
    if (!(a0 > 0.0)) return false;
    double tp = __builtin_huge_val();
    bool exact = g.ssa_left > 0;
    if (exact) g.ssa_left -= 1;
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
        if (!exact && hor[s] != 0) {
            double mu = 0.0, sig = 0.0;
#pragma unroll
            for (int j = 0; j < RMAX; ++j) {
                if (j < net.R) {
                    const double dd = (double)lane_delta(net, j, s);
                    mu = mu + dd * prop[j];
                    sig = sig + dd * dd * prop[j];
                }
            }
            const double bi = fmax(eps * (double)x[s] / leap_g(hor[s], hnu[s], (double)x[s]), 1.0);
            if (mu != 0.0) tp = fmin(tp, bi / fabs(mu));
            if (sig != 0.0) tp = fmin(tp, bi * bi / sig);
        }
    }
    if (!exact && tp < 10.0 / a0) {
        // leaping does not pay here: this and the next LEAP_SSA_RUN - 1 steps
        // are exact events (a run of about 100, as Cao, Gillespie and Petzold
        // recommend, before the bound is tried again)
        exact = true;
        g.ssa_left = LEAP_SSA_RUN - 1;
    }
    if (exact) {
        // one exact event, as in lane_event
        const U4 r = philox4x32_10(w.e, w.slot, iter, 0u, w.k0, w.k1);
        w.e += 1;
        const double u1 = uniform53(r.x, r.y);
        const double u2 = uniform53(r.z, r.w);
        const double dt = neg_log1m(u1) * recip(a0);
        if (w.t + dt > tau) return false;
        w.t = w.t + dt;
        const double target = u2 * a0;
        // the first j whose running sum exceeds the target (one pass from the
        // last reaction to the first, as in lane_event), else the last
        // reaction with a positive propensity
        double cum[RMAX];
        double c = 0.0;
#pragma unroll
        for (int j = 0; j < RMAX; ++j) {
            if (REG || j < net.R) c = c + prop[j];
            cum[j] = c;
        }
        int32_t jsel = -1;
#pragma unroll
        for (int j = RMAX - 1; j >= 0; --j) jsel = cum[j] > target ? j : jsel;
        if (!(c > target)) {
#pragma unroll
            for (int j = 0; j < RMAX; ++j)
                if ((REG || j < net.R) && prop[j] > 0.0) jsel = j;
        }
        w.fired += 1;
        int32_t any = 0;
#pragma unroll
        for (int s = 0; s < SMAX; ++s) {
            int32_t dv = 0;
#pragma unroll
            for (int j = 0; j < RMAX; ++j)
                if (j == jsel) dv = lane_delta(net, j, s);
            x[s] += dv;
            any |= x[s];
        }
        if (any & ~WE_COUNT_MAX_DEV) {
            w.bad = true;
            return false;
        }
        return true;
    }
    for (;;) {
        const double rest = tau - w.t;
        const bool last = !(tp < rest);
        const double dt = last ? rest : tp;
        int64_t xn[SMAX];
#pragma unroll
        for (int s = 0; s < SMAX; ++s) xn[s] = x[s];
        uint32_t kf = 0;
        // one reaction at a time (a single copy of the sampler); its
        // propensity and delta row are picked by register selects
#pragma unroll 1
        for (int j = 0; j < net.R; ++j) {
            double pj = 0.0;
#pragma unroll
            for (int jj = 0; jj < RMAX; ++jj) pj = (jj == j) ? prop[jj] : pj;
            const int64_t K = leap_poisson(g, pj * dt, w.slot, iter, w.k0, w.k1);
            kf += (uint32_t)K;
#pragma unroll
            for (int s = 0; s < SMAX; ++s) {
                int32_t d = 0;
                if constexpr (REG) {
#pragma unroll
                    for (int jj = 0; jj < RMAX; ++jj) d = (jj == j) ? lane_delta(net, jj, s) : d;
                } else {
                    d = lane_delta(net, j, s);
                }
                xn[s] += K * (int64_t)d;
            }
        }
        bool neg = false, big = false;
#pragma unroll
        for (int s = 0; s < SMAX; ++s) {
            neg = neg || xn[s] < 0;
            big = big || xn[s] > WE_COUNT_MAX_DEV;
        }
        if (neg) {
            tp = tp * 0.5;
            continue;
        }
        if (big) {
            w.bad = true;
            return false;
        }
#pragma unroll
        for (int s = 0; s < SMAX; ++s) x[s] = (int32_t)xn[s];
        w.fired += kf;
        if (last) {
            w.t = tau;
            return false;
        }
        w.t = w.t + dt;
        return w.t < tau;
    }
}

template <int SMAX>
__device__ __forceinline__ void lane_finish(const SimArgs &a, const LaneWalker &w, const int32_t (&x)[SMAX],
                                            int32_t *__restrict__ xr, size_t gslot) {
    if (w.bad) atomicOr(a.err, WE_DERR_OVERFLOW);
#pragma unroll
    for (int s = 0; s < SMAX; ++s)
        if (s < a.S) xr[s] = x[s];
    a.ev_walker[gslot] = w.fired;
}

// One walker through one interval (one lane per walker, fixed assignment).
template <int SMAX, int RMAX>
__device__ __forceinline__ void lane_walker(const SimArgs &a, int32_t *__restrict__ xs, int32_t run,
                                            int32_t k, uint32_t iter, const int32_t *rows) {
    LaneNet<SMAX, RMAX> net;
    net.load(a, rows);
    const size_t gslot = (size_t)run * a.cap + k;
    int32_t *xr = xs + gslot * a.S;
    LaneWalker w;
    int32_t x[SMAX];
    w.begin(x, xr, a.S, (uint32_t)k, a.seeds[run], iter);
    while (lane_event(net, w, x, iter, a.tau)) {
    }
    lane_finish(a, w, x, xr, gslot);
}
