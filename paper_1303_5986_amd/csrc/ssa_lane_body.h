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

// One walker's progress through the current interval (its counts live in a
// separate register array, which keeps this struct out of LDS).
struct LaneWalker {
    double t;
    uint32_t e, fired;
    uint32_t slot, k0, k1;
    bool bad;

    template <int SMAX>
    __device__ __forceinline__ void begin(int32_t (&x)[SMAX], const int32_t *__restrict__ xr, int32_t S, uint32_t k,
                                          uint64_t seed) {
#pragma unroll
        for (int s = 0; s < SMAX; ++s) x[s] = (s < S) ? xr[s] : 0;
        t = 0.0;
        e = 0;
        fired = 0;
        slot = k;
        k0 = (uint32_t)seed;
        k1 = (uint32_t)(seed >> 32);
        bad = false;
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
        if (j < net.R) {
            prop[j] = lane_propensity<SMAX>(d, x);
            if constexpr (HILL) prop[j] = lane_repress<SMAX>(prop[j], REG ? net.hl[REG ? j : 0] : lane_hill(net.hill, j), x);
            a0 = a0 + prop[j];
        }
    }
    if (!(a0 > 0.0)) return false;
    const U4 r = philox4x32_10(w.e, w.slot, iter, 0u, w.k0, w.k1);
    w.e += 1;
    const double u1 = uniform53(r.x, r.y);
    const double u2 = uniform53(r.z, r.w);
    const double dt = -log(1.0 - u1) / a0;
    if (w.t + dt > tau) return false;
    w.t = w.t + dt;
    const double target = u2 * a0;
    double cum = 0.0;
    int32_t jsel = -1, last_pos = -1;
    uint32_t dsel[W];
#pragma unroll
    for (int q = 0; q < W; ++q) dsel[q] = 0u;
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
    if (jsel < 0) {   // rounding left the target above the running sum
        jsel = last_pos;
        if constexpr (REG) {
#pragma unroll
            for (int q = 0; q < W; ++q) dsel[q] = (uint32_t)net.dpack[jsel * WE_DPACK_WORDS + q];
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
    w.begin(x, xr, a.S, (uint32_t)k, a.seeds[run]);
    while (lane_event(net, w, x, iter, a.tau)) {
    }
    lane_finish(a, w, x, xr, gslot);
}
