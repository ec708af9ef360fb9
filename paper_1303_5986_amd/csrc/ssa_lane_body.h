// ssa_lane_body.h -- the lane-per-walker event loop (one walker through one
// interval), shared by the per-sim kernel and the batched persistent kernel.
#pragma once
#include "we_common.h"

template <int SMAX, int RMAX>
__device__ __forceinline__ void lane_walker(const SimArgs &a, int32_t *__restrict__ xs, int32_t run,
                                            int32_t k, uint32_t iter) {
    const int32_t S = a.S, R = a.R;
    int32_t *xw = xs + ((size_t)run * a.cap + k) * S;
    int32_t x[SMAX];
#pragma unroll
    for (int s = 0; s < SMAX; ++s) x[s] = (s < S) ? xw[s] : 0;

    const uint64_t seed = a.seeds[run];
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const double tau = a.tau;
    double t = 0.0;
    uint32_t e = 0, fired = 0;
    int32_t bad = 0;
    double prop[RMAX];

    for (;;) {
        double a0 = 0.0;
#pragma unroll
        for (int j = 0; j < RMAX; ++j) {
            if (j < R) {
                const RxnDesc d = a.desc[j];
                prop[j] = propensity_from(d, (uint32_t)x[d.s1], (uint32_t)x[d.s2]);
                a0 = a0 + prop[j];
            } else {
                prop[j] = 0.0;
            }
        }
        if (!(a0 > 0.0)) break;
        const U4 r = philox4x32_10(e, (uint32_t)k, iter, 0u, k0, k1);
        e += 1;
        const double u1 = uniform53(r.x, r.y);
        const double u2 = uniform53(r.z, r.w);
        const double dt = -log(1.0 - u1) / a0;
        if (t + dt > tau) break;
        t = t + dt;
        const double target = u2 * a0;
        double cum = 0.0;
        int32_t jsel = -1, last_pos = -1;
#pragma unroll
        for (int j = 0; j < RMAX; ++j) {
            if (j < R) {
                cum = cum + prop[j];
                if (prop[j] > 0.0) last_pos = j;
                if (jsel < 0 && cum > target) jsel = j;
            }
        }
        if (jsel < 0) jsel = last_pos;
        fired += 1;
        // apply nu_jsel: uniform loop over reactions, lane-predicated
        for (int j = 0; j < R; ++j) {
            if (j == jsel) {
                const int32_t p0 = a.chg_ptr[j], p1 = a.chg_ptr[j + 1];
                for (int32_t p = p0; p < p1; ++p) {
                    const int32_t c = a.chg[p];
                    const int32_t s = change_species(c);
                    const int32_t v = x[s] + change_delta(c);
                    x[s] = v;
                    bad |= (v < 0) | (v > WE_COUNT_MAX_DEV);
                }
            }
        }
        if (bad) break;
    }
    if (bad) atomicOr(a.err, WE_DERR_OVERFLOW);
#pragma unroll
    for (int s = 0; s < SMAX; ++s)
        if (s < S) xw[s] = x[s];
    a.ev_walker[(size_t)run * a.cap + k] = fired;
}

