// ssa_wave_fact.h -- the wave-per-walker event loop with every table it
// reads in LDS: reaction descriptors, the factored dependency graph (an
// 8-byte change header per reaction, a start/count word per species and the
// species -> reaction incidence lists, see fact_code in we_common.h) and the
// walker's counts.  No global memory is touched between the first and the
// last event of an interval.
//
// Per event (one 64-wide wave, Sec. II.A's direct method):
//  1. a0 and the chunk holding u2*a0: inclusive scan of the 64 chunk sums
//     (lane c holds the sum of reactions 64c .. 64c+63) and a ballot;
//  2. the reaction inside the chunk: the chunk's 64 propensities from the
//     counts, a second scan and a ballot; each lane also loads its
//     reaction's change header, so the chosen one is two readlanes away;
//     lanes 0-3 then read the changed species' incidence words and counts;
//  3. the dependents: the incidence lists of the changed species, laid end
//     to end over the lanes (one or two rounds of 64); a reaction listed
//     under two changed species counts under the first only.  Each lane reads
//     its reaction's descriptor and counts before the firing and its counts
//     again after it (the firing is one LDS store per changed species; the
//     wave's LDS accesses complete in order);
//  4. each dependent's change of propensity is added to its chunk's sum,
//     held per wave in LDS, by an LDS atomic (ds_add_f64); the chunk lanes
//     then reload their sums.  The LDS unit applies the lanes of one atomic
//     instruction that hit the same address in a fixed order, so a run
//     still repeats bit for bit.
// A reaction whose dependents exceed two rounds rebuilds every chunk sum.
// Every 16 events the wave's issue priority follows its walker's expected
// remaining events (chain_priority), so the longest chains issue first.
#pragma once
#include "ssa_wave_body.h"

#define FACT_DEP_ROUNDS 2

namespace {

union DescBits {
    RxnDesc d;
    uint4 u;
};

__device__ __forceinline__ RxnDesc desc_of(const uint4 &u) {
    DescBits b;
    b.u = u;
    return b.d;
}

__device__ __forceinline__ double prop_u4(const uint4 &u, uint32_t x1, uint32_t x2) {
    return propensity_from(desc_of(u), x1, x2);
}

}  // namespace

struct FactTables {
    const uint4 *d;        // LDS [R] descriptors
    const uint2 *h;        // LDS [R] change headers
    const uint32_t *tab;   // LDS [S] incidence start | count << 16
    const uint16_t *inc;   // LDS [n_inc] incidence lists
};

// One walker through one interval on the calling wave; lchunk (64 doubles,
// the chunk sums) and lx (S ints) are this wave's LDS slices.
__device__ inline void wave_walker_fact(const SimArgs &a, const FactTables &tab, int32_t *__restrict__ xs,
                                        int32_t run, int32_t k, uint32_t iter, double *lchunk, int32_t *lx) {
    const int lane = threadIdx.x & 63;
    const int32_t S = a.S, R = a.R;
    const int32_t K = (R + 63) >> 6;
    int32_t *xw = xs + ((size_t)run * a.cap + k) * S;
    for (int s = lane; s < S; s += 64) lx[s] = xw[s];
    __builtin_amdgcn_wave_barrier();

    // chunk sums from scratch
    auto rebuild = [&]() {
        double cs_ = 0.0;
        for (int c = 0; c < K; ++c) {
            const int r = c * 64 + lane;
            double v = 0.0;
            if (r < R) {
                const RxnDesc d = desc_of(tab.d[r]);
                v = propensity_from(d, (uint32_t)lx[d.s1], (uint32_t)lx[d.s2]);
            }
            const double tot = lane_value(scan_incl(v), 63);
            if (lane == c) cs_ = tot;
        }
        return cs_;
    };
    double csum = rebuild();
    lchunk[lane] = csum;

    const uint64_t seed = a.seeds[run];
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const double tau = a.tau;
    double t = 0.0;
    uint32_t e = 0, fired = 0;
    bool bad = false;
    double rexp = 0.0, ru2 = 0.0;   // random numbers of 64 events, one per lane

    for (;;) {
        const double P = scan_incl(csum);
        const double a0 = lane_value(P, 63);
        if (!(a0 > 0.0)) break;
        if ((e & 63u) == 0u) {
            const U4 rnd = philox4x32_10(e + (uint32_t)lane, (uint32_t)k, iter, 0u, k0, k1);
            rexp = -log(1.0 - uniform53(rnd.x, rnd.y));
            ru2 = uniform53(rnd.z, rnd.w);
        }
        const double ex = lane_value(rexp, (int)(e & 63u));
        const double u2 = lane_value(ru2, (int)(e & 63u));
        e += 1;
        const double dt = ex * recip(a0);
        if (t + dt > tau) break;
        t = t + dt;
        if ((e & 15u) == 1u) chain_priority((tau - t) * a0);
        const double target = u2 * a0;

        // chunk holding the target
        const unsigned long long m1 = __ballot(P > target);
        int cs = m1 ? (__ffsll((long long)m1) - 1) : last_set(__ballot(csum > 0.0));
        if (cs < 0) cs = 0;
        cs = __builtin_amdgcn_readfirstlane(cs);
        const double base = lane_value(P - csum, cs);
        const double target2 = target - base;
        // reaction inside the chunk, with every lane's descriptor and header
        const int rsel = cs * 64 + lane;
        double v = 0.0;
        uint4 dsel{0u, 0u, 0u, 0u};
        uint2 hsel{0u, 0u};
        if (rsel < R) {
            dsel = tab.d[rsel];
            hsel = tab.h[rsel];
            const RxnDesc d = desc_of(dsel);
            v = propensity_from(d, (uint32_t)lx[d.s1], (uint32_t)lx[d.s2]);
        }
        const double Q = scan_incl(v);
        const unsigned long long m2 = __ballot(Q > target2);
        const int ls = m2 ? (__ffsll((long long)m2) - 1) : last_set(__ballot(v > 0.0));
        if (ls < 0) {              // chunk sum drifted above an all-zero chunk
            if (lane == 0) atomicOr(a.err, WE_DERR_SELECT);
            break;
        }
        // the fired reaction's changes (wave-uniform)
        const int32_t nchg = (int32_t)((__builtin_amdgcn_readlane((int)dsel.w, ls) >> 16) & 0xFF);
        const uint32_t hlo = (uint32_t)__builtin_amdgcn_readlane((int)hsel.x, ls);
        const uint32_t hhi = (uint32_t)__builtin_amdgcn_readlane((int)hsel.y, ls);
        const int32_t sp0 = fact_species(hlo), sp1 = fact_species(hlo >> 16), sp2 = fact_species(hhi),
                      sp3 = fact_species(hhi >> 16);
        const int32_t dl0 = fact_delta(hlo), dl1 = fact_delta(hlo >> 16), dl2 = fact_delta(hhi),
                      dl3 = fact_delta(hhi >> 16);
        // lanes 0..nchg-1: the changed species' old counts and incidence words
        const int32_t spl = lane == 0 ? sp0 : lane == 1 ? sp1 : lane == 2 ? sp2 : sp3;
        const int32_t dll = lane == 0 ? dl0 : lane == 1 ? dl1 : lane == 2 ? dl2 : dl3;
        int32_t xold = 0;
        uint32_t iw = 0u;
        if (lane < nchg) {
            xold = lx[spl];
            iw = tab.tab[spl];
        }
        const uint32_t iw0 = (uint32_t)__builtin_amdgcn_readlane((int)iw, 0);
        const uint32_t iw1 = (uint32_t)__builtin_amdgcn_readlane((int)iw, 1);
        const uint32_t iw2 = (uint32_t)__builtin_amdgcn_readlane((int)iw, 2);
        const uint32_t iw3 = (uint32_t)__builtin_amdgcn_readlane((int)iw, 3);
        const int32_t n0 = (int32_t)(iw0 >> 16), n1 = (int32_t)(iw1 >> 16), n2 = (int32_t)(iw2 >> 16),
                      n3 = (int32_t)(iw3 >> 16);
        const int32_t o1 = n0, o2 = o1 + n1, o3 = o2 + n2, nd = o3 + n3;
        const int32_t b0 = (int32_t)(iw0 & 0xFFFFu), b1 = (int32_t)(iw1 & 0xFFFFu), b2 = (int32_t)(iw2 & 0xFFFFu),
                      b3 = (int32_t)(iw3 & 0xFFFFu);

        // the dependents' descriptors and counts, before the firing
        const bool fits = nd <= 64 * FACT_DEP_ROUNDS;
        uint4 dq[FACT_DEP_ROUNDS];
        int32_t x1q[FACT_DEP_ROUNDS], x2q[FACT_DEP_ROUNDS], chk[FACT_DEP_ROUNDS], kq[FACT_DEP_ROUNDS];
#pragma unroll
        for (int q = 0; q < FACT_DEP_ROUNDS; ++q) {
            chk[q] = -1;
            kq[q] = 0;
            x1q[q] = 0;
            x2q[q] = 0;
            dq[q] = uint4{0u, 0u, 0u, 0u};
            const int32_t idx = q * 64 + lane;
            if (q > 0 && nd <= 64 * q) continue;   // uniform: no lane has a dependent here
            if (fits && idx < nd) {
                const int32_t kk = (idx >= o1 ? 1 : 0) + (idx >= o2 ? 1 : 0) + (idx >= o3 ? 1 : 0);
                const int32_t beg = kk == 0 ? b0 : kk == 1 ? b1 : kk == 2 ? b2 : b3;
                const int32_t off = kk == 0 ? 0 : kk == 1 ? o1 : kk == 2 ? o2 : o3;
                const int32_t r = tab.inc[beg + idx - off];
                dq[q] = tab.d[r];
                const RxnDesc d = desc_of(dq[q]);
                x1q[q] = lx[d.s1];
                x2q[q] = lx[d.s2];
                kq[q] = kk;
                chk[q] = r >> 6;
            }
        }
        // fire j (the dependents' old counts were read above)
        bool lbad = false;
        if (lane < nchg) {
            const int32_t nv = xold + dll;
            lx[spl] = nv;
            lbad = (nv < 0) || (nv > WE_COUNT_MAX_DEV);
        }
        fired += 1;
        if (__ballot(lbad)) { bad = true; break; }

        __builtin_amdgcn_wave_barrier();
        if (!fits) {
            csum = rebuild();
            lchunk[lane] = csum;
            continue;
        }
#pragma unroll
        for (int q = 0; q < FACT_DEP_ROUNDS; ++q) {
            if (q * 64 >= nd) break;
            if (chk[q] >= 0) {
                const RxnDesc d = desc_of(dq[q]);
                // listed under an earlier changed species too: counted there
                // (its other reactant is one of sp0 .. sp(k-1))
                const int32_t kk = kq[q];
                const int32_t spk = kk == 0 ? sp0 : kk == 1 ? sp1 : kk == 2 ? sp2 : sp3;
                const int32_t other = d.s1 == spk ? (int32_t)d.s2 : (int32_t)d.s1;
                const bool dup = d.nu2 > 0 && ((kk >= 1 && other == sp0) || (kk >= 2 && other == sp1) ||
                                               (kk >= 3 && other == sp2));
                if (!dup) {
                    const double before = propensity_from(d, (uint32_t)x1q[q], (uint32_t)x2q[q]);
                    const double after = propensity_from(d, (uint32_t)lx[d.s1], (uint32_t)lx[d.s2]);
                    lds_add_f64(&lchunk[chk[q]], after - before);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        csum = lchunk[lane];
    }
    if (bad && lane == 0) atomicOr(a.err, WE_DERR_OVERFLOW);
    __builtin_amdgcn_wave_barrier();
    for (int s = lane; s < S; s += 64) xw[s] = lx[s];
    if (lane == 0) a.ev_walker[(size_t)run * a.cap + k] = fired;
}
