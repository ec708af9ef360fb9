// ssa_group_body.h -- Gillespie direct-method SSA with L lanes per walker,
// 64 / L walkers per wave (gfx950); shared by ssa_group.hip and batch.hip.
//
// The middle ground between the lane kernels (one lane per walker, tables in
// registers, up to 64 reactions) and the wave kernels (one wave per walker):
// a group of L consecutive lanes (L = 2 ... 32) carries one walker, and lane
// g of the group owns the block of reactions [g B, (g + 1) B), B = ceil(R/L).
// Per event (Sec. II.A):
//   1. each lane sums its block's propensities, recomputed from the walker's
//      counts in LDS (descriptors and changes from the network tables: an
//      LDS copy in ssa_group_kernel when they fit, else through the cache);
//   2. an inclusive scan over the group's L partial sums (log2 L DPP
//      steps) gives a0 and, with a ballot, the lane whose block holds u2 a0;
//      the random numbers of L events are drawn at once, one event per lane
//      of the group, and read by the event that uses them;
//   3. that lane walks its block again to find j;
//   4. the group applies j's changes to the counts, one change per lane.
// The blocks follow the reactions' own order, so j is the reaction the
// sequential direct method picks; u1, u2 come from Philox4x32-10 at (event,
// slot, iteration, 0) with the run's seed as key, as in the oracle, and
// dt = -log(1 - u1) / a0 with the overshoot past tau discarded.  Only the
// summation order differs from the oracle's (partial sums, then a scan), so
// a0 and the running sums may differ in the last bits: an event changes only
// when u2 a0 or t + dt falls within a few ulps of a boundary.
//
// The groups of a wave run their walkers' event loops in lockstep: the loop
// ends when every group's walker has reached tau; a group that is done
// idles.  All cross-lane steps are executed by the whole wave.
#pragma once

#include "queue_first.h"
#include "we_common.h"

#include <algorithm>

// Largest group walker table: counts of 64 / L walkers per wave in LDS.
#define GROUP_LDS_INTS_PER_WAVE 4096

__host__ __device__ inline bool group_lanes_valid(int32_t lanes) {
    return lanes == 2 || lanes == 4 || lanes == 8 || lanes == 16 || lanes == 32;
}

// Whether L lanes per walker fit: the counts of 64 / L walkers per wave,
// GROUP_LDS_INTS_PER_WAVE ints, and 16-bit species ids.
__host__ __device__ inline bool group_kernel_fits(int32_t S, int32_t R, int32_t lanes) {
    return group_lanes_valid(lanes) && R >= 1 && R <= 65535 && S >= 1 && (64 / lanes) * S <= GROUP_LDS_INTS_PER_WAVE;
}

union GroupF64 {
    double d;
    int32_t w[2];
};

// Row-shift DPP move of a double (source outside the 16-lane row: 0).
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ double group_dpp(double v) {
    GroupF64 in, out;
    in.d = v;
    out.w[0] = __builtin_amdgcn_update_dpp(0, in.w[0], CTRL, ROW_MASK, 0xF, BOUND);
    out.w[1] = __builtin_amdgcn_update_dpp(0, in.w[1], CTRL, ROW_MASK, 0xF, BOUND);
    return out.d;
}

// Inclusive scan within groups of L lanes by DPP row shifts (groups of up
// to 16 lie inside a row); a group of 32 adds the first row's total to its
// second row by a row broadcast.  A step adds its source only from the same
// group, so the sums follow a fixed order.
template <int L>
__device__ __forceinline__ double group_scan_incl(double v) {
    const int gl = (int)threadIdx.x & (L - 1);
    double u;
    if (L > 1) { u = group_dpp<0x111, 0xF, true>(v); if (gl >= 1) v += u; }    // row_shr:1
    if (L > 2) { u = group_dpp<0x112, 0xF, true>(v); if (gl >= 2) v += u; }    // row_shr:2
    if (L > 4) { u = group_dpp<0x114, 0xF, true>(v); if (gl >= 4) v += u; }    // row_shr:4
    if (L > 8) { u = group_dpp<0x118, 0xF, true>(v); if (gl >= 8) v += u; }    // row_shr:8
    if (L > 16) { u = group_dpp<0x142, 0xA, false>(v); if (gl >= 16) v += u; } // row_bcast:15, rows 1, 3
    return v;
}

// The network tables a group walker reads: a.desc, a.chg_ptr and a.chg, or
// a block's LDS copy of them.
struct GroupTables {
    const RxnDesc *desc;
    const int32_t *chg_ptr;
    const int32_t *chg;
};

// The walkers in slots k of run `run` for the groups with live set (k may
// differ per group); lx is this group's slice of S counts in LDS.  Every lane
// of the wave must call it.  BR > 0 (blocks of at most BR reactions): each
// lane keeps its block's descriptors in registers for the whole interval and
// its block's propensities from step 1 for step 3, instead of reading the
// descriptors again every event.
template <int L, int BR = 0>
__device__ inline void group_walker(const SimArgs &a, const GroupTables &tb, int32_t *__restrict__ xs, int32_t run,
                                    int32_t k, bool live, uint32_t iter, int32_t *lx) {
    const int lane = threadIdx.x & 63;
    const int gl = lane & (L - 1);
    const int gbase = lane - gl;
    const uint64_t gmask = (L == 64) ? ~0ull : (((1ull << L) - 1ull) << gbase);
    const int32_t S = a.S, R = a.R;
    const int32_t B = (R + L - 1) / L;
    const int32_t r_lo = std::min(R, gl * B), r_hi = std::min(R, r_lo + B);
    int32_t *xw = live ? xs + ((size_t)run * a.cap + k) * S : nullptr;
    if (live)
        for (int32_t s = gl; s < S; s += L) lx[s] = xw[s];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    uint32_t k0 = 0, k1 = 0;
    if (live) {
        const uint64_t seed = a.seeds[run];
        k0 = (uint32_t)seed;
        k1 = (uint32_t)(seed >> 32);
    }
    const double tau = a.tau;
    double t = 0.0;
    uint32_t e = 0, fired = 0;
    bool go = live, bad = false, nosel = false;
    // random numbers of L events at a time: lane gl of a group holds
    // -log(1 - u1) and u2 of the group's event (e & ~(L - 1)) + gl
    double rexp = 0.0, ru2 = 0.0;
    constexpr int NR = BR > 0 ? BR : 1;
    RxnDesc dr[NR];
    double pr[NR];
    if constexpr (BR > 0) {
#pragma unroll
        for (int b = 0; b < NR; ++b) {
            dr[b] = RxnDesc{};
            pr[b] = 0.0;
            if (r_lo + b < r_hi) dr[b] = tb.desc[r_lo + b];
        }
    }
    while (__ballot(go)) {
        // 1. this lane's partial sum over its block
        double part = 0.0;
        if constexpr (BR > 0) {
            if (go)
#pragma unroll
                for (int b = 0; b < NR; ++b)
                    if (r_lo + b < r_hi) {
                        pr[b] = propensity_from(dr[b], (uint32_t)lx[dr[b].s1], (uint32_t)lx[dr[b].s2]);
                        part += pr[b];
                    }
        } else if (go) {
            for (int32_t r = r_lo; r < r_hi; ++r) {
                const RxnDesc d = tb.desc[r];
                part += propensity_from(d, (uint32_t)lx[d.s1], (uint32_t)lx[d.s2]);
            }
        }
        // 2. group scan, a0, waiting time (e is the same on a group's lanes)
        if (go && (e & (L - 1)) == 0u) {
            const U4 rnd = philox4x32_10(e + (uint32_t)gl, (uint32_t)k, iter, 0u, k0, k1);
            rexp = -log(1.0 - uniform53(rnd.x, rnd.y));
            ru2 = uniform53(rnd.z, rnd.w);
        }
        const int src = gbase + (int)(e & (L - 1));
        const double ex = __shfl(rexp, src, 64);
        const double uu = __shfl(ru2, src, 64);
        const double incl = group_scan_incl<L>(part);
        const double a0 = __shfl(incl, gbase + L - 1, 64);
        double u2 = 0.0;
        if (go) {
            if (!(a0 > 0.0)) {
                go = false;
            } else {
                const double dt = ex / a0;
                u2 = uu;
                e += 1;
                if (t + dt > tau) go = false;
                else t = t + dt;
            }
        }
        const double target = u2 * a0;
        const uint64_t over = __ballot(go && incl > target) & gmask;
        const uint64_t pos = __ballot(go && part > 0.0) & gmask;
        // the lane holding the target; rounding past the last block: the
        // last lane with a positive sum
        const int chosen = over ? (__ffsll((long long)over) - 1)
                                : (pos ? 63 - __builtin_clzll(pos) : gbase + L - 1);
        const double excl = incl - part;
        // 3. reaction inside the chosen lane's block
        int32_t j = -1;
        if (go && lane == chosen) {
            const double t2 = target - excl;
            double run_s = 0.0;
            int32_t last = -1;
            if constexpr (BR > 0) {
                // the propensities of step 1, in the same order
#pragma unroll
                for (int b = 0; b < NR; ++b)
                    if (j < 0 && r_lo + b < r_hi && pr[b] > 0.0) {
                        last = r_lo + b;
                        run_s += pr[b];
                        if (run_s > t2) j = r_lo + b;
                    }
            } else {
                for (int32_t r = r_lo; r < r_hi; ++r) {
                    const RxnDesc d = tb.desc[r];
                    const double ar = propensity_from(d, (uint32_t)lx[d.s1], (uint32_t)lx[d.s2]);
                    if (ar > 0.0) {
                        last = r;
                        run_s += ar;
                        if (run_s > t2) {
                            j = r;
                            break;
                        }
                    }
                }
            }
            if (j < 0) j = last;
        }
        j = __shfl(j, chosen, 64);
        if (go && j < 0) {
            nosel = true;
            go = false;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // 4. state update, one change per lane
        bool lbad = false;
        if (go) {
            const int32_t c0 = tb.chg_ptr[j], c1 = tb.chg_ptr[j + 1];
            for (int32_t c = c0 + gl; c < c1; c += L) {
                const int32_t p = tb.chg[c];
                const int32_t sp = change_species(p);
                const int32_t nv = lx[sp] + change_delta(p);
                lx[sp] = nv;
                lbad = lbad || nv < 0 || nv > WE_COUNT_MAX_DEV;
            }
            fired += 1;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (__ballot(lbad) & gmask) {
            bad = true;
            go = false;
        }
    }
    if (live && gl == 0) {
        if (bad) atomicOr(a.err, WE_DERR_OVERFLOW);
        if (nosel) atomicOr(a.err, WE_DERR_SELECT);
    }
    if (live)
        for (int32_t s = gl; s < S; s += L) xw[s] = lx[s];
    if (live && gl == 0) a.ev_walker[(size_t)run * a.cap + k] = fired;
}
