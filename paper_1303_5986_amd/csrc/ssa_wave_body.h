// ssa_wave_body.h -- the wave-per-walker event loop, shared by the per-sim
// kernel and the batched persistent kernel.
//
// Cross-lane work uses the CDNA data-parallel primitives directly:
//  * inclusive prefix sums of FP64 values: four DPP row shifts (1, 2, 4, 8)
//    build scans inside each 16-lane row, then the row_bcast:15 and
//    row_bcast:31 broadcasts carry row totals across the wave -- six steps
//    of two 32-bit DPP moves and one add, no LDS round trip;
//  * broadcasts of one lane: v_readlane;
//  * the dependents' propensity changes go into the per-wave chunk sums in
//    LDS by ds_add_f64, one instruction per round of 64 dependents.
// Per event the dependent loads from global memory are: the descriptors of
// the chosen chunk (64 lanes, one 16-byte load each), then one packed
// header of the chosen reaction, then its dependency entries (each carrying
// the descriptor of the reaction it names) together with its changes.
#pragma once
#include "queue_first.h"
#include "we_common.h"

#define WAVE_WALKERS_PER_BLOCK 4
#define WAVE_DEP_ROUNDS 2

namespace {

template <class D>
__device__ __forceinline__ double prop_lds(const D &d, const int32_t *lx) {
    return propensity_from(d, (uint32_t)lx[d.s1], (uint32_t)lx[d.s2]);
}

union F64Bits {
    double d;
    int32_t w[2];
};

template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ double dpp_f64(double v) {
    F64Bits in, out;
    in.d = v;
    out.w[0] = __builtin_amdgcn_update_dpp(0, in.w[0], CTRL, ROW_MASK, 0xF, BOUND);
    out.w[1] = __builtin_amdgcn_update_dpp(0, in.w[1], CTRL, ROW_MASK, 0xF, BOUND);
    return out.d;
}

// Inclusive prefix sum over the 64 lanes (fixed order, reproducible).
__device__ __forceinline__ double scan_incl(double v) {
    v = v + dpp_f64<0x111, 0xF, true>(v);    // row_shr:1
    v = v + dpp_f64<0x112, 0xF, true>(v);    // row_shr:2
    v = v + dpp_f64<0x114, 0xF, true>(v);    // row_shr:4
    v = v + dpp_f64<0x118, 0xF, true>(v);    // row_shr:8
    v = v + dpp_f64<0x142, 0xA, false>(v);   // row_bcast:15 into rows 1 and 3
    v = v + dpp_f64<0x143, 0xC, false>(v);   // row_bcast:31 into rows 2 and 3
    return v;
}

__device__ __forceinline__ double lane_value(double v, int lane) {
    F64Bits in, out;
    in.d = v;
    out.w[0] = __builtin_amdgcn_readlane(in.w[0], lane);
    out.w[1] = __builtin_amdgcn_readlane(in.w[1], lane);
    return out.d;
}

__device__ __forceinline__ int32_t last_set(unsigned long long m) {
    return m ? 63 - __clzll((long long)m) : -1;
}

// Issue priority of the calling wave from its walker's expected remaining
// events in the interval, (tau - t) * a0: longest remaining chain first.  A
// launch lasts as long as its longest walker chain, and waves sharing a SIMD
// compete for issue; the wave with more left to do then issues first and the
// others fill its dependency stalls.  Four levels (s_setprio 0..3), at 16,
// 48 and 96 remaining events.  Scheduling only: no result depends on it.
__device__ __forceinline__ void chain_priority(double rem) {
    if (rem > 96.0)
        __builtin_amdgcn_s_setprio(3);
    else if (rem > 48.0)
        __builtin_amdgcn_s_setprio(2);
    else if (rem > 16.0)
        __builtin_amdgcn_s_setprio(1);
    else
        __builtin_amdgcn_s_setprio(0);
}

// Sum of all 64 propensities of chunk c (last lane of the scan).
template <class T>
__device__ __forceinline__ double chunk_total(const T &tab, int32_t R, const int32_t *lx, int c, int lane) {
    const int r = c * 64 + lane;
    double v = 0.0;
    if (r < R) v = prop_lds(tab.desc(r), lx);
    return lane_value(scan_incl(v), 63);
}

// Add v to a double in LDS with one ds_add_f64 (no return value).  The LDS
// unit applies the lanes of one such instruction that hit the same address
// in a fixed order, so a sum built this way repeats bit for bit.
__device__ __forceinline__ void lds_add_f64(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Add each lane's propensity change dv of dependent reaction rr (rr < 0 for
// idle lanes) to its chunk's sum.
__device__ __forceinline__ void add_chunk_deltas(double *lchunk, int rr, double dv) {
    if (rr >= 0) lds_add_f64(&lchunk[rr >> 6], dv);
}

}  // namespace

// Where the wave reads the network from.
//  GlobalTables: descriptors, reaction headers and dependency entries (each
//    with its reaction's descriptor inline) from global memory;
//  LdsTables: descriptors from the block's LDS copy, headers from LDS or
//    global memory, the dependency lists (16-bit reaction ids) from global
//    memory and the dependents' descriptors from LDS.
struct GlobalTables {
    const RxnDesc *__restrict__ d;
    const RxnInfo *__restrict__ h;
    const DepEntry *__restrict__ e;
    __device__ __forceinline__ RxnDesc desc(int r) const { return d[r]; }
    __device__ __forceinline__ RxnInfo info(int j) const { return h[j]; }
    __device__ __forceinline__ DepEntry dep(int i) const { return e[i]; }
};

struct LdsTables {
    const RxnDesc *d;                  // LDS
    const RxnInfo *h;                  // LDS or global
    const uint16_t *__restrict__ ids;  // global
    __device__ __forceinline__ RxnDesc desc(int r) const { return d[r]; }
    __device__ __forceinline__ RxnInfo info(int j) const { return h[j]; }
    __device__ __forceinline__ DepEntry dep(int i) const {
        const int r = ids[i];
        const RxnDesc q = d[r];
        DepEntry o;
        o.c = q.c;
        o.s1 = q.s1;
        o.s2 = q.s2;
        o.nu1 = q.nu1;
        o.nu2 = q.nu2;
        o.r = (uint16_t)r;
        return o;
    }
};

// One walker through one interval on the calling wave; lchunk (64 doubles)
// and lx (S ints) are this wave's LDS slices.
template <class T>
__device__ inline void wave_walker_t(const SimArgs &a, const T &tab, int32_t *__restrict__ xs, int32_t run,
                                     int32_t k, uint32_t iter, double *lchunk, int32_t *lx) {
    const int lane = threadIdx.x & 63;
    const int32_t S = a.S, R = a.R;
    const int32_t K = (R + 63) >> 6;
    int32_t *xw = xs + ((size_t)run * a.cap + k) * S;
    for (int s = lane; s < S; s += 64) lx[s] = xw[s];
    __builtin_amdgcn_wave_barrier();

    // chunk sums from scratch
    double csum = 0.0;
    for (int c = 0; c < K; ++c) {
        const double tot = chunk_total(tab, R, lx, c, lane);
        if (lane == c) csum = tot;
    }
    lchunk[lane] = csum;

    const uint64_t seed = a.seeds[run];
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const double tau = a.tau;
    double t = 0.0;
    uint32_t e = 0, fired = 0;
    bool bad = false;
    // random numbers of 64 events at a time, one event per lane: lane l holds
    // -log(1 - u1) and u2 of event (e & ~63) + l.  The general-purpose log is
    // kept here: it runs once per 64 events, and the lane kernels' shorter one
    // would hold its coefficients in registers across the whole event loop
    // (132 VGPRs instead of 124, one block per CU instead of two).
    double rexp = 0.0, ru2 = 0.0;

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
        const double dt = ex / a0;
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
        // reaction inside the chunk; each lane also fetches its reaction's
        // header, so the chosen one is a readlane away once j is known
        const int rsel = cs * 64 + lane;
        double v = 0.0;
        RxnInfo hinfo{0, 0, 0, 0};
        if (rsel < R) {
            hinfo = tab.info(rsel);
            v = prop_lds(tab.desc(rsel), lx);
        }
        const double Q = scan_incl(v);
        const unsigned long long m2 = __ballot(Q > target2);
        const int ls = m2 ? (__ffsll((long long)m2) - 1) : last_set(__ballot(v > 0.0));
        if (ls < 0) {              // chunk sum drifted above an all-zero chunk
            if (lane == 0) atomicOr(a.err, WE_DERR_SELECT);
            break;
        }
        // header of j; its dependents (with descriptors) and changes
        RxnInfo info;
        info.dep_begin = __builtin_amdgcn_readlane(hinfo.dep_begin, ls);
        info.dep_count = __builtin_amdgcn_readlane(hinfo.dep_count, ls);
        info.chg_begin = __builtin_amdgcn_readlane(hinfo.chg_begin, ls);
        info.chg_count = __builtin_amdgcn_readlane(hinfo.chg_count, ls);
        const int32_t nd = info.dep_count;
        const int nround = (nd + 63) >> 6;
        int32_t pc = 0;
        if (lane < info.chg_count) pc = a.chg[info.chg_begin + lane];
        int rr[WAVE_DEP_ROUNDS];
        double old[WAVE_DEP_ROUNDS];
        DepEntry de[WAVE_DEP_ROUNDS];
        if (nround <= WAVE_DEP_ROUNDS) {
#pragma unroll
            for (int q = 0; q < WAVE_DEP_ROUNDS; ++q) {
                rr[q] = -1;
                old[q] = 0.0;
                if (q < nround) {
                    const int idx = q * 64 + lane;
                    if (idx < nd) {
                        de[q] = tab.dep(info.dep_begin + idx);
                        rr[q] = de[q].r;
                        old[q] = prop_lds(de[q], lx);
                    }
                }
            }
        }
        // fire j
        __builtin_amdgcn_wave_barrier();
        bool lbad = false;
        if (lane < info.chg_count) {
            const int32_t s = change_species(pc);
            const int32_t nv = lx[s] + change_delta(pc);
            lx[s] = nv;
            lbad = (nv < 0) || (nv > WE_COUNT_MAX_DEV);
        }
        __builtin_amdgcn_wave_barrier();
        fired += 1;
        if (__ballot(lbad)) { bad = true; break; }

        // fold the dependents' changes into the chunk sums
        if (nround <= WAVE_DEP_ROUNDS) {
#pragma unroll
            for (int q = 0; q < WAVE_DEP_ROUNDS; ++q) {
                if (q < nround) {
                    double dv = 0.0;
                    if (rr[q] >= 0) dv = prop_lds(de[q], lx) - old[q];
                    add_chunk_deltas(lchunk, rr[q], dv);
                    __builtin_amdgcn_wave_barrier();
                }
            }
            csum = lchunk[lane];
        } else {
            // very long dependency list: rebuild every chunk sum
            csum = 0.0;
            for (int c = 0; c < K; ++c) {
                const double tot = chunk_total(tab, R, lx, c, lane);
                if (lane == c) csum = tot;
            }
            lchunk[lane] = csum;
        }
    }
    if (bad && lane == 0) atomicOr(a.err, WE_DERR_OVERFLOW);
    __builtin_amdgcn_wave_barrier();
    for (int s = lane; s < S; s += 64) xw[s] = lx[s];
    if (lane == 0) a.ev_walker[(size_t)run * a.cap + k] = fired;
}

__device__ inline void wave_walker(const SimArgs &a, int32_t *__restrict__ xs, int32_t run, int32_t k,
                                   uint32_t iter, double *lchunk, int32_t *lx) {
    GlobalTables tab;
    tab.d = a.desc;
    tab.h = a.rinfo;
    tab.e = a.deps;
    wave_walker_t(a, tab, xs, run, k, iter, lchunk, lx);
}
