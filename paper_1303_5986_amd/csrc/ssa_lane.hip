// ssa_lane.hip -- Gillespie direct-method SSA, one lane per walker (gfx950).
//
// Each lane carries one walker through one WE interval tau (Sec. II.A, the
// propagation step of the WE procedure in Sec. II.B):
//   1. all propensities a_j = c_j * prod_s C(x_s, nu_js) and their total a0,
//      summed in reaction order;
//   2. waiting time dt = -log(1 - u1) / a0; stop when t + dt > tau (the
//      exponential is memoryless, so the overshoot is simply discarded);
//   3. reaction j = first index whose running sum exceeds u2 * a0;
//   4. x += nu_j, t += dt.
// u1, u2 come from one Philox4x32-10 block at counter (event, slot, iter, 0).
//
// Design for CDNA4: walker state and propensities live in VGPRs, the
// reaction table is wave-uniform and read through scalar loads, and the
// stoichiometric update is a uniform loop over reactions with per-lane
// predication, so no per-lane gather ever touches memory inside the event
// loop.  HBM traffic is one read and one write of the state per interval.
// Walkers are laid out bin-major, so neighbouring lanes have similar total
// propensity and the wave diverges little.
#include "we_common.h"

template <int SMAX, int RMAX>
__global__ __launch_bounds__(256) void ssa_lane_kernel(SimArgs a, int32_t *__restrict__ xs) {
    const int32_t gid = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    const int32_t run = gid / a.cap;
    const int32_t k = gid - run * a.cap;
    if (run >= a.n_runs) return;
    const int32_t n = a.n_walk[run];
    if (k >= n) return;

    const int32_t S = a.S, R = a.R;
    int32_t *xw = xs + ((size_t)run * a.cap + k) * S;
    int32_t x[SMAX];
#pragma unroll
    for (int s = 0; s < SMAX; ++s) x[s] = (s < S) ? xw[s] : 0;

    const uint32_t iter = *a.iter_dev;
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

// Launch helper: picks the smallest register footprint that holds the network.
hipError_t launch_ssa_lane(const SimArgs &a, int32_t *xs, hipStream_t st) {
    const int64_t total = (int64_t)a.n_runs * a.cap;
    const dim3 block(256);
    const dim3 grid((unsigned)((total + 255) / 256));
    if (a.S <= 1 && a.R <= 4)
        hipLaunchKernelGGL((ssa_lane_kernel<1, 4>), grid, block, 0, st, a, xs);
    else if (a.S <= 2 && a.R <= 8)
        hipLaunchKernelGGL((ssa_lane_kernel<2, 8>), grid, block, 0, st, a, xs);
    else if (a.S <= 8 && a.R <= 16)
        hipLaunchKernelGGL((ssa_lane_kernel<8, 16>), grid, block, 0, st, a, xs);
    else if (a.S <= 16 && a.R <= 32)
        hipLaunchKernelGGL((ssa_lane_kernel<16, 32>), grid, block, 0, st, a, xs);
    else if (a.S <= 32 && a.R <= 64)
        hipLaunchKernelGGL((ssa_lane_kernel<32, 64>), grid, block, 0, st, a, xs);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

bool lane_kernel_fits(int32_t S, int32_t R) { return S <= 32 && R <= 64; }
