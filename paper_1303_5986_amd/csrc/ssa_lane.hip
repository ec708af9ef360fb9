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
// reaction table is wave-uniform (scalar loads), and the state change of the
// chosen reaction is an int8 delta row picked by register selects (up to 8
// reactions) or read from the wave's LDS copy of the rows, so nothing in the
// event loop waits on global memory.  HBM traffic is one read and one write
// of the state per interval.  Walkers are laid out bin-major, so neighbouring
// lanes have similar total propensity and the wave diverges little.
#include "ssa_lane_body.h"

template <int SMAX, int RMAX>
__global__ __launch_bounds__(256) void ssa_lane_kernel(SimArgs a, int32_t *__restrict__ xs) {
    constexpr bool REG = RMAX <= LANE_REG_RMAX;
    constexpr int ROWS = REG ? 1 : RMAX * LaneRow<SMAX>::W;
    __shared__ int32_t rows[4 * ROWS];
    int32_t *wrows = rows + (threadIdx.x >> 6) * ROWS;
    if constexpr (!REG) lane_stage_rows<SMAX>(a, wrows);
    const int32_t gid = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    const int32_t run = gid / a.cap;
    const int32_t k = gid - run * a.cap;
    if (run >= a.n_runs) return;
    if (k >= a.n_walk[run]) return;
    lane_walker<SMAX, RMAX>(a, xs, run, k, *a.iter_dev, wrows);
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

// Deltas travel as int8, so every change must lie in [-128, 127].
bool lane_kernel_fits(int32_t S, int32_t R, int32_t max_delta) {
    return S <= 32 && R <= 64 && max_delta <= 127;
}
