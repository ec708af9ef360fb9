// ssa_wave.hip -- Gillespie direct-method SSA, one 64-wide wavefront per
// walker (gfx950), for networks with up to 4096 reactions.
//
// The method per event is the same as the lane kernel (Sec. II.A): total
// propensity a0, dt = -log(1 - u1)/a0 with the overshoot past tau
// discarded, reaction j = first index whose running sum exceeds u2 * a0,
// x += nu_j, with u1, u2 from Philox4x32-10 at (event, slot, iter, 0).
// What changes is how the work is spread over the wave:
//
//  * reactions are grouped in chunks of 64 (reaction r is lane r % 64 of
//    chunk r / 64); the wave keeps one FP64 partial sum per chunk, lane c
//    holding chunk c's sum (so up to 64 chunks = 4096 reactions);
//  * a0 and the chunk holding u2*a0 come from one inclusive prefix scan of
//    the chunk sums across the wave plus a ballot; the reaction inside the
//    chunk from a second scan over that chunk's 64 propensities,
//    recomputed from the counts -- two wave-level prefix scans per event
//    instead of an O(R) sequential pass;
//  * after firing j, only the reactions whose propensity can change (the
//    dependency list of j: every reaction taking a changed species as a
//    reactant, sorted and without repeats) are re-evaluated, one per lane,
//    and their propensity changes are added to the chunk sums by a
//    segmented reduction in a fixed order, so results are reproducible;
//  * the chunk sums are rebuilt from scratch at the start of every interval,
//    which bounds the rounding drift of the incremental updates to one
//    interval.
//
// Memory: walker counts (int32) and chunk sums live in LDS (about 2 KB per
// walker at 354 species), so a CU holds many walkers at once; reaction
// descriptors, stoichiometry and dependency lists are read from global
// memory, where the whole network (~0.3 MB at 3680 reactions) stays
// resident in the L2 caches.  No per-reaction propensity array is stored.
//
// Summation order differs from the sequential order of the oracle (chunked
// scans), so a0 and the running sums can differ in the last bits; an event
// changes only if u2*a0 or t+dt falls within a few ulps of a boundary.
#include "ssa_wave_body.h"

__global__ __launch_bounds__(256) void ssa_wave_kernel(SimArgs a, int32_t *__restrict__ xs,
                                                       int32_t s_pad) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int wv = threadIdx.x >> 6;
    double *lchunk = reinterpret_cast<double *>(smem) + wv * 64;
    int32_t *lx = reinterpret_cast<int32_t *>(smem + WAVE_WALKERS_PER_BLOCK * 64 * sizeof(double)) +
                  wv * s_pad;
    const int64_t gw = (int64_t)blockIdx.x * WAVE_WALKERS_PER_BLOCK + wv;
    const int32_t run = (int32_t)(gw / a.cap);
    const int32_t k = (int32_t)(gw - (int64_t)run * a.cap);
    if (run >= a.n_runs) return;
    if (k >= a.n_walk[run]) return;
    wave_walker(a, xs, run, k, *a.iter_dev, lchunk, lx);
}

bool wave_kernel_fits(int32_t S, int32_t R) { return R <= 4096 && S <= 8192; }

hipError_t launch_ssa_wave(const SimArgs &a, int32_t *xs, hipStream_t st) {
    if (!wave_kernel_fits(a.S, a.R)) return hipErrorInvalidValue;
    const int32_t s_pad = (a.S + 3) & ~3;
    const size_t shmem = WAVE_WALKERS_PER_BLOCK * (64 * sizeof(double) + sizeof(int32_t) * (size_t)s_pad);
    const int64_t walkers = (int64_t)a.n_runs * a.cap;
    const unsigned blocks = (unsigned)((walkers + WAVE_WALKERS_PER_BLOCK - 1) / WAVE_WALKERS_PER_BLOCK);
    hipLaunchKernelGGL(ssa_wave_kernel, dim3(blocks), dim3(64 * WAVE_WALKERS_PER_BLOCK), shmem, st, a,
                       xs, s_pad);
    return hipGetLastError();
}
