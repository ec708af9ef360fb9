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
//    and their propensity changes are added to the chunk sums, held in
//    LDS, by LDS atomic adds (one ds_add_f64 per lane; the LDS unit applies
//    the lanes of one instruction in a fixed order, so results repeat bit
//    for bit);
//  * the chunk sums are rebuilt from scratch at the start of every interval,
//    which bounds the rounding drift of the incremental updates to one
//    interval.
//
// Memory: walker counts (int32) and chunk sums live in LDS (about 2 KB per
// walker at 354 species).  Two kernels share that scheme:
//  * ssa_wave_fact_kernel keeps every table in LDS: descriptors, an 8-byte
//    change header per reaction and the factored dependency graph (per
//    species, the reactions taking it as a reactant); nothing in its event
//    loop reads global memory;
//  * ssa_wave_lds_kernel keeps the descriptors (and, when they fit, 16-byte
//    reaction headers) in LDS and reads each fired reaction's sorted
//    dependency list and changes from global memory, where they stay in L2;
//    its smaller tables leave room for two blocks per CU.
// No per-reaction propensity array is stored.
//
// Summation order differs from the sequential order of the oracle (chunked
// scans), so a0 and the running sums can differ in the last bits; an event
// changes only if u2*a0 or t+dt falls within a few ulps of a boundary.
#include "ssa_wave_body.h"
#include "ssa_wave_fact.h"

#include <algorithm>

// LDS-table variant: the block copies the descriptor table (16 bytes per
// reaction, 59 KB at 3680 reactions) into LDS once -- and, with HDR, the
// reaction headers too (another 16 bytes per reaction) -- and its waves then
// take walkers from the work queue until it is empty.  Without HDR two
// blocks of 8 walkers fit a CU instead of one, which pays when there are
// more walkers than one block per CU can hold; with HDR the headers need no
// global load.  Per event the remaining global traffic is the chosen chunk's
// 64 headers (without HDR, fetched with the descriptors, in parallel) and the
// fired reaction's dependency ids and changes (16-bit ids: 0.3 MB for the
// whole 3680-reaction network, which stays in L2).
#define WAVE_LDS_MAX_WAVES 8
#define WAVE_LDS_BYTES (160 * 1024)

// At least 4 waves per SIMD (two blocks per CU), so at most 128 VGPRs: one
// more register and the <false> variant drops to one block per CU (measured:
// 132 VGPRs took 8 replicas of the 3680-reaction network from 1.41 to 2.14 ms
// per launch).
template <bool HDR>
__global__ __launch_bounds__(64 * WAVE_LDS_MAX_WAVES, 4) void ssa_wave_lds_kernel(SimArgs a, int32_t *__restrict__ xs,
                                                                                 int32_t s_pad) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t R = a.R;
    RxnDesc *ldesc = reinterpret_cast<RxnDesc *>(smem);
    RxnInfo *linfo = reinterpret_cast<RxnInfo *>(smem + 16 * (size_t)R);
    unsigned char *wbase = smem + (HDR ? 32 : 16) * (size_t)R;
    const int nw = blockDim.x >> 6, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double *lchunk = reinterpret_cast<double *>(wbase) + wv * 64;
    int32_t *lx = reinterpret_cast<int32_t *>(wbase + (size_t)nw * 64 * sizeof(double)) + wv * s_pad;
    const uint4 *gd = reinterpret_cast<const uint4 *>(a.desc);
    const uint4 *gh = reinterpret_cast<const uint4 *>(a.rinfo);
    uint4 *sd = reinterpret_cast<uint4 *>(ldesc);
    uint4 *sh = reinterpret_cast<uint4 *>(linfo);
    for (int32_t i = threadIdx.x; i < R; i += blockDim.x) {
        sd[i] = gd[i];
        if (HDR) sh[i] = gh[i];
    }
    __syncthreads();
    LdsTables tab;
    tab.d = ldesc;
    tab.h = HDR ? linfo : a.rinfo;
    tab.ids = a.dep;
    const uint32_t iter = *a.iter_dev;
    const uint32_t M = (uint32_t)a.m_targ, cap = (uint32_t)a.cap;
    const uint32_t total = a.queue[1] * M;
    // Every lane executes the atomic (lane 0 adds one, the others zero) and
    // lane 0's result is broadcast.  With the atomic inside `if (lane == 0)`
    // the compiler routed lanes 1-63 around it (their result is always
    // zero) into an inner loop of their own, so they ran the next walker
    // without lane 0 -- and wave_walker_t needs the whole wave.
    uint32_t q = first_position();
    for (;;) {
        if (q >= total) break;
        const uint32_t sg = q / M, o = q - sg * M;
        const int2 seg = a.seg[sg];
        if ((int32_t)o < seg.y) {
            const uint32_t g = (uint32_t)seg.x + o;
            const uint32_t run = g / cap;
            wave_walker_t(a, tab, xs, (int32_t)run, (int32_t)(g - run * cap), iter, lchunk, lx);
        }
        const uint32_t got = atomicAdd(&a.queue[0], lane == 0 ? 1u : 0u);
        q = gridDim.x * (uint32_t)nw + (uint32_t)__shfl((int)got, 0, 64);
    }
}

// Factored-table variant: the block copies the descriptors (16 bytes per
// reaction), the change headers (8 bytes), the per-species incidence words
// (4 bytes) and the incidence lists (2 bytes per entry) into LDS -- 98 KB at
// 354 species / 3680 reactions -- and each wave keeps its walker's counts and
// its 64 chunk sums beside them (16 walkers per CU at that size); waves take
// walkers from the work queue until it is empty.  Nothing
// in the event loop reads global memory.
#define WAVE_FACT_MAX_WAVES 16

__global__ __launch_bounds__(64 * WAVE_FACT_MAX_WAVES) void ssa_wave_fact_kernel(SimArgs a, int32_t *__restrict__ xs,
                                                                                int32_t s_pad) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t R = a.R, S = a.S;
    uint4 *ld = reinterpret_cast<uint4 *>(smem);
    uint2 *lh = reinterpret_cast<uint2 *>(smem + fact_off_hdr(R));
    uint32_t *ltab = reinterpret_cast<uint32_t *>(smem + fact_off_tab(R));
    uint16_t *linc = reinterpret_cast<uint16_t *>(smem + fact_off_inc(R, S));
    unsigned char *wbase = smem + fact_tables_bytes(R, S, a.n_inc);
    const int nw = blockDim.x >> 6, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double *lchunk = reinterpret_cast<double *>(wbase) + wv * 64;
    int32_t *lx = reinterpret_cast<int32_t *>(wbase + (size_t)nw * 64 * sizeof(double)) + wv * s_pad;
    const uint4 *gd = reinterpret_cast<const uint4 *>(a.desc);
    for (int32_t i = threadIdx.x; i < R; i += blockDim.x) {
        ld[i] = gd[i];
        lh[i] = a.fhdr[i];
    }
    for (int32_t i = threadIdx.x; i < S; i += blockDim.x) ltab[i] = a.inc_tab[i];
    for (int32_t i = threadIdx.x; i < a.n_inc; i += blockDim.x) linc[i] = a.inc[i];
    __syncthreads();
    FactTables tab;
    tab.d = ld;
    tab.h = lh;
    tab.tab = ltab;
    tab.inc = linc;
    const uint32_t iter = *a.iter_dev;
    const uint32_t M = (uint32_t)a.m_targ, cap = (uint32_t)a.cap;
    const uint32_t total = a.queue[1] * M;
    // static first position, then the whole-wave queue atomic: see
    // ssa_wave_lds_kernel
    uint32_t q = first_position();
    for (;;) {
        if (q >= total) break;
        const uint32_t sg = q / M, o = q - sg * M;
        const int2 seg = a.seg[sg];
        if ((int32_t)o < seg.y) {
            const uint32_t g = (uint32_t)seg.x + o;
            const uint32_t run = g / cap;
            wave_walker_fact(a, tab, xs, (int32_t)run, (int32_t)(g - run * cap), iter, lchunk, lx);
        }
        const uint32_t got = atomicAdd(&a.queue[0], lane == 0 ? 1u : 0u);
        q = gridDim.x * (uint32_t)nw + (uint32_t)__shfl((int)got, 0, 64);
    }
}

bool wave_kernel_fits(int32_t S, int32_t R) { return R <= 4096 && S <= 8192; }

namespace {
// Blocks of an LDS variant that stay resident per CU, for a given LDS size.
template <bool HDR>
int lds_blocks_per_cu(int waves, size_t shmem) {
    static size_t last_shmem = 0;
    static int last_waves = 0, last = 1;
    if (shmem != last_shmem || waves != last_waves) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ssa_wave_lds_kernel<HDR>, 64 * waves, shmem) !=
                hipSuccess || nb < 1)
            nb = 1;
        last = nb;
        last_shmem = shmem;
        last_waves = waves;
    }
    return last;
}

int device_cus() {
    static int n = 0;
    if (n == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
            n = 1;
    }
    return n;
}

template <bool HDR>
hipError_t launch_lds(const SimArgs &a, int32_t *xs, int32_t s_pad, size_t tables, size_t per_wave, int64_t walkers,
                      hipStream_t st) {
    const int nw = (int)std::min<size_t>(WAVE_LDS_MAX_WAVES, (WAVE_LDS_BYTES - tables) / per_wave);
    const size_t shmem = tables + nw * per_wave;
    const int64_t resident = (int64_t)lds_blocks_per_cu<HDR>(nw, shmem) * device_cus();
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(resident, (walkers + nw - 1) / nw));
    hipLaunchKernelGGL(ssa_wave_lds_kernel<HDR>, dim3(blocks), dim3(64 * nw), shmem, st, a, xs, s_pad);
    return hipGetLastError();
}
}  // namespace

// The LDS variants need the work queue built by launch_work_queue.  The
// descriptors (16 B per reaction) and two walkers always fit one CU's LDS
// within wave_kernel_fits (R <= 4096, S <= 8192: at most 64 KB + 2 x 33 KB).
// Headers go to LDS too when they fit and the run's slots would fill at most
// two rounds of one such block per CU (WE keeps roughly half its slots live);
// beyond that the second block per CU is worth more than the header loads it
// saves.
// The factored-table kernel when the network has its tables and they fit
// beside one wave's slice.
bool wave_fact_fits(const SimArgs &a, size_t *tables, size_t *per_wave) {
    if (!a.fhdr || !a.inc || !a.inc_tab) return false;
    *tables = fact_tables_bytes(a.R, a.S, a.n_inc);
    *per_wave = 64 * sizeof(double) + sizeof(int32_t) * (size_t)((a.S + 3) & ~3);
    return *tables + *per_wave <= WAVE_LDS_BYTES;
}

namespace {
int fact_blocks_per_cu(int waves, size_t shmem) {
    static size_t last_shmem = 0;
    static int last_waves = 0, last = 1;
    if (shmem != last_shmem || waves != last_waves) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ssa_wave_fact_kernel, 64 * waves, shmem) != hipSuccess ||
            nb < 1)
            nb = 1;
        last = nb;
        last_shmem = shmem;
        last_waves = waves;
    }
    return last;
}
}  // namespace

// Which variant: the factored-table kernel when every live walker gets a wave
// at once (WE keeps roughly half its slots live), i.e. when each walker's
// event chain is the bound; otherwise the descriptor-table kernel, which
// issues fewer instructions per event (the incidence-list walk is the
// difference) and holds up to 16 walkers per CU in two blocks.  Measured on
// the 354/3680 network (before the chunk sums took LDS atomic adds): one run
// (2465 live walkers) 0.417-0.430 ms per launch against 0.458 ms; eight runs
// (19,600 live walkers) 1.59 ms against 1.41 ms.
namespace {
// Waves per block of the factored-table kernel when it is the one to run
// (0: the descriptor-table kernel), with its LDS bytes.
int fact_choice(const SimArgs &a, size_t *shmem_out) {
    size_t tables = 0, per_wave = 0;
    if (!wave_fact_fits(a, &tables, &per_wave)) return 0;
    const int nw = (int)std::min<size_t>(WAVE_FACT_MAX_WAVES, (WAVE_LDS_BYTES - tables) / per_wave);
    const size_t shmem = tables + nw * per_wave;
    const int64_t live = ((int64_t)a.n_runs * a.cap + 1) / 2;
    if (nw < 1 || live > (int64_t)fact_blocks_per_cu(nw, shmem) * nw * device_cus()) return 0;
    *shmem_out = shmem;
    return nw;
}

bool lds_headers(const SimArgs &a, int32_t s_pad, size_t per_wave) {
    const int64_t walkers = (int64_t)a.n_runs * a.cap;
    const size_t desc_bytes = 16 * (size_t)a.R;
    if (2 * desc_bytes + 2 * per_wave > WAVE_LDS_BYTES) return false;
    const int nw = (int)std::min<size_t>(WAVE_LDS_MAX_WAVES, (WAVE_LDS_BYTES - 2 * desc_bytes) / per_wave);
    return walkers <= 2 * (int64_t)nw * device_cus();
}
}  // namespace

const char *ssa_wave_name(const SimArgs &a) {
    size_t shmem = 0;
    if (fact_choice(a, &shmem) > 0) return "ssa_wave_fact_kernel";
    const int32_t s_pad = (a.S + 3) & ~3;
    const size_t per_wave = 64 * sizeof(double) + sizeof(int32_t) * (size_t)s_pad;
    return lds_headers(a, s_pad, per_wave) ? "ssa_wave_lds_kernel<true>" : "ssa_wave_lds_kernel<false>";
}

hipError_t launch_ssa_wave(const SimArgs &a, int32_t *xs, hipStream_t st) {
    if (!wave_kernel_fits(a.S, a.R)) return hipErrorInvalidValue;
    {
        size_t shmem = 0;
        const int nw = fact_choice(a, &shmem);
        if (nw > 0) {
            const int64_t walkers = (int64_t)a.n_runs * a.cap;
            const int64_t resident = (int64_t)fact_blocks_per_cu(nw, shmem) * device_cus();
            const unsigned blocks =
                (unsigned)std::max<int64_t>(1, std::min<int64_t>(resident, (walkers + nw - 1) / nw));
            const int32_t s_pad = (a.S + 3) & ~3;
            hipLaunchKernelGGL(ssa_wave_fact_kernel, dim3(blocks), dim3(64 * nw), shmem, st, a, xs, s_pad);
            return hipGetLastError();
        }
    }
    const int32_t s_pad = (a.S + 3) & ~3;
    const size_t per_wave = 64 * sizeof(double) + sizeof(int32_t) * (size_t)s_pad;
    const int64_t walkers = (int64_t)a.n_runs * a.cap;
    const size_t desc_bytes = 16 * (size_t)a.R;
    if (lds_headers(a, s_pad, per_wave))
        return launch_lds<true>(a, xs, s_pad, 2 * desc_bytes, per_wave, walkers, st);
    return launch_lds<false>(a, xs, s_pad, desc_bytes, per_wave, walkers, st);
}
