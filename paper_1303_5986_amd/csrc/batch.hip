// batch.hip -- many independent WE runs of different networks stepped
// together (gfx950).
//
// Runs are independent (the paper runs independent replicas for its error
// bars, Sec. IV), so a batch is a set of ordinary sims sharing one stream.
// What is batched is the propagation: instead of one SSA launch per run --
// each too small to fill 256 CUs when a run holds a few hundred walkers --
// every kernel variant gets ONE persistent launch whose waves pull work
// items (run, tile) from a device counter until the list is exhausted:
//   lane variants: a tile is 64 consecutive walker slots, one per lane;
//   group variants: a tile is 64 / L consecutive slots, L lanes each;
//   wave variant:  a tile is one walker slot, one wave.
// Items of cheap and expensive runs mix freely, so uneven runs balance
// across the chip.  The bookkeeping is batched the same way: recycle/bin,
// resample (one workgroup per run of every member), gather, observe and the
// iteration counters are one launch each, with the member index on grid y;
// a member's arguments and buffers are read from device tables.  The whole
// iteration can be captured as a HIP graph (the work counters are cleared
// by a kernel, not a memset, so replays are safe).  Members may record their
// ensembles (eager steps only) and, once a member's committor is trained and
// switched on, bin on it: one batched launch evaluates every such member's
// model after the batched recycle/bin.
//
// Autotuning: every kernel a network fits -- lane (64 walkers per wave),
// group with 32, 16, 8, 4 or 2 walkers per wave, wave (one) -- runs a short
// pilot (one interval with every slot filled, timed with HIP events, best of
// autotune_iters) and the fastest is kept; the choice is cached in a JSON
// file keyed by (species, reactions, walker slots, runs, tau).
#include <algorithm>
#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "ssa_group_body.h"
#include "ssa_lane_body.h"
#include "ssa_wave_body.h"
#include "we_internal.h"

namespace {

// V_GROUPR_L: the group kernel with L lanes per walker for members whose
// lane blocks hold at most BATCH_GROUP_REG reactions (descriptors and
// propensities in registers, read once per walker and interval).
enum Variant {
    V_LANE_1_4 = 0, V_LANE_2_8, V_LANE_8_16, V_LANE_16_32,
    V_GROUP_2, V_GROUP_4, V_GROUP_8, V_GROUP_16, V_GROUP_32,
    V_GROUPR_2, V_GROUPR_4, V_GROUPR_8, V_GROUPR_16, V_GROUPR_32,
    V_WAVE, V_COUNT
};
#define BATCH_GROUP_REG 8

// Walker slots per work item of a variant.
int32_t tile_of(int v) {
    switch (v) {
    case V_GROUP_2: case V_GROUPR_2: return 32;
    case V_GROUP_4: case V_GROUPR_4: return 16;
    case V_GROUP_8: case V_GROUPR_8: return 8;
    case V_GROUP_16: case V_GROUPR_16: return 4;
    case V_GROUP_32: case V_GROUPR_32: return 2;
    case V_WAVE: return 1;
    default: return 64;
    }
}

struct Item {
    int32_t sim, run, slot;
};

Variant variant_of(const we_sim *s) {
    const int32_t S = s->S, R = s->net->R;
    if (s->kernel == WE_KERNEL_WAVE) return V_WAVE;
    if (s->kernel == WE_KERNEL_GROUP) {
        const bool reg = (R + s->group_lanes - 1) / s->group_lanes <= BATCH_GROUP_REG;
        switch (s->group_lanes) {
        case 2: return reg ? V_GROUPR_2 : V_GROUP_2;
        case 4: return reg ? V_GROUPR_4 : V_GROUP_4;
        case 8: return reg ? V_GROUPR_8 : V_GROUP_8;
        case 16: return reg ? V_GROUPR_16 : V_GROUP_16;
        default: return reg ? V_GROUPR_32 : V_GROUP_32;
        }
    }
    if (S <= 1 && R <= 4) return V_LANE_1_4;
    if (S <= 2 && R <= 8) return V_LANE_2_8;
    if (S <= 8 && R <= 16) return V_LANE_8_16;
    if (S <= 16 && R <= 32) return V_LANE_16_32;
    return V_WAVE;
}

}  // namespace

template <int SMAX, int RMAX>
__global__ __launch_bounds__(256) void batch_lane_kernel(const SimArgs *__restrict__ args,
                                                         int32_t *const *__restrict__ xptr,
                                                         const Item *__restrict__ items, int32_t n_items,
                                                         uint32_t *__restrict__ counter) {
    constexpr bool REG = RMAX <= LANE_REG_RMAX;
    constexpr int ROWS = REG ? 1 : RMAX * LaneRow<SMAX>::W;
    __shared__ int32_t rows[4 * ROWS];
    int32_t *wrows = rows + (threadIdx.x >> 6) * ROWS;
    const int lane = threadIdx.x & 63;
    const uint32_t n_static = gridDim.x * (blockDim.x >> 6);
    uint32_t idx = first_position();
    for (;;) {
        if (idx >= (uint32_t)n_items) break;
        const Item it = items[idx];
        const SimArgs &a = args[it.sim];
        if constexpr (!REG) lane_stage_rows<SMAX>(a, wrows);
        const int32_t k = it.slot + lane;
        if (k < a.n_walk[it.run]) lane_walker<SMAX, RMAX>(a, xptr[it.sim], it.run, k, *a.iter_dev, wrows);
        // every lane executes the atomic (lane 0 adds one): no lane takes a
        // path of its own around the wave-wide steps of the walker
        const uint32_t got = atomicAdd(counter, lane == 0 ? 1u : 0u);
        idx = n_static + (uint32_t)__shfl((int)got, 0, 64);
    }
}

__global__ __launch_bounds__(256) void batch_wave_kernel(const SimArgs *__restrict__ args,
                                                         int32_t *const *__restrict__ xptr,
                                                         const Item *__restrict__ items, int32_t n_items,
                                                         uint32_t *__restrict__ counter, int32_t s_pad) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    double *lchunk = reinterpret_cast<double *>(smem) + wv * 64;
    int32_t *lx = reinterpret_cast<int32_t *>(smem + WAVE_WALKERS_PER_BLOCK * 64 * sizeof(double)) + wv * s_pad;
    const uint32_t n_static = gridDim.x * (blockDim.x >> 6);
    uint32_t idx = first_position();
    for (;;) {
        if (idx >= (uint32_t)n_items) break;
        const Item it = items[idx];
        const SimArgs &a = args[it.sim];
        if (it.slot < a.n_walk[it.run]) wave_walker(a, xptr[it.sim], it.run, it.slot, *a.iter_dev, lchunk, lx);
        __builtin_amdgcn_wave_barrier();
        // every lane executes the atomic (lane 0 adds one): no lane takes a
        // path of its own around the wave-wide steps of the walker
        const uint32_t got = atomicAdd(counter, lane == 0 ? 1u : 0u);
        idx = n_static + (uint32_t)__shfl((int)got, 0, 64);
    }
}

// Group variant: a work item is 64 / L consecutive slots of one run, one
// group of L lanes per slot; lx slices are s_max ints (the largest species
// count among the members on this variant).  BR > 0: the members' lane
// blocks hold at most BR reactions, kept in registers (group_walker).
template <int L, int BR = 0>
__global__ __launch_bounds__(256) void batch_group_kernel(const SimArgs *__restrict__ args,
                                                          int32_t *const *__restrict__ xptr,
                                                          const Item *__restrict__ items, int32_t n_items,
                                                          uint32_t *__restrict__ counter, int32_t s_max) {
    extern __shared__ int32_t bglds[];
    constexpr int G = 64 / L;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int grp = lane / L;
    int32_t *lx = bglds + ((size_t)wv * G + grp) * s_max;
    const uint32_t n_static = gridDim.x * (blockDim.x >> 6);
    uint32_t idx = first_position();
    for (;;) {
        if (idx >= (uint32_t)n_items) break;
        const Item it = items[idx];
        const SimArgs &a = args[it.sim];
        const int32_t k = it.slot + grp;
        const bool live = k < a.cap && k < a.n_walk[it.run];
        const GroupTables tb{a.desc, a.chg_ptr, a.chg};
        group_walker<L, BR>(a, tb, xptr[it.sim], it.run, k, live, *a.iter_dev, lx);
        // every lane executes the atomic (lane 0 adds one): see batch_lane_kernel
        const uint32_t got = atomicAdd(counter, lane == 0 ? 1u : 0u);
        idx = n_static + (uint32_t)__shfl((int)got, 0, 64);
    }
}

__global__ void batch_reset_kernel(uint32_t *counters, int32_t n) {
    const int32_t i = threadIdx.x;
    if (i < n) counters[i] = 0u;
}

struct BatchPtrs {
    const SimArgs *args;
    int32_t *const *x_cur;
    int32_t *const *x_nxt;
    const double *const *w_cur;
    double *const *w_nxt;
    const int32_t *use_lds;
    const int32_t *grid_bins;
};
hipError_t launch_batch_bookkeeping(const BatchPtrs &b, int32_t n_sims, int64_t max_slots, int32_t max_runs,
                                    int64_t max_cells, size_t shmem, bool observe, const CmBatchModel *models,
                                    int32_t s_max_cm, hipStream_t st);
bool resample_uses_lds(const SimArgs &a);
size_t resample_lds_bytes(const SimArgs &a, bool use_lds);
int32_t resample_place_rows(const SimArgs &a, int64_t blocks);

struct we_batch {
    hipStream_t stream = nullptr;
    std::vector<we_sim *> sims;
    std::vector<Variant> var;
    std::vector<Item> items[V_COUNT];
    Item *d_items[V_COUNT] = {};
    uint32_t *d_counters = nullptr;
    SimArgs *d_args = nullptr;
    int32_t **d_xptr[2] = {nullptr, nullptr};
    double **d_wptr[2] = {nullptr, nullptr};
    int32_t *d_use_lds = nullptr, *d_grid_bins = nullptr;
    int64_t max_slots = 0, max_cells = 0;
    int32_t max_runs = 0;
    size_t resample_shmem = 0;
    bool observe = false;
    int32_t s_pad = 4;
    int32_t s_group = 1;              // largest species count among group-kernel members
    int32_t iter = 0, max_iters = 0;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t capture_stream = nullptr;
    int32_t graph_iters = 0;
    bool capturing = false;
    // learned bins: each member's active model as the device tables hold it
    std::vector<CmBatchModel> cm_host, cm_graph;
    std::vector<int32_t> grid_bins_host;
    CmBatchModel *d_models = nullptr;
    int32_t s_max_cm = 0;
    bool any_cm = false;
};

namespace {

// Pilot timing of one kernel choice.  Each of `reps` throw-away sims starts
// with every slot of every run holding a walker at x0 (weight 1 / cap) and
// times its first interval: propagation at full occupancy, the regime a WE
// run spends most of its time near once its bins fill, rather than the
// sparse initial ensemble (a few walkers per run favour the kernels with
// the fewest walkers per wave, which lose once the bins fill).  The fastest
// repetition counts.
we_status pilot_ms(const we_network *net, const we_grid *g, const we_params *p, int32_t kernel,
                   int32_t walkers_per_wave, int32_t reps, hipStream_t st, double *ms) {
    we_params q = *p;
    q.kernel = kernel;
    q.walkers_per_wave = walkers_per_wave;
    q.max_iters = 1;
    q.record_iters = 0;
    q.n_joint = 0;
    q.hist_hi = q.hist_lo - 1;
    *ms = 0.0;
    for (int32_t rep = 0; rep < std::max(reps, 1); ++rep) {
        we_sim *s = nullptr;
        we_status r = we_init(net, g, &q, st, nullptr, 0, &s);
        if (r != WE_OK) return r;
        const int32_t cap = s->cap, S = s->S;
        std::vector<int32_t> xs((size_t)cap * S);
        for (int32_t k = 0; k < cap; ++k) std::copy(p->x0, p->x0 + S, xs.begin() + (size_t)k * S);
        const std::vector<double> ws(cap, 1.0 / cap);
        for (int32_t run = 0; run < s->n_runs && r == WE_OK; ++run)
            r = we_set_ensemble(s, run, cap, xs.data(), ws.data());
        hipEvent_t e0 = nullptr, e1 = nullptr;
        float t = 0.f;
        if (r == WE_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
            r = we_fail(WE_EDEVICE, "hipEventCreate failed");
        if (r == WE_OK && hipEventRecord(e0, st) != hipSuccess) r = we_fail(WE_EDEVICE, "hipEventRecord failed");
        if (r == WE_OK) r = we_step_intervals(s, 1);
        if (r == WE_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&t, e0, e1) != hipSuccess))
            r = we_fail(WE_EDEVICE, "pilot timing failed");
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (r == WE_OK) r = we_synchronize(s);
        we_destroy(s);
        if (r != WE_OK) return r;
        if (rep == 0 || t < *ms) *ms = t;
    }
    return WE_OK;
}

std::map<std::string, int> read_cache(const char *path) {
    std::map<std::string, int> m;
    if (!path || !*path) return m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    // flat object of "key": value pairs
    size_t pos = 0;
    while ((pos = t.find('"', pos)) != std::string::npos) {
        const size_t end = t.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = t.substr(pos + 1, end - pos - 1);
        const size_t colon = t.find(':', end);
        if (colon == std::string::npos) break;
        m[key] = std::atoi(t.c_str() + colon + 1);
        pos = t.find_first_of(",}", colon);
        if (pos == std::string::npos) break;
    }
    return m;
}

void write_cache(const char *path, const std::map<std::string, int> &m) {
    if (!path || !*path) return;
    std::ofstream f(path);
    f << "{";
    bool first = true;
    for (const auto &kv : m) {
        f << (first ? "" : ",") << "\n  \"" << kv.first << "\": " << kv.second;
        first = false;
    }
    f << "\n}\n";
}

we_status build_items(we_batch *b) {
    for (int v = 0; v < V_COUNT; ++v) b->items[v].clear();
    for (size_t i = 0; i < b->sims.size(); ++i) {
        we_sim *s = b->sims[i];
        const Variant v = b->var[i];
        const int32_t step = tile_of(v);
        for (int32_t r = 0; r < s->n_runs; ++r)
            for (int32_t k = 0; k < s->cap; k += step) b->items[v].push_back(Item{(int32_t)i, r, k});
    }
    for (int v = 0; v < V_COUNT; ++v) {
        if (b->d_items[v]) { (void)hipFree(b->d_items[v]); b->d_items[v] = nullptr; }
        if (b->items[v].empty()) continue;
        HIP_TRY(hipMalloc(&b->d_items[v], sizeof(Item) * b->items[v].size()));
        HIP_TRY(hipMemcpy(b->d_items[v], b->items[v].data(), sizeof(Item) * b->items[v].size(),
                          hipMemcpyHostToDevice));
    }
    return WE_OK;
}

bool same_models(const std::vector<CmBatchModel> &x, const std::vector<CmBatchModel> &y) {
    if (x.size() != y.size()) return false;
    for (size_t i = 0; i < x.size(); ++i)
        if (x[i].params != y[i].params || x[i].wt != y[i].wt || x[i].feat != y[i].feat || x[i].qedges != y[i].qedges)
            return false;
    return true;
}

std::vector<CmBatchModel> current_models(const we_batch *b) {
    std::vector<CmBatchModel> m;
    for (const we_sim *s : b->sims) m.push_back(committor_batch_model(s));
    return m;
}

// Bring the device tables of learned bins up to date with the members'
// committors (trained and switched on since the last iteration, or off).
we_status refresh_models(we_batch *b) {
    std::vector<CmBatchModel> m = current_models(b);
    if (same_models(m, b->cm_host)) return WE_OK;
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->any_cm = false;
    b->s_max_cm = 0;
    for (size_t i = 0; i < m.size(); ++i) {
        const bool on = m[i].params != nullptr;
        b->grid_bins_host[i] = on ? 0 : 1;
        if (on) {
            b->any_cm = true;
            b->s_max_cm = std::max(b->s_max_cm, b->sims[i]->S);
        }
    }
    HIP_TRY(hipMemcpy(b->d_models, m.data(), sizeof(CmBatchModel) * m.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(b->d_grid_bins, b->grid_bins_host.data(), sizeof(int32_t) * m.size(), hipMemcpyHostToDevice));
    b->cm_host = m;
    return WE_OK;
}

we_status launch_batch_iteration(we_batch *b, hipStream_t st, bool capture) {
    if (!capture) {
        we_status r = refresh_models(b);
        if (r != WE_OK) return r;
    }
    const int32_t parity = b->sims[0]->cur;
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, st, b->d_counters, (int32_t)V_COUNT);
    HIP_TRY(hipGetLastError());
    int32_t *const *xp = b->d_xptr[parity];
    for (int v = 0; v < V_COUNT; ++v) {
        const int32_t n = (int32_t)b->items[v].size();
        if (n == 0) continue;
        const unsigned blocks = (unsigned)std::min<int64_t>((n + 3) / 4, 2048);
        uint32_t *cnt = b->d_counters + v;
        switch (v) {
        case V_LANE_1_4:
            hipLaunchKernelGGL((batch_lane_kernel<1, 4>), dim3(blocks), dim3(256), 0, st, b->d_args, xp, b->d_items[v], n, cnt);
            break;
        case V_LANE_2_8:
            hipLaunchKernelGGL((batch_lane_kernel<2, 8>), dim3(blocks), dim3(256), 0, st, b->d_args, xp, b->d_items[v], n, cnt);
            break;
        case V_LANE_8_16:
            hipLaunchKernelGGL((batch_lane_kernel<8, 16>), dim3(blocks), dim3(256), 0, st, b->d_args, xp, b->d_items[v], n, cnt);
            break;
        case V_LANE_16_32:
            hipLaunchKernelGGL((batch_lane_kernel<16, 32>), dim3(blocks), dim3(256), 0, st, b->d_args, xp, b->d_items[v], n, cnt);
            break;
        case V_GROUPR_2:
        case V_GROUPR_4:
        case V_GROUPR_8:
        case V_GROUPR_16:
        case V_GROUPR_32: {
            const int32_t G = tile_of(v);
            const size_t shmem = sizeof(int32_t) * 4 * (size_t)G * b->s_group;
            if (v == V_GROUPR_2)
                hipLaunchKernelGGL((batch_group_kernel<2, BATCH_GROUP_REG>), dim3(blocks), dim3(256), shmem, st, b->d_args, xp, b->d_items[v], n, cnt, b->s_group);
            else if (v == V_GROUPR_4)
                hipLaunchKernelGGL((batch_group_kernel<4, BATCH_GROUP_REG>), dim3(blocks), dim3(256), shmem, st, b->d_args, xp, b->d_items[v], n, cnt, b->s_group);
            else if (v == V_GROUPR_8)
                hipLaunchKernelGGL((batch_group_kernel<8, BATCH_GROUP_REG>), dim3(blocks), dim3(256), shmem, st, b->d_args, xp, b->d_items[v], n, cnt, b->s_group);
            else if (v == V_GROUPR_16)
                hipLaunchKernelGGL((batch_group_kernel<16, BATCH_GROUP_REG>), dim3(blocks), dim3(256), shmem, st, b->d_args, xp, b->d_items[v], n, cnt, b->s_group);
            else
                hipLaunchKernelGGL((batch_group_kernel<32, BATCH_GROUP_REG>), dim3(blocks), dim3(256), shmem, st, b->d_args, xp, b->d_items[v], n, cnt, b->s_group);
            break;
        }
        case V_GROUP_2:
        case V_GROUP_4:
        case V_GROUP_8:
        case V_GROUP_16:
        case V_GROUP_32: {
            const int32_t G = tile_of(v);
            const size_t shmem = sizeof(int32_t) * 4 * (size_t)G * b->s_group;
            if (v == V_GROUP_2)
                hipLaunchKernelGGL((batch_group_kernel<2>), dim3(blocks), dim3(256), shmem, st, b->d_args, xp, b->d_items[v], n, cnt, b->s_group);
            else if (v == V_GROUP_4)
                hipLaunchKernelGGL((batch_group_kernel<4>), dim3(blocks), dim3(256), shmem, st, b->d_args, xp, b->d_items[v], n, cnt, b->s_group);
            else if (v == V_GROUP_8)
                hipLaunchKernelGGL((batch_group_kernel<8>), dim3(blocks), dim3(256), shmem, st, b->d_args, xp, b->d_items[v], n, cnt, b->s_group);
            else if (v == V_GROUP_16)
                hipLaunchKernelGGL((batch_group_kernel<16>), dim3(blocks), dim3(256), shmem, st, b->d_args, xp, b->d_items[v], n, cnt, b->s_group);
            else
                hipLaunchKernelGGL((batch_group_kernel<32>), dim3(blocks), dim3(256), shmem, st, b->d_args, xp, b->d_items[v], n, cnt, b->s_group);
            break;
        }
        default: {
            const size_t shmem = WAVE_WALKERS_PER_BLOCK * (64 * sizeof(double) + sizeof(int32_t) * (size_t)b->s_pad);
            hipLaunchKernelGGL(batch_wave_kernel, dim3(blocks), dim3(256), shmem, st, b->d_args, xp, b->d_items[v],
                               n, cnt, b->s_pad);
        }
        }
        HIP_TRY(hipGetLastError());
    }
    // recycle/bin, committor bins where active, resample, gather, observe,
    // advance: one launch per step for all members
    BatchPtrs bp{b->d_args, b->d_xptr[parity], b->d_xptr[1 - parity],
                 (const double *const *)b->d_wptr[parity], b->d_wptr[1 - parity], b->d_use_lds,
                 b->d_grid_bins};
    HIP_TRY(launch_batch_bookkeeping(bp, (int32_t)b->sims.size(), b->max_slots, b->max_runs, b->max_cells,
                                     b->resample_shmem, b->observe, b->any_cm ? b->d_models : nullptr,
                                     b->s_max_cm, st));
    for (we_sim *s : b->sims) s->cur = 1 - s->cur;
    if (!capture)
        for (we_sim *s : b->sims) HIP_TRY(committor_record(s, st));
    return WE_OK;
}

bool recording(const we_batch *b) {
    for (const we_sim *s : b->sims)
        if (s->rec.cap_iters > 0 && s->rec.n_iters < s->rec.cap_iters) return true;
    return false;
}

}  // namespace

extern "C" we_status we_batch_create(int32_t n, const we_network *const *nets, const we_grid *grids,
                                     const we_params *params, void *hip_stream, int32_t autotune_iters,
                                     const char *cache_path, we_batch **out) {
    if (!out || n <= 0 || !nets || !grids || !params) return we_fail(WE_EINVAL, "bad arguments");
    *out = nullptr;
    we_batch *b = new we_batch();
    b->stream = (hipStream_t)hip_stream;
    std::map<std::string, int> cache = read_cache(cache_path);
    bool cache_dirty = false;
    for (int32_t i = 0; i < n; ++i) {
        we_params p = params[i];
        if (p.rw_period > 0) {
            we_batch_destroy(b);
            return we_fail(WE_EINVAL, "reweighting is not supported inside a batch");
        }
        if (p.engine != 0) {
            we_batch_destroy(b);
            return we_fail(WE_EINVAL, "tau-leaping is not supported inside a batch");
        }
        if (!nets[i]->hill.empty()) {
            we_batch_destroy(b);
            return we_fail(WE_EINVAL, "Hill-type rates are not supported inside a batch");
        }
        const int32_t S = nets[i]->S, R = nets[i]->R;
        if (p.kernel == WE_KERNEL_AUTO) {
            const bool lane_ok = lane_kernel_fits(S, R, nets[i]->max_delta);
            if (autotune_iters > 0) {
                char key[128];
                std::snprintf(key, sizeof key, "S%d_R%d_cap%d_runs%d_tau%g", S, R, p.m_targ * grids[i].n_bins,
                              p.n_runs, p.tau);
                auto it = cache.find(key);
                if (it != cache.end()) {
                    // value: kernel + 16 * walkers per wave (group kernel)
                    p.kernel = it->second % 16;
                    p.walkers_per_wave = it->second / 16;
                } else {
                    std::vector<std::pair<int32_t, int32_t>> cand;
                    if (lane_ok) cand.push_back({WE_KERNEL_LANE, 0});
                    for (int32_t wpw : {32, 16, 8, 4, 2})
                        if (group_kernel_fits(S, R, 64 / wpw)) cand.push_back({WE_KERNEL_GROUP, wpw});
                    if (wave_kernel_fits(S, R) && nets[i]->max_chg <= 64) cand.push_back({WE_KERNEL_WAVE, 0});
                    double best = 0.0;
                    for (size_t c = 0; c < cand.size(); ++c) {
                        double t = 0.0;
                        we_status r = pilot_ms(nets[i], &grids[i], &p, cand[c].first, cand[c].second, autotune_iters,
                                               b->stream, &t);
                        if (r != WE_OK) { we_batch_destroy(b); return r; }
                        if (c == 0 || t < best) {
                            best = t;
                            p.kernel = cand[c].first;
                            p.walkers_per_wave = cand[c].second;
                        }
                    }
                    cache[key] = p.kernel + 16 * p.walkers_per_wave;
                    cache_dirty = true;
                }
            } else {
                p.kernel = (lane_ok && R <= 32) ? WE_KERNEL_LANE : WE_KERNEL_WAVE;
            }
        }
        we_sim *s = nullptr;
        we_status r = we_init(nets[i], &grids[i], &p, b->stream, nullptr, 0, &s);
        if (r != WE_OK) { we_batch_destroy(b); return r; }
        b->sims.push_back(s);
        b->var.push_back(variant_of(s));
        b->s_pad = std::max(b->s_pad, (S + 3) & ~3);
        if (s->kernel == WE_KERNEL_GROUP) b->s_group = std::max(b->s_group, S);
        b->max_iters = (i == 0) ? s->max_iters : std::min(b->max_iters, s->max_iters);
    }
    if (cache_dirty) write_cache(cache_path, cache);
    if ((size_t)WAVE_WALKERS_PER_BLOCK * (64 * sizeof(double) + 4 * (size_t)b->s_pad) > 64 * 1024) {
        we_batch_destroy(b);
        return we_fail(WE_EINVAL, "species count too large for the batched wave kernel");
    }
    std::vector<SimArgs> args;
    std::vector<int32_t *> xp0, xp1;
    std::vector<double *> wp0, wp1;
    std::vector<int32_t> use_lds, grid_bins;
    int32_t runs_hi = 0;
    for (we_sim *s : b->sims) runs_hi = std::max(runs_hi, s->n_runs);
    for (we_sim *s : b->sims) {
        args.push_back(s->args);
        args.back().queue_stats = 0;   // the batched kernels keep their own work queue
        // cursor rows for the batched launch's block size
        args.back().place_rows = resample_place_rows(s->args, (int64_t)runs_hi * (int64_t)b->sims.size());
        xp0.push_back(s->x[0]);
        xp1.push_back(s->x[1]);
        wp0.push_back(s->w[0]);
        wp1.push_back(s->w[1]);
        const bool ul = resample_uses_lds(s->args);
        use_lds.push_back(ul ? 1 : 0);
        grid_bins.push_back(1);
        b->resample_shmem = std::max(b->resample_shmem, resample_lds_bytes(args.back(), ul));
        b->max_slots = std::max<int64_t>(b->max_slots, (int64_t)s->n_runs * s->cap);
        b->max_cells = std::max<int64_t>(b->max_cells, (int64_t)s->n_runs * s->cap * s->S);
        b->max_runs = std::max(b->max_runs, s->n_runs);
        b->observe = b->observe || s->args.nh > 0 || s->args.n_joint > 0;
    }
    HIP_TRY(hipMalloc(&b->d_wptr[0], sizeof(double *) * n));
    HIP_TRY(hipMalloc(&b->d_wptr[1], sizeof(double *) * n));
    HIP_TRY(hipMemcpy(b->d_wptr[0], wp0.data(), sizeof(double *) * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(b->d_wptr[1], wp1.data(), sizeof(double *) * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&b->d_models, sizeof(CmBatchModel) * n));
    b->cm_host.assign(n, CmBatchModel{});
    b->grid_bins_host.assign(n, 1);
    HIP_TRY(hipMemcpy(b->d_models, b->cm_host.data(), sizeof(CmBatchModel) * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&b->d_use_lds, sizeof(int32_t) * n));
    HIP_TRY(hipMalloc(&b->d_grid_bins, sizeof(int32_t) * n));
    HIP_TRY(hipMemcpy(b->d_use_lds, use_lds.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(b->d_grid_bins, grid_bins.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&b->d_args, sizeof(SimArgs) * n));
    HIP_TRY(hipMemcpy(b->d_args, args.data(), sizeof(SimArgs) * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&b->d_xptr[0], sizeof(int32_t *) * n));
    HIP_TRY(hipMalloc(&b->d_xptr[1], sizeof(int32_t *) * n));
    HIP_TRY(hipMemcpy(b->d_xptr[0], xp0.data(), sizeof(int32_t *) * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(b->d_xptr[1], xp1.data(), sizeof(int32_t *) * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&b->d_counters, sizeof(uint32_t) * V_COUNT));
    we_status r = build_items(b);
    if (r != WE_OK) { we_batch_destroy(b); return r; }
    *out = b;
    return WE_OK;
}

extern "C" we_status we_batch_step(we_batch *b, int32_t n) {
    if (!b) return we_fail(WE_EINVAL, "NULL batch");
    if (n < 0 || (int64_t)b->iter + n > b->max_iters) return we_fail(WE_ECAPACITY, "max_iters exceeded");
    for (int32_t i = 0; i < n; ++i) {
        we_status r = launch_batch_iteration(b, b->stream, false);
        if (r != WE_OK) return r;
        b->iter += 1;
        for (we_sim *s : b->sims) {
            s->iter += 1;
            if (s->args.nh > 0) s->hist_iters += 1;
        }
    }
    return WE_OK;
}

extern "C" we_status we_batch_graph_capture(we_batch *b, int32_t n) {
    if (!b) return we_fail(WE_EINVAL, "NULL batch");
    if (n <= 0 || (n & 1)) return we_fail(WE_EINVAL, "capture an even, positive number of iterations");
    if (b->graph_exec) { (void)hipGraphExecDestroy(b->graph_exec); b->graph_exec = nullptr; }
    if (!b->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (recording(b)) return we_fail(WE_ESTATE, "a member is recording: step eagerly until its record buffer is full");
    {
        we_status r = refresh_models(b);
        if (r != WE_OK) return r;
    }
    std::vector<int32_t> cur0;
    for (we_sim *s : b->sims) { cur0.push_back(s->cur); s->capturing = true; }
    HIP_TRY(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
    we_status r = WE_OK;
    for (int32_t i = 0; i < n && r == WE_OK; ++i) r = launch_batch_iteration(b, b->capture_stream, true);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->capture_stream, &g);
    for (size_t i = 0; i < b->sims.size(); ++i) { b->sims[i]->cur = cur0[i]; b->sims[i]->capturing = false; }
    if (r != WE_OK) { if (g) (void)hipGraphDestroy(g); return r; }
    if (e != hipSuccess) return we_hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return we_hip_fail(e, "hipGraphInstantiate");
    b->graph_iters = n;
    b->cm_graph = b->cm_host;
    return WE_OK;
}

extern "C" we_status we_batch_graph_replay(we_batch *b, int32_t times) {
    if (!b) return we_fail(WE_EINVAL, "NULL batch");
    if (!b->graph_exec) return we_fail(WE_ESTATE, "no captured graph");
    if (times < 0 || (int64_t)b->iter + (int64_t)times * b->graph_iters > b->max_iters)
        return we_fail(WE_ECAPACITY, "max_iters exceeded");
    if (!same_models(current_models(b), b->cm_graph))
        return we_fail(WE_ESTATE, "a member's bins changed since the capture: capture again");
    for (int32_t t = 0; t < times; ++t) {
        HIP_TRY(hipGraphLaunch(b->graph_exec, b->stream));
        b->iter += b->graph_iters;
        for (we_sim *s : b->sims) {
            s->iter += b->graph_iters;
            if (s->args.nh > 0) s->hist_iters += b->graph_iters;
        }
    }
    return WE_OK;
}

extern "C" we_sim *we_batch_sim(we_batch *b, int32_t i) {
    if (!b || i < 0 || i >= (int32_t)b->sims.size()) return nullptr;
    return b->sims[i];
}

extern "C" we_status we_batch_info(we_batch *b, int32_t *n_sims, int32_t *kernels, int32_t *walkers_per_wave) {
    if (!b) return we_fail(WE_EINVAL, "NULL batch");
    if (n_sims) *n_sims = (int32_t)b->sims.size();
    for (size_t i = 0; i < b->sims.size(); ++i) {
        const we_sim *s = b->sims[i];
        if (kernels) kernels[i] = s->kernel;
        if (walkers_per_wave)
            walkers_per_wave[i] = s->kernel == WE_KERNEL_GROUP ? 64 / s->group_lanes
                                  : s->kernel == WE_KERNEL_WAVE ? 1 : 64;
    }
    return WE_OK;
}

extern "C" void we_batch_destroy(we_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (we_sim *s : b->sims) we_destroy(s);
    for (int v = 0; v < V_COUNT; ++v) (void)hipFree(b->d_items[v]);
    (void)hipFree(b->d_counters);
    (void)hipFree(b->d_args);
    (void)hipFree(b->d_xptr[0]);
    (void)hipFree(b->d_xptr[1]);
    (void)hipFree(b->d_wptr[0]);
    (void)hipFree(b->d_wptr[1]);
    (void)hipFree(b->d_use_lds);
    (void)hipFree(b->d_grid_bins);
    (void)hipFree(b->d_models);
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    delete b;
}
