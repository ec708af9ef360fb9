// we_internal.h -- host-side structures shared by the translation units of
// libwe.so (not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/we.h"
#include "we_common.h"

we_status we_fail(we_status st, const std::string &msg);
we_status we_hip_fail(hipError_t e, const char *what);

#define HIP_TRY(expr)                                          \
    do {                                                       \
        hipError_t _e = (expr);                                \
        if (_e != hipSuccess) return we_hip_fail(_e, #expr);   \
    } while (0)

struct we_network {
    int32_t S = 0, R = 0;
    int32_t max_order = 0;
    int32_t max_chg = 0;
    int32_t max_delta = 0;          // largest |change| of any species
    std::vector<RxnDesc> desc;
    std::vector<int32_t> chg_ptr, chg, dep_ptr;
    std::vector<uint16_t> dep;
    RxnDesc *d_desc = nullptr;
    int32_t *d_chg_ptr = nullptr, *d_chg = nullptr, *d_dep_ptr = nullptr;
    uint16_t *d_dep = nullptr;
    RxnInfo *d_rinfo = nullptr;
    DepEntry *d_deps = nullptr;
    int32_t *d_dpack = nullptr;     // [R][WE_DPACK_WORDS] int8 deltas (species < 32)
    std::vector<uint2> fhdr;        // factored change headers (empty: do not fit)
    std::vector<uint32_t> inc_tab;  // per species: incidence start | count << 16
    std::vector<uint16_t> inc;      // incidence lists, species by species
    uint2 *d_fhdr = nullptr;
    uint32_t *d_inc_tab = nullptr;
    uint16_t *d_inc = nullptr;
    std::vector<HillDesc> hill;     // empty: no Hill-type rates
    HillDesc *d_hill = nullptr;     // [R padded to 64]
};

// The learned committor attached to a sim (see committor.hip).
struct Committor {
    bool trained = false;
    bool active = false;            // bins come from q(x) instead of the grid
    int32_t n_in = 0;               // = number of species
    int32_t n_params = 0;
    float *d_params = nullptr;      // [n_params] FP32
    float *d_adam_m = nullptr, *d_adam_v = nullptr, *d_grad = nullptr;
    float *d_feat = nullptr;        // [2*n_in] mean, 1/std of log1p(x)
    double *d_qedges = nullptr;     // [n_qbins+1]
    float *d_wt = nullptr;          // W1 and W2 transposed ([n_in][64], [64][64]) for inference
    int32_t n_qbins = 0;
};

// Per-iteration ensemble records kept for committor training.
struct Records {
    int32_t cap_iters = 0;          // iterations that fit
    int32_t n_iters = 0;            // iterations recorded so far
    int32_t *d_x = nullptr;         // [cap_iters][n_runs*cap][S]
    int32_t *d_origin = nullptr;    // [cap_iters][n_runs*cap]
    uint8_t *d_rec = nullptr;       // [cap_iters][n_runs*cap] parent reached B this iteration
    int32_t *d_n = nullptr;         // [cap_iters][n_runs]
};

// Host copy of a sim's grid and parameters (the arrays the we_grid and
// we_params pointers referred to at init).
struct SimConfig {
    we_params p{};
    int32_t n_bins = 0, n_bins2 = 0;
    std::vector<double> coef, edges, coef2, edges2, tgt_coef;
    std::vector<uint64_t> seeds;
    std::vector<int32_t> x0, x_rec, joint;
    size_t ws_bytes = 0;
};

struct we_sim {
    const we_network *net = nullptr;
    hipStream_t stream = nullptr;
    SimArgs args{};
    int32_t kernel = WE_KERNEL_LANE;
    int32_t group_lanes = 0;        // lanes per walker of the group kernel
    int32_t *rs_binfo = nullptr;    // [n_runs][3][NB] bin-parallel resampling (workspace)
    int32_t S = 0, NB = 0, M = 0, n_runs = 0, cap = 0, max_iters = 0;
    double tau = 0.0;
    int32_t iter = 0;
    int32_t cur = 0;
    int32_t hist_iters = 0;
    bool owns_ws = false;
    void *ws = nullptr;
    int32_t *x[2] = {nullptr, nullptr};
    double *w[2] = {nullptr, nullptr};
    std::vector<int32_t> n_host;
    // per-kernel timing: 4 events per profiled iteration
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    double prof_ms[3] = {0.0, 0.0, 0.0};
    int64_t prof_iters = 0;
    // captured iterations
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t capture_stream = nullptr;
    int32_t graph_iters = 0;
    bool capturing = false;
    // committor
    Records rec;
    Committor cm;
    double *d_bin_edges_grid = nullptr;
    // the configuration the sim was built from (checkpoints, we_set_bins)
    SimConfig cfg;
};

// we_runtime.hip
extern "C" void we_batch_destroy(we_batch *b);
we_status we_read_err(we_sim *s);
we_status we_sim_bookkeeping(we_sim *s, hipStream_t st, hipEvent_t *ev);
hipError_t launch_ssa_lane(const SimArgs &a, int32_t *xs, hipStream_t st);
hipError_t launch_work_queue(const SimArgs &a, hipStream_t st);
hipError_t launch_ssa_wave(const SimArgs &a, int32_t *xs, hipStream_t st);
bool lane_kernel_fits(int32_t S, int32_t R, int32_t max_delta);
bool wave_kernel_fits(int32_t S, int32_t R);
const char *ssa_lane_name(const SimArgs &a);
const char *ssa_wave_name(const SimArgs &a);
hipError_t launch_ssa_group(const SimArgs &a, int32_t *xs, int32_t lanes, hipStream_t st);
const char *ssa_group_name(const SimArgs &a, int32_t lanes);
// reweight.hip
#define WE_RW_MAX_BINS 512
bool rw_solve_in_lds(int32_t n_bins);
hipError_t launch_reweight(const SimArgs &a, double *w_nxt, hipStream_t st);

// committor.hip
struct CommittorHost {
    bool trained = false, active = false;
    int32_t n_in = 0, n_qbins = 0;
    std::vector<float> params, adam_m, adam_v, feat, wt;
    std::vector<double> qedges;
};
we_status committor_export(we_sim *s, CommittorHost &h);
we_status committor_import(we_sim *s, const CommittorHost &h);
we_status committor_set_edges(we_sim *s, const double *edges);
hipError_t committor_record(we_sim *s, hipStream_t st);
hipError_t committor_bin(we_sim *s, int32_t *x_cur, hipStream_t st);
// A batch member's active model as device pointers (all NULL: grid bins).
struct CmBatchModel {
    const float *params, *wt, *feat;
    const double *qedges;
};
CmBatchModel committor_batch_model(const we_sim *s);
// Learned bins of all members with a model: d_models[n_sims] on the device,
// s_max >= every such member's species count.
hipError_t committor_bin_batch(const SimArgs *d_args, int32_t *const *d_x, const CmBatchModel *d_models,
                               int32_t n_sims, int64_t max_slots, int32_t s_max, hipStream_t st);
void committor_free(we_sim *s);
