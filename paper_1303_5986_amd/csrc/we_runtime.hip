// we_runtime.hip -- host side of libwe.so: network compilation, device
// layout, the iteration scheduler and the C ABI declared in include/we.h.
//
// Device layout of a sim (one workspace, 256-byte aligned pieces):
//   x[2]      int32 [n_runs][cap][S]   walker states, walker-major, double-buffered
//   w[2]      f64   [n_runs][cap]      weights
//   bin, origin int32 [n_runs][cap]    after resampling
//   ev_walker u32   [n_runs][cap]      reactions fired in the last interval
//   flux      f64   [n_runs][max_iters] weight recycled per iteration
//   ev_iter   i64   [n_runs][max_iters] reactions fired per iteration
//   scratch for resampling, histogram accumulator, small parameter arrays.
// cap = m_targ * n_bins is the most walkers a run can hold after resampling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "ssa_group_body.h"
#include "we_internal.h"

hipError_t launch_ssa_lane(const SimArgs &a, int32_t *xs, hipStream_t st);
hipError_t launch_work_queue(const SimArgs &a, hipStream_t st);
bool lane_kernel_fits(int32_t S, int32_t R, int32_t max_delta);
hipError_t launch_ssa_wave(const SimArgs &a, int32_t *xs, hipStream_t st);
bool wave_kernel_fits(int32_t S, int32_t R);
hipError_t launch_recycle_bin(const SimArgs &a, int32_t *x_cur, bool grid_bins, hipStream_t st);
int32_t resample_place_rows(const SimArgs &a, int64_t blocks);
hipError_t launch_resample(const SimArgs &a, int32_t *x_cur, const double *w_cur, int32_t *x_nxt,
                           double *w_nxt, int32_t *binfo, hipStream_t st);
hipError_t launch_advance(const SimArgs &a, hipStream_t st);
hipError_t launch_observe(const SimArgs &a, const int32_t *xs, const double *ws, hipStream_t st,
                          bool *advanced);

namespace {
thread_local std::string g_err;
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
we_status fail(we_status st, const std::string &msg) {
    g_err = msg;
    return st;
}
we_status hip_fail(hipError_t e, const char *what) {
    return fail(WE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
}  // namespace

we_status we_fail(we_status st, const std::string &msg) { return fail(st, msg); }
we_status we_hip_fail(hipError_t e, const char *what) { return hip_fail(e, what); }

namespace {
hipError_t next_event(we_sim *s, hipEvent_t *out) {
    if (s->ev_used == s->ev_pool.size()) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        s->ev_pool.push_back(e);
    }
    *out = s->ev_pool[s->ev_used++];
    return hipSuccess;
}

hipError_t drain_profile(we_sim *s) {
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return e;
    for (size_t i = 0; i + 3 < s->ev_used; i += 4) {
        float t[3] = {0.f, 0.f, 0.f};
        for (int k = 0; k < 3; ++k) {
            e = hipEventElapsedTime(&t[k], s->ev_pool[i + k], s->ev_pool[i + k + 1]);
            if (e != hipSuccess) return e;
            s->prof_ms[k] += t[k];
        }
        s->prof_iters += 1;
    }
    s->ev_used = 0;
    return hipSuccess;
}
}  // namespace

// ------------------------------------------------------------------ network
extern "C" we_status we_create_network(int32_t S, int32_t R, const int32_t *reac_ptr,
                                       const int32_t *reac_species, const int32_t *reac_mult,
                                       const int32_t *chg_ptr, const int32_t *chg_species,
                                       const int32_t *chg_delta, const double *rate_c,
                                       we_network **out) {
    if (!out) return fail(WE_EINVAL, "out is NULL");
    *out = nullptr;
    if (S <= 0 || R <= 0 || S > 65535 || R > 65535)
        return fail(WE_EINVAL, "species and reactions must be in [1, 65535]");
    if (!reac_ptr || !chg_ptr || !rate_c) return fail(WE_EINVAL, "NULL network array");
    if (reac_ptr[0] != 0 || chg_ptr[0] != 0) return fail(WE_EINVAL, "CSR must start at 0");
    we_network *net = new we_network();
    net->S = S;
    net->R = R;
    net->desc.resize(R);
    net->chg_ptr.assign(chg_ptr, chg_ptr + R + 1);
    // species -> reactions having it as a reactant (to build the dependency lists)
    std::vector<std::vector<int32_t>> users(S);
    for (int32_t j = 0; j < R; ++j) {
        RxnDesc d{};
        d.c = rate_c[j];
        if (!(rate_c[j] >= 0.0) || std::isinf(rate_c[j])) {
            delete net;
            return fail(WE_EINVAL, "rate constant must be finite and >= 0 (reaction " +
                                       std::to_string(j) + ")");
        }
        const int32_t r0 = reac_ptr[j], r1 = reac_ptr[j + 1];
        if (r1 < r0 || r1 - r0 > 2) {
            delete net;
            return fail(WE_EINVAL, "each reaction takes at most two distinct reactant species");
        }
        int32_t order = 0;
        for (int32_t p = r0; p < r1; ++p) {
            const int32_t s = reac_species[p], nu = reac_mult[p];
            if (s < 0 || s >= S || nu < 1 || nu > 3) {
                delete net;
                return fail(WE_EINVAL, "reactant species or multiplicity out of range (reaction " +
                                           std::to_string(j) + ")");
            }
            if (p == r0) { d.s1 = (uint16_t)s; d.nu1 = (uint8_t)nu; }
            else {
                if (s == d.s1) { delete net; return fail(WE_EINVAL, "repeated reactant species"); }
                d.s2 = (uint16_t)s; d.nu2 = (uint8_t)nu;
            }
            order += nu;
            users[s].push_back(j);
        }
        if (order > 3) { delete net; return fail(WE_EINVAL, "reaction order above 3"); }
        d.order = (uint8_t)order;
        const int32_t c0 = chg_ptr[j], c1 = chg_ptr[j + 1];
        if (c1 < c0) { delete net; return fail(WE_EINVAL, "change CSR not monotone"); }
        d.nchg = (uint8_t)std::min(c1 - c0, 255);
        for (int32_t p = c0; p < c1; ++p) {
            const int32_t s = chg_species[p], dl = chg_delta[p];
            if (s < 0 || s >= S || dl == 0 || dl < -3 || dl > 32767) {
                delete net;
                return fail(WE_EINVAL, "change species or delta out of range (reaction " +
                                           std::to_string(j) + ")");
            }
            for (int32_t q = c0; q < p; ++q)
                if (chg_species[q] == s) { delete net; return fail(WE_EINVAL, "repeated change species"); }
            if (dl < 0) {
                int32_t nu = 0;
                if (r1 > r0 && reac_species[r0] == s) nu = reac_mult[r0];
                if (r1 > r0 + 1 && reac_species[r0 + 1] == s) nu = reac_mult[r0 + 1];
                if (nu < -dl) {
                    delete net;
                    return fail(WE_EINVAL, "a reaction consumes a species it does not take as reactant");
                }
            }
            net->chg.push_back(pack_change(s, dl));
            net->max_delta = std::max(net->max_delta, std::abs(dl));
        }
        net->max_order = std::max(net->max_order, order);
        net->max_chg = std::max(net->max_chg, c1 - c0);
        net->desc[j] = d;
    }
    // dependency lists: reactions whose propensity reaction j changes
    net->dep_ptr.push_back(0);
    std::vector<int32_t> mark(R, -1);
    std::vector<int32_t> tmp;
    for (int32_t j = 0; j < R; ++j) {
        tmp.clear();
        for (int32_t p = chg_ptr[j]; p < chg_ptr[j + 1]; ++p)
            for (int32_t r : users[chg_species[p]])
                if (mark[r] != j) { mark[r] = j; tmp.push_back(r); }
        std::sort(tmp.begin(), tmp.end());
        for (int32_t r : tmp) net->dep.push_back((uint16_t)r);
        net->dep_ptr.push_back((int32_t)net->dep.size());
    }
    // factored form (change headers + incidence lists) for the LDS-resident
    // wave kernel, when the network fits its packed fields
    {
        bool fits = S <= FACT_MAX_SPECIES;
        size_t n_inc = 0;
        for (int32_t sp = 0; sp < S; ++sp) n_inc += users[sp].size();
        fits = fits && n_inc <= FACT_MAX_INC;
        for (int32_t j = 0; j < R && fits; ++j) {
            fits = chg_ptr[j + 1] - chg_ptr[j] <= FACT_MAX_CHANGES;
            for (int32_t p = chg_ptr[j]; p < chg_ptr[j + 1] && fits; ++p)
                fits = chg_delta[p] >= -8 && chg_delta[p] <= 7;
        }
        if (fits) {
            net->inc_tab.assign(S, 0u);
            for (int32_t sp = 0; sp < S; ++sp) {
                net->inc_tab[sp] = fact_inc_word((int32_t)net->inc.size(), (int32_t)users[sp].size());
                for (int32_t r : users[sp]) net->inc.push_back((uint16_t)r);   // ascending r
            }
            net->fhdr.assign(R, uint2{0u, 0u});
            for (int32_t j = 0; j < R; ++j) {
                uint64_t h = 0;
                for (int32_t p = chg_ptr[j]; p < chg_ptr[j + 1]; ++p)
                    h |= (uint64_t)fact_code(chg_species[p], chg_delta[p]) << (16 * (p - chg_ptr[j]));
                net->fhdr[j] = uint2{(uint32_t)h, (uint32_t)(h >> 32)};
            }
            if (net->inc.empty()) net->inc.push_back(0);
        }
    }
    std::vector<RxnInfo> rinfo(R);
    std::vector<DepEntry> deps;
    for (int32_t j = 0; j < R; ++j) {
        rinfo[j] = RxnInfo{net->dep_ptr[j], net->dep_ptr[j + 1] - net->dep_ptr[j], chg_ptr[j],
                           chg_ptr[j + 1] - chg_ptr[j]};
        for (int32_t p = net->dep_ptr[j]; p < net->dep_ptr[j + 1]; ++p) {
            const RxnDesc &d = net->desc[net->dep[p]];
            deps.push_back(DepEntry{d.c, d.s1, d.s2, d.nu1, d.nu2, net->dep[p]});
        }
    }
    // int8 delta rows for the lane kernel (species 0..31; bytes stay zero
    // for other species, and the lane kernel is not used when S > 32)
    std::vector<int32_t> dpack((size_t)R * WE_DPACK_WORDS, 0);
    for (int32_t j = 0; j < R; ++j)
        for (int32_t p = chg_ptr[j]; p < chg_ptr[j + 1]; ++p) {
            const int32_t sp = chg_species[p], dl = chg_delta[p];
            if (sp < 4 * WE_DPACK_WORDS && dl >= -128 && dl <= 127) {
                uint32_t &wd = reinterpret_cast<uint32_t &>(dpack[(size_t)j * WE_DPACK_WORDS + sp / 4]);
                wd |= ((uint32_t)dl & 0xFFu) << (8 * (sp % 4));
            }
        }
    if (deps.empty()) deps.push_back(DepEntry{});
    if (net->dep.empty()) net->dep.push_back(0);
    if (net->chg.empty()) net->chg.push_back(0);
    auto up = [&](void **dst, const void *src, size_t bytes) -> hipError_t {
        hipError_t e = hipMalloc(dst, bytes);
        if (e != hipSuccess) return e;
        return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    };
    // descriptor and delta tables padded with zero-rate rows to a multiple of
    // 64, so the lane kernel can load a whole variant's rows unconditionally
    const int32_t R_pad = (R + 63) / 64 * 64;
    std::vector<RxnDesc> desc_pad(net->desc);
    desc_pad.resize(R_pad, RxnDesc{});
    dpack.resize((size_t)R_pad * WE_DPACK_WORDS, 0);
    hipError_t e = up((void **)&net->d_desc, desc_pad.data(), sizeof(RxnDesc) * R_pad);
    if (e == hipSuccess) e = up((void **)&net->d_chg_ptr, net->chg_ptr.data(), 4 * (R + 1));
    if (e == hipSuccess) e = up((void **)&net->d_chg, net->chg.data(), 4 * net->chg.size());
    if (e == hipSuccess) e = up((void **)&net->d_dep_ptr, net->dep_ptr.data(), 4 * (R + 1));
    if (e == hipSuccess) e = up((void **)&net->d_dep, net->dep.data(), 2 * net->dep.size());
    if (e == hipSuccess) e = up((void **)&net->d_rinfo, rinfo.data(), sizeof(RxnInfo) * R);
    if (e == hipSuccess) e = up((void **)&net->d_deps, deps.data(), sizeof(DepEntry) * deps.size());
    if (e == hipSuccess) e = up((void **)&net->d_dpack, dpack.data(), 4 * dpack.size());
    if (e == hipSuccess && !net->fhdr.empty()) {
        e = up((void **)&net->d_fhdr, net->fhdr.data(), sizeof(uint2) * net->fhdr.size());
        if (e == hipSuccess) e = up((void **)&net->d_inc_tab, net->inc_tab.data(), 4 * net->inc_tab.size());
        if (e == hipSuccess) e = up((void **)&net->d_inc, net->inc.data(), 2 * net->inc.size());
    }
    if (e != hipSuccess) {
        we_destroy_network(net);
        return hip_fail(e, "network upload");
    }
    *out = net;
    return WE_OK;
}

extern "C" we_status we_set_hill(we_network *net, int32_t reaction, int32_t species, int32_t n,
                                 double K) {
    if (!net) return fail(WE_EINVAL, "NULL network");
    if (reaction < 0 || reaction >= net->R || species < 0 || species >= net->S)
        return fail(WE_EINVAL, "reaction or species out of range");
    if (n < 1 || n > 8 || !(K > 0.0) || std::isinf(K)) return fail(WE_EINVAL, "need 1 <= n <= 8 and K > 0");
    const int32_t R_pad = (net->R + 63) / 64 * 64;
    if (net->hill.empty()) {
        HillDesc none{};
        none.K = 1.0;
        none.species = -1;
        none.n = 0;
        net->hill.assign(R_pad, none);
        HIP_TRY(hipMalloc(&net->d_hill, sizeof(HillDesc) * R_pad));
    }
    net->hill[reaction].K = K;
    net->hill[reaction].species = species;
    net->hill[reaction].n = n;
    HIP_TRY(hipMemcpy(net->d_hill, net->hill.data(), sizeof(HillDesc) * R_pad, hipMemcpyHostToDevice));
    return WE_OK;
}

extern "C" void we_destroy_network(we_network *net) {
    if (!net) return;
    (void)hipFree(net->d_fhdr);
    (void)hipFree(net->d_inc_tab);
    (void)hipFree(net->d_inc);
    (void)hipFree(net->d_hill);
    (void)hipFree(net->d_desc);
    (void)hipFree(net->d_chg_ptr);
    (void)hipFree(net->d_chg);
    (void)hipFree(net->d_dep_ptr);
    (void)hipFree(net->d_dep);
    (void)hipFree(net->d_rinfo);
    (void)hipFree(net->d_deps);
    (void)hipFree(net->d_dpack);
    delete net;
}

// ------------------------------------------------------------------ sim
namespace {

struct Layout {
    size_t off[48];
    size_t total = 0;
    int n = 0;
    size_t add(size_t bytes) {
        off[n] = total;
        total += align256(std::max<size_t>(bytes, 1));
        return n++;
    }
};

// Order of the pieces in the workspace; make_layout and we_init agree on it.
enum Piece { P_X0, P_X1, P_W0, P_W1, P_BIN, P_ORIG, P_N, P_EVW, P_FLUX, P_EVI, P_SBIN, P_SREC,
             P_SLIST, P_SW, P_SCNT, P_HIST, P_SEEDS, P_BCOEF, P_EDGES, P_TCOEF, P_XREC, P_ERR,
             P_SEG, P_ITER, P_JHIST, P_SCHED, P_SEGLIST, P_QUEUE, P_NZ, P_RWF, P_RWR, P_RWS,
             P_RSB, P_COUNT };
static_assert(P_COUNT <= 48, "Layout holds at most 48 pieces");

// Counter replicas per bin of the work-queue statistics: about 16 runs per
// replica (replica run % rep), enough to spread the runs' atomics without a
// long scan of nearly empty replicas when there are few runs.
int32_t seg_rep_for(int32_t NB, int32_t n_runs) {
    return std::max(1, std::min(std::min(128, 16384 / NB), n_runs / 16));
}

Layout make_layout(int32_t S, int32_t NB, int32_t n_bins2, int32_t n_runs, int32_t cap, int32_t max_iters,
                   int32_t nh, int64_t jcells, bool rw) {
    Layout L;
    const size_t W = (size_t)n_runs * cap;
    L.add(4 * W * S); L.add(4 * W * S);
    L.add(8 * W); L.add(8 * W);
    L.add(4 * W); L.add(4 * W);
    L.add(4 * (size_t)n_runs);
    L.add(4 * W);
    L.add(8 * (size_t)n_runs * max_iters);
    L.add(8 * (size_t)n_runs * max_iters);
    L.add(4 * W); L.add(4 * W); L.add(4 * W); L.add(8 * W); L.add(4 * W);
    L.add(8 * (size_t)n_runs * std::max(nh, 1));
    L.add(8 * (size_t)n_runs);
    L.add(8 * 2 * (size_t)S);
    L.add(8 * (size_t)(NB + 1 + n_bins2 + 1));
    L.add(8 * (size_t)S);
    L.add(4 * (size_t)S);
    L.add(4);
    L.add(4 * (size_t)n_runs * max_iters);
    L.add(4);
    L.add(8 * (size_t)n_runs * (size_t)jcells);
    L.add(4 * 5 * (size_t)seg_rep_for(NB, n_runs) * (size_t)NB);
    L.add(8 * (size_t)n_runs * NB);
    L.add(8);
    L.add(4 * 3 * (size_t)S);
    const size_t nb2 = (size_t)NB * NB;
    L.add(rw ? 8 * (size_t)n_runs * nb2 : 0);
    L.add(rw && !rw_solve_in_lds(NB) ? 8 * (size_t)n_runs * nb2 : 0);
    L.add(rw ? 4 * 2 * (size_t)n_runs : 0);
    L.add(4 * 3 * (size_t)n_runs * NB);          // bin-parallel resampling: count, start, output start
    return L;
}

int32_t grid_bins(const we_grid *g) { return g->n_bins * (g->n_bins2 > 1 ? g->n_bins2 : 1); }
int32_t grid_bins2(const we_grid *g) { return g->n_bins2 > 1 ? g->n_bins2 : 1; }

we_status check_params(const we_network *net, const we_grid *g, const we_params *p) {
    if (!net || !g || !p) return fail(WE_EINVAL, "NULL argument");
    if (g->n_bins < 1 || !g->coef || !g->edges) return fail(WE_EINVAL, "bad grid");
    for (int32_t b = 0; b < g->n_bins; ++b)
        if (!(g->edges[b] < g->edges[b + 1])) return fail(WE_EINVAL, "edges must increase strictly");
    if (g->n_bins2 < 0) return fail(WE_EINVAL, "n_bins2 must be >= 0");
    if (g->n_bins2 > 1) {
        if (!g->coef2 || !g->edges2) return fail(WE_EINVAL, "the second grid axis needs coef2 and edges2");
        for (int32_t b = 0; b < g->n_bins2; ++b)
            if (!(g->edges2[b] < g->edges2[b + 1])) return fail(WE_EINVAL, "edges2 must increase strictly");
        if ((int64_t)g->n_bins * g->n_bins2 > 8192) return fail(WE_EINVAL, "at most 8192 bins");
    }
    if (!(p->tau > 0.0) || std::isinf(p->tau)) return fail(WE_EINVAL, "tau must be > 0");
    if (p->m_targ < 1 || p->n_runs < 1 || p->max_iters < 0)
        return fail(WE_EINVAL, "m_targ, n_runs must be >= 1");
    if (!p->seeds || !p->x0) return fail(WE_EINVAL, "seeds and x0 are required");
    const int64_t cap = (int64_t)p->m_targ * grid_bins(g);
    if (g->n_bins > 8192) return fail(WE_EINVAL, "at most 8192 bins");
    if (cap > (1 << 22) || cap * p->n_runs > (int64_t)1 << 30)
        return fail(WE_EINVAL, "too many walker slots");
    for (int32_t s = 0; s < net->S; ++s)
        if (p->x0[s] < 0 || p->x0[s] > WE_COUNT_MAX) return fail(WE_EINVAL, "x0 out of range");
    if (p->recycle) {
        if (!p->tgt_coef) return fail(WE_EINVAL, "recycling needs tgt_coef");
        if (p->x_rec)
            for (int32_t s = 0; s < net->S; ++s)
                if (p->x_rec[s] < 0 || p->x_rec[s] > WE_COUNT_MAX)
                    return fail(WE_EINVAL, "x_rec out of range");
    }
    if (p->hist_hi >= p->hist_lo && (p->hist_species < 0 || p->hist_species >= net->S))
        return fail(WE_EINVAL, "hist_species out of range");
    if (p->kernel < WE_KERNEL_AUTO || p->kernel > WE_KERNEL_GROUP)
        return fail(WE_EINVAL, "unknown kernel");
    if (p->n_joint < 0 || p->n_joint > 5) return fail(WE_EINVAL, "n_joint must be in [0, 5]");
    if (p->record_iters < 0) return fail(WE_EINVAL, "record_iters must be >= 0");
    if (p->rw_period < 0) return fail(WE_EINVAL, "rw_period must be >= 0");
    if (p->engine != 0 && p->engine != 1) return fail(WE_EINVAL, "engine must be 0 (SSA) or 1 (tau-leaping)");
    if (p->engine == 1 && !(p->leap_eps > 0.0 && p->leap_eps < 1.0))
        return fail(WE_EINVAL, "leap_eps must lie in (0, 1)");
    if (p->resample_rule != 0 && p->resample_rule != 1)
        return fail(WE_EINVAL, "resample_rule must be 0 (count-only) or 1 (weight-equalizing)");
    if (p->rw_period > 0 && grid_bins(g) > WE_RW_MAX_BINS)
        return fail(WE_EINVAL, "reweighting needs at most 512 bins");
    if (p->rw_period > 0 && (int64_t)p->n_runs * grid_bins(g) * grid_bins(g) > ((int64_t)1 << 31))
        return fail(WE_EINVAL, "reweighting: n_runs * n_bins^2 too large");
    if (p->n_joint > 0) {
        if (!p->joint_species || p->joint_bins < 1 || p->joint_width < 1)
            return fail(WE_EINVAL, "joint histogram needs species, bins >= 1, width >= 1");
        int64_t cells = 1;
        for (int32_t d = 0; d < p->n_joint; ++d) {
            if (p->joint_species[d] < 0 || p->joint_species[d] >= net->S)
                return fail(WE_EINVAL, "joint species out of range");
            cells *= p->joint_bins;
        }
        if (cells > (1 << 24)) return fail(WE_EINVAL, "joint histogram too large");
    }
    return WE_OK;
}

int64_t joint_cells(const we_params *p) {
    int64_t c = p->n_joint > 0 ? 1 : 0;
    for (int32_t d = 0; d < p->n_joint; ++d) c *= p->joint_bins;
    return c;
}

}  // namespace

extern "C" we_status we_workspace_size(const we_network *net, const we_grid *g, const we_params *p,
                                       size_t *bytes) {
    we_status st = check_params(net, g, p);
    if (st != WE_OK) return st;
    if (!bytes) return fail(WE_EINVAL, "bytes is NULL");
    const int32_t nh = p->hist_hi >= p->hist_lo ? p->hist_hi - p->hist_lo + 1 : 0;
    *bytes = make_layout(net->S, grid_bins(g), grid_bins2(g), p->n_runs, p->m_targ * grid_bins(g),
                         std::max(p->max_iters, 1), nh, joint_cells(p), p->rw_period > 0).total;
    return WE_OK;
}

// Bin coefficients, edges and the lists of species with nonzero bin and
// target coefficients, from the sim's configuration, on the sim's stream
// (synchronous).
hipError_t upload_grid(we_sim *s) {
    SimArgs &a = s->args;
    const SimConfig &cf = s->cfg;
    const int32_t S = s->S, NB1 = cf.n_bins, NB2 = cf.n_bins2 > 1 ? cf.n_bins2 : 1;
    std::vector<double> coefs, edges_all;
    std::vector<int32_t> nz;
    coefs.assign(2 * (size_t)S, 0.0);
    edges_all.assign((size_t)NB1 + 1 + NB2 + 1, 0.0);
    for (int32_t sp = 0; sp < S; ++sp) {
        coefs[sp] = cf.coef[sp];
        if (NB2 > 1) coefs[S + sp] = cf.coef2[sp];
    }
    for (int32_t b = 0; b <= NB1; ++b) edges_all[b] = cf.edges[b];
    for (int32_t b = 0; b <= NB2; ++b) edges_all[NB1 + 1 + b] = NB2 > 1 ? cf.edges2[b] : (double)b;
    nz.assign(3 * (size_t)S, 0);
    a.n_bin_nz = a.n_tgt_nz = a.n_bin_nz2 = 0;
    for (int32_t sp = 0; sp < S; ++sp) {
        if (cf.coef[sp] != 0.0) nz[a.n_bin_nz++] = sp;
        if (cf.tgt_coef[sp] != 0.0) nz[S + a.n_tgt_nz++] = sp;
        if (NB2 > 1 && cf.coef2[sp] != 0.0) nz[2 * S + a.n_bin_nz2++] = sp;
    }
    hipError_t e = hipMemcpyAsync((void *)a.bin_coef, coefs.data(), 8 * coefs.size(), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync((void *)a.edges, edges_all.data(), 8 * edges_all.size(), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync((void *)a.bin_nz, nz.data(), 4 * nz.size(), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    return e;
}

extern "C" we_status we_init(const we_network *net, const we_grid *g, const we_params *p,
                             void *hip_stream, void *workspace, size_t workspace_bytes,
                             we_sim **out) {
    if (!out) return fail(WE_EINVAL, "out is NULL");
    *out = nullptr;
    we_status st = check_params(net, g, p);
    if (st != WE_OK) return st;
    const int32_t S = net->S, NB = grid_bins(g), NB1 = g->n_bins, NB2 = grid_bins2(g);
    const int32_t M = p->m_targ, n_runs = p->n_runs;
    const int32_t cap = M * NB, max_iters = std::max(p->max_iters, 1);
    const int32_t nh = p->hist_hi >= p->hist_lo ? p->hist_hi - p->hist_lo + 1 : 0;
    int32_t kernel = p->kernel;
    const bool hill = !net->hill.empty();
    const bool other = kernel == WE_KERNEL_WAVE || kernel == WE_KERNEL_GROUP;
    if (p->engine == 1 && (hill || other || S > 8 || net->R > 16 || net->max_delta > 127))
        return fail(WE_EINVAL, "tau-leaping runs on the lane kernel only (mass action, S <= 8, R <= 16)");
    if (hill && (other || S > 8 || net->R > 16 || net->max_delta > 127))
        return fail(WE_EINVAL, "Hill-type rates run on the lane kernel only (S <= 8, R <= 16)");
    int32_t group_lanes = 0;
    if (kernel == WE_KERNEL_GROUP) {
        const int32_t wpw = p->walkers_per_wave;
        if (!(wpw == 2 || wpw == 4 || wpw == 8 || wpw == 16 || wpw == 32))
            return fail(WE_EINVAL, "the group kernel takes 2, 4, 8, 16 or 32 walkers per wave");
        group_lanes = 64 / wpw;
        if (!group_kernel_fits(S, net->R, group_lanes))
            return fail(WE_EINVAL, "network does not fit the group kernel ((64 / L) * S <= 4096, R <= 65535)");
    }
    if (kernel == WE_KERNEL_AUTO)
        kernel = hill || (lane_kernel_fits(S, net->R, net->max_delta) && net->R <= 32) ? WE_KERNEL_LANE
                                                                                       : WE_KERNEL_WAVE;
    if (kernel == WE_KERNEL_LANE && !lane_kernel_fits(S, net->R, net->max_delta))
        return fail(WE_EINVAL, "network does not fit the lane-per-walker kernel (S <= 32, R <= 64, |change| <= 127)");
    if (kernel == WE_KERNEL_WAVE && (!wave_kernel_fits(S, net->R) || net->max_chg > 64))
        return fail(WE_EINVAL, "network too large for the wave-per-walker kernel");

    const int64_t jcells = joint_cells(p);
    Layout L = make_layout(S, NB, NB2, n_runs, cap, max_iters, nh, jcells, p->rw_period > 0);
    we_sim *s = new we_sim();
    s->net = net;
    s->stream = (hipStream_t)hip_stream;
    s->kernel = kernel;
    s->group_lanes = group_lanes;
    s->S = S; s->NB = NB; s->M = M; s->n_runs = n_runs; s->cap = cap; s->max_iters = max_iters;
    s->tau = p->tau;
    if (workspace) {
        if (workspace_bytes < L.total || ((uintptr_t)workspace & 255)) {
            delete s;
            return fail(WE_EINVAL, "workspace too small or not 256-byte aligned");
        }
        s->ws = workspace;
    } else {
        hipError_t e = hipMalloc(&s->ws, L.total);
        if (e != hipSuccess) { delete s; return fail(WE_ENOMEM, "hipMalloc of the workspace failed"); }
        s->owns_ws = true;
    }
    char *base = (char *)s->ws;
    auto at = [&](int piece) { return (void *)(base + L.off[piece]); };
    s->x[0] = (int32_t *)at(P_X0); s->x[1] = (int32_t *)at(P_X1);
    s->w[0] = (double *)at(P_W0); s->w[1] = (double *)at(P_W1);
    SimArgs &a = s->args;
    a.desc = net->d_desc; a.chg_ptr = net->d_chg_ptr; a.chg = net->d_chg; a.dpack = net->d_dpack;
    a.dep_ptr = net->d_dep_ptr; a.dep = net->d_dep;
    a.rinfo = net->d_rinfo; a.deps = net->d_deps;
    a.hill = hill ? net->d_hill : nullptr;
    a.fhdr = net->d_fhdr;
    a.inc_tab = net->d_inc_tab;
    a.inc = net->d_inc;
    a.n_inc = (int32_t)net->inc.size();
    a.n_chg = (int32_t)net->chg.size();
    a.engine = p->engine;
    a.leap_eps = p->engine == 1 ? p->leap_eps : 0.0;
    a.S = S; a.R = net->R;
    a.n_runs = n_runs; a.cap = cap; a.n_bins = NB; a.m_targ = M; a.max_iters = max_iters;
    a.rs_rule = p->resample_rule;
    a.tau = p->tau;
    a.seeds = (const uint64_t *)at(P_SEEDS);
    a.bin_coef = (const double *)at(P_BCOEF);
    a.edges = (const double *)at(P_EDGES);
    a.n_bins1 = NB1;
    a.n_bins2 = NB2;
    a.bin_coef2 = a.bin_coef + S;
    a.edges2 = a.edges + NB1 + 1;
    a.recycle = p->recycle ? 1 : 0;
    a.tgt_thr = p->tgt_thr;
    a.tgt_coef = (const double *)at(P_TCOEF);
    a.bin_nz = (const int32_t *)at(P_NZ);
    a.tgt_nz = a.bin_nz + S;
    a.bin_nz2 = a.bin_nz + 2 * S;
    a.x_rec = (const int32_t *)at(P_XREC);
    a.n_walk = (int32_t *)at(P_N);
    a.bin = (int32_t *)at(P_BIN);
    a.origin = (int32_t *)at(P_ORIG);
    a.ev_walker = (uint32_t *)at(P_EVW);
    a.flux = (double *)at(P_FLUX);
    a.ev_iter = (int64_t *)at(P_EVI);
    a.seg_iter = (int32_t *)at(P_SEG);
    a.s_bin = (int32_t *)at(P_SBIN); a.s_rec = (int32_t *)at(P_SREC);
    a.s_list = (int32_t *)at(P_SLIST); a.s_w = (double *)at(P_SW); a.s_cnt = (int32_t *)at(P_SCNT);
    a.hist = (double *)at(P_HIST);
    a.hist_species = nh > 0 ? p->hist_species : 0;
    a.hist_lo = p->hist_lo;
    a.nh = nh;
    a.err = (int32_t *)at(P_ERR);
    a.iter_dev = (uint32_t *)at(P_ITER);
    a.jhist = (double *)at(P_JHIST);
    a.queue_stats = 1;
    a.place_rows = resample_place_rows(a, n_runs);
    a.rw_period = p->rw_period;
    a.rw_reset = p->rw_reset ? 1 : 0;
    a.rw_F = p->rw_period > 0 ? (double *)at(P_RWF) : nullptr;
    a.rw_R = p->rw_period > 0 && !rw_solve_in_lds(NB) ? (double *)at(P_RWR) : nullptr;
    a.rw_stat = p->rw_period > 0 ? (int32_t *)at(P_RWS) : nullptr;
    a.seg_rep = seg_rep_for(NB, n_runs);
    a.ev_bin = (float *)at(P_SCHED);
    a.n_bin = (int32_t *)at(P_SCHED) + a.seg_rep * NB;
    a.occ_bin = a.n_bin + a.seg_rep * NB;
    a.seg_off = a.occ_bin + a.seg_rep * NB;
    a.seg_cur = a.seg_off + a.seg_rep * NB;
    a.seg = (int2 *)at(P_SEGLIST);
    a.queue = (uint32_t *)at(P_QUEUE);
    s->rs_binfo = (int32_t *)at(P_RSB);
    a.n_joint = p->n_joint;
    a.joint_bins = p->n_joint > 0 ? p->joint_bins : 1;
    a.joint_width = p->n_joint > 0 ? p->joint_width : 1;
    a.jcells = (int32_t)jcells;
    for (int32_t d = 0; d < 5; ++d) a.joint_species[d] = d < p->n_joint ? p->joint_species[d] : 0;

    // initial ensemble: m_targ walkers at x0, weight 1/m_targ
    const size_t W = (size_t)n_runs * cap;
    std::vector<int32_t> hx(W * S, 0);
    std::vector<double> hw(W, 0.0);
    std::vector<int32_t> hn(n_runs, M), horig(W, -1), hbin(W, 0);
    for (int32_t r = 0; r < n_runs; ++r)
        for (int32_t k = 0; k < M; ++k) {
            for (int32_t q = 0; q < S; ++q) hx[((size_t)r * cap + k) * S + q] = p->x0[q];
            hw[(size_t)r * cap + k] = 1.0 / (double)M;
        }
    const hipStream_t st_ = s->stream;
    auto put = [&](int piece, const void *src, size_t bytes) -> hipError_t {
        return hipMemcpyAsync(at(piece), src, bytes, hipMemcpyHostToDevice, st_);
    };
    hipError_t e = hipMemsetAsync(s->ws, 0, L.total, st_);
    if (e == hipSuccess) e = put(P_X0, hx.data(), 4 * W * S);
    if (e == hipSuccess) e = put(P_W0, hw.data(), 8 * W);
    if (e == hipSuccess) e = put(P_N, hn.data(), 4 * (size_t)n_runs);
    if (e == hipSuccess) e = put(P_ORIG, horig.data(), 4 * W);
    if (e == hipSuccess) e = put(P_SEEDS, p->seeds, 8 * (size_t)n_runs);
    // the configuration, kept for checkpoints and we_set_bins
    SimConfig &cf = s->cfg;
    cf.p = *p;
    cf.p.kernel = kernel;
    cf.n_bins = NB1;
    cf.n_bins2 = g->n_bins2;
    cf.coef.assign(g->coef, g->coef + S);
    cf.edges.assign(g->edges, g->edges + NB1 + 1);
    if (NB2 > 1) {
        cf.coef2.assign(g->coef2, g->coef2 + S);
        cf.edges2.assign(g->edges2, g->edges2 + NB2 + 1);
    }
    cf.tgt_coef.assign(S, 0.0);
    if (p->tgt_coef) cf.tgt_coef.assign(p->tgt_coef, p->tgt_coef + S);
    cf.seeds.assign(p->seeds, p->seeds + n_runs);
    cf.x0.assign(p->x0, p->x0 + S);
    cf.x_rec.assign(p->x_rec ? p->x_rec : p->x0, (p->x_rec ? p->x_rec : p->x0) + S);
    cf.joint.assign(p->joint_species ? p->joint_species : p->x0,
                    (p->joint_species ? p->joint_species : p->x0) + (p->n_joint > 0 ? p->n_joint : 0));
    cf.ws_bytes = L.total;
    cf.p.seeds = nullptr; cf.p.x0 = nullptr; cf.p.tgt_coef = nullptr; cf.p.x_rec = nullptr;
    cf.p.joint_species = nullptr;
    if (e == hipSuccess) e = put(P_TCOEF, cf.tgt_coef.data(), 8 * (size_t)S);
    if (e == hipSuccess) e = upload_grid(s);
    if (e == hipSuccess) e = put(P_XREC, p->x_rec ? p->x_rec : p->x0, 4 * (size_t)S);
    if (e == hipSuccess) e = hipStreamSynchronize(st_);
    if (e != hipSuccess) {
        we_destroy(s);
        return hip_fail(e, "sim upload");
    }
    s->n_host = hn;
    if (p->record_iters > 0) {
        Records &R = s->rec;
        R.cap_iters = p->record_iters;
        const size_t W = (size_t)n_runs * cap;
        hipError_t er = hipMalloc(&R.d_x, 4 * W * S * R.cap_iters);
        if (er == hipSuccess) er = hipMalloc(&R.d_origin, 4 * W * R.cap_iters);
        if (er == hipSuccess) er = hipMalloc(&R.d_rec, W * R.cap_iters);
        if (er == hipSuccess) er = hipMalloc(&R.d_n, 4 * (size_t)n_runs * R.cap_iters);
        if (er != hipSuccess) {
            we_destroy(s);
            return fail(WE_ENOMEM, "record buffer allocation failed");
        }
    }
    *out = s;
    return WE_OK;
}

extern "C" we_status we_set_ensemble(we_sim *s, int32_t run, int32_t n, const int32_t *x,
                                     const double *w) {
    if (!s) return fail(WE_EINVAL, "NULL sim");
    if (s->iter != 0) return fail(WE_ESTATE, "ensemble can only be set before the first step");
    if (run < 0 || run >= s->n_runs) return fail(WE_EINVAL, "run out of range");
    if (n < 0 || n > s->cap) return fail(WE_ECAPACITY, "more walkers than slots");
    if (n > 0 && (!x || !w)) return fail(WE_EINVAL, "NULL ensemble arrays");
    for (int64_t i = 0; i < (int64_t)n * s->S; ++i)
        if (x[i] < 0 || x[i] > WE_COUNT_MAX) return fail(WE_EINVAL, "count out of range");
    for (int32_t i = 0; i < n; ++i)
        if (!(w[i] >= 0.0) || std::isinf(w[i])) return fail(WE_EINVAL, "weights must be finite, >= 0");
    const size_t base = (size_t)run * s->cap;
    HIP_TRY(hipMemcpyAsync(s->x[s->cur] + base * s->S, x, 4 * (size_t)n * s->S,
                           hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->w[s->cur] + base, w, 8 * (size_t)n, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->args.n_walk + run, &n, 4, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->n_host[run] = n;
    return WE_OK;
}

namespace {
we_status read_err(we_sim *s) {
    int32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, s->args.err, 4, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (err & WE_DERR_OVERFLOW) return fail(WE_EOVERFLOW, "a copy number left [0, WE_COUNT_MAX]");
    if (err & WE_DERR_CAPACITY) return fail(WE_ECAPACITY, "resampling exceeded the slot reservation");
    if (err & WE_DERR_SELECT) return fail(WE_EDEVICE, "reaction selection found no positive propensity");
    return WE_OK;
}
}  // namespace

we_status we_read_err(we_sim *s) { return read_err(s); }

// Everything after propagation: recycle and bin, resample and gather,
// observables, the device iteration counter, records; flips the buffers.
// ev (optional) points at three events: ev[0] already recorded after the
// SSA step; ev[1] and ev[2] are recorded here.
we_status we_sim_bookkeeping(we_sim *s, hipStream_t st, hipEvent_t *ev) {
    SimArgs &a = s->args;
    const int32_t c = s->cur, nx = 1 - c;
    hipError_t e = launch_recycle_bin(a, s->x[c], !s->cm.active, st);
    if (e != hipSuccess) return hip_fail(e, "recycle/bin launch");
    if (s->cm.active) {
        e = committor_bin(s, s->x[c], st);
        if (e != hipSuccess) return hip_fail(e, "committor bin launch");
    }
    e = launch_resample(a, s->x[c], s->w[c], s->x[nx], s->w[nx], s->rs_binfo, st);
    if (e != hipSuccess) return hip_fail(e, "resample launch");
    if (a.rw_period > 0) {
        e = launch_reweight(a, s->w[nx], st);
        if (e != hipSuccess) return hip_fail(e, "reweight launch");
    }
    if (ev) HIP_TRY(hipEventRecord(ev[1], st));
    bool advanced = false;
    if (a.nh > 0 || a.n_joint > 0) {
        e = launch_observe(a, s->x[nx], s->w[nx], st, &advanced);
        if (e != hipSuccess) return hip_fail(e, "observe launch");
    }
    if (!advanced) {
        e = launch_advance(a, st);
        if (e != hipSuccess) return hip_fail(e, "advance launch");
    }
    if (ev) HIP_TRY(hipEventRecord(ev[2], st));
    s->cur = nx;
    if (!s->capturing) {
        e = committor_record(s, st);
        if (e != hipSuccess) return hip_fail(e, "record launch");
    }
    return WE_OK;
}

namespace {
// Launch one WE iteration on stream st.  Buffers alternate between
// iterations; the iteration number is read by the kernels from device memory.
we_status launch_iteration(we_sim *s, hipStream_t st, bool profile) {
    SimArgs &a = s->args;
    const int32_t c = s->cur;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    {
        const hipError_t e = launch_work_queue(a, st);
        if (e != hipSuccess) return hip_fail(e, "work-queue launch");
    }
    if (profile) {
        if (s->ev_used + 4 > 4096) HIP_TRY(drain_profile(s));
        for (int k = 0; k < 4; ++k) HIP_TRY(next_event(s, &ev[k]));
        HIP_TRY(hipEventRecord(ev[0], st));
    }
    hipError_t e = (s->kernel == WE_KERNEL_WAVE)    ? launch_ssa_wave(a, s->x[c], st)
                   : (s->kernel == WE_KERNEL_GROUP) ? launch_ssa_group(a, s->x[c], s->group_lanes, st)
                                                    : launch_ssa_lane(a, s->x[c], st);
    if (e != hipSuccess) return hip_fail(e, "SSA launch");
    if (profile) HIP_TRY(hipEventRecord(ev[1], st));
    return we_sim_bookkeeping(s, st, profile ? ev + 1 : nullptr);
}
}  // namespace

extern "C" we_status we_step_intervals(we_sim *s, int32_t n) {
    if (!s) return fail(WE_EINVAL, "NULL sim");
    if (n < 0) return fail(WE_EINVAL, "negative iteration count");
    if ((int64_t)s->iter + n > s->max_iters) return fail(WE_ECAPACITY, "max_iters exceeded");
    for (int32_t i = 0; i < n; ++i) {
        we_status st = launch_iteration(s, s->stream, s->profiling);
        if (st != WE_OK) return st;
        if (s->args.nh > 0) s->hist_iters += 1;
        s->iter += 1;
    }
    return WE_OK;
}

extern "C" we_status we_graph_capture(we_sim *s, int32_t n) {
    if (!s) return fail(WE_EINVAL, "NULL sim");
    if (n <= 0 || (n & 1)) return fail(WE_EINVAL, "capture an even, positive number of iterations");
    if (s->graph_exec) {
        (void)hipGraphExecDestroy(s->graph_exec);
        s->graph_exec = nullptr;
    }
    if (!s->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (s->rec.cap_iters > 0 && s->rec.n_iters < s->rec.cap_iters)
        return fail(WE_ESTATE, "recording is active: step eagerly until the record buffer is full");
    const int32_t cur0 = s->cur;
    HIP_TRY(hipStreamBeginCapture(s->capture_stream, hipStreamCaptureModeThreadLocal));
    we_status st = WE_OK;
    s->capturing = true;
    for (int32_t i = 0; i < n && st == WE_OK; ++i) st = launch_iteration(s, s->capture_stream, false);
    s->capturing = false;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s->capture_stream, &g);
    s->cur = cur0;   // n is even: a replay leaves the buffers where they were
    if (st != WE_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&s->graph_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    s->graph_iters = n;
    return WE_OK;
}

extern "C" we_status we_graph_replay(we_sim *s, int32_t times) {
    if (!s) return fail(WE_EINVAL, "NULL sim");
    if (!s->graph_exec) return fail(WE_ESTATE, "no captured graph");
    if (times < 0) return fail(WE_EINVAL, "negative replay count");
    if ((int64_t)s->iter + (int64_t)times * s->graph_iters > s->max_iters)
        return fail(WE_ECAPACITY, "max_iters exceeded");
    for (int32_t r = 0; r < times; ++r) {
        HIP_TRY(hipGraphLaunch(s->graph_exec, s->stream));
        s->iter += s->graph_iters;
        if (s->args.nh > 0) s->hist_iters += s->graph_iters;
    }
    return WE_OK;
}

extern "C" we_status we_synchronize(we_sim *s) {
    if (!s) return fail(WE_EINVAL, "NULL sim");
    return read_err(s);
}

extern "C" we_status we_get_walkers(we_sim *s, int32_t run, int32_t *n, int32_t *x, double *w,
                                    int32_t *bin, int32_t *origin) {
    if (!s) return fail(WE_EINVAL, "NULL sim");
    if (run < 0 || run >= s->n_runs) return fail(WE_EINVAL, "run out of range");
    we_status st = read_err(s);
    if (st != WE_OK) return st;
    int32_t nn = 0;
    HIP_TRY(hipMemcpy(&nn, s->args.n_walk + run, 4, hipMemcpyDeviceToHost));
    const size_t base = (size_t)run * s->cap;
    if (n) *n = nn;
    if (x) HIP_TRY(hipMemcpy(x, s->x[s->cur] + base * s->S, 4 * (size_t)nn * s->S, hipMemcpyDeviceToHost));
    if (w) HIP_TRY(hipMemcpy(w, s->w[s->cur] + base, 8 * (size_t)nn, hipMemcpyDeviceToHost));
    if (bin) HIP_TRY(hipMemcpy(bin, s->args.bin + base, 4 * (size_t)nn, hipMemcpyDeviceToHost));
    if (origin) HIP_TRY(hipMemcpy(origin, s->args.origin + base, 4 * (size_t)nn, hipMemcpyDeviceToHost));
    return WE_OK;
}

extern "C" we_status we_histogram(we_sim *s, int32_t run, int32_t species, int32_t lo, int32_t hi,
                                  double *out) {
    if (!s || !out) return fail(WE_EINVAL, "NULL argument");
    if (species < 0 || species >= s->S || hi < lo) return fail(WE_EINVAL, "bad histogram range");
    int32_t n = 0;
    std::vector<int32_t> x((size_t)s->cap * s->S);
    std::vector<double> w(s->cap);
    we_status st = we_get_walkers(s, run, &n, x.data(), w.data(), nullptr, nullptr);
    if (st != WE_OK) return st;
    std::fill(out, out + (hi - lo + 1), 0.0);
    for (int32_t k = 0; k < n; ++k) {
        const int32_t v = x[(size_t)k * s->S + species];
        if (v >= lo && v <= hi) out[v - lo] += w[k];
    }
    return WE_OK;
}

extern "C" we_status we_histogram_accum(we_sim *s, double *out, int32_t *n_iters) {
    if (!s || !out) return fail(WE_EINVAL, "NULL argument");
    if (s->args.nh <= 0) return fail(WE_ESTATE, "no histogram was requested at init");
    we_status st = read_err(s);
    if (st != WE_OK) return st;
    HIP_TRY(hipMemcpy(out, s->args.hist, 8 * (size_t)s->n_runs * s->args.nh, hipMemcpyDeviceToHost));
    if (n_iters) *n_iters = s->hist_iters;
    return WE_OK;
}

extern "C" we_status we_joint_histogram(we_sim *s, double *out) {
    if (!s || !out) return fail(WE_EINVAL, "NULL argument");
    if (s->args.n_joint <= 0) return fail(WE_ESTATE, "no joint histogram was requested at init");
    we_status st = read_err(s);
    if (st != WE_OK) return st;
    HIP_TRY(hipMemcpy(out, s->args.jhist, 8 * (size_t)s->n_runs * s->args.jcells, hipMemcpyDeviceToHost));
    return WE_OK;
}

extern "C" we_status we_flux(we_sim *s, int32_t run, int32_t first, int32_t count, double *out) {
    if (!s || (!out && count > 0)) return fail(WE_EINVAL, "NULL argument");
    if (run < 0 || run >= s->n_runs || first < 0 || count < 0 || first + count > s->iter)
        return fail(WE_EINVAL, "flux range out of bounds");
    we_status st = read_err(s);
    if (st != WE_OK) return st;
    if (count > 0)
        HIP_TRY(hipMemcpy(out, s->args.flux + (size_t)run * s->max_iters + first, 8 * (size_t)count,
                          hipMemcpyDeviceToHost));
    return WE_OK;
}

extern "C" we_status we_mfpt(we_sim *s, int32_t discard, double *mfpt, double *flux_mean,
                             double *flux_sem) {
    if (!s) return fail(WE_EINVAL, "NULL sim");
    if (discard < 0 || discard >= s->iter) return fail(WE_EINVAL, "discard must be < iterations run");
    const int32_t cnt = s->iter - discard;
    std::vector<double> f(cnt), per_run(s->n_runs);
    for (int32_t r = 0; r < s->n_runs; ++r) {
        we_status st = we_flux(s, r, discard, cnt, f.data());
        if (st != WE_OK) return st;
        double acc = 0.0;
        for (double v : f) acc += v;
        per_run[r] = acc / cnt / s->tau;
    }
    double mean = 0.0;
    for (double v : per_run) mean += v;
    mean /= s->n_runs;
    double var = 0.0;
    for (double v : per_run) var += (v - mean) * (v - mean);
    const double sem = s->n_runs > 1 ? std::sqrt(var / (s->n_runs - 1) / s->n_runs) : NAN;
    if (flux_mean) *flux_mean = mean;
    if (flux_sem) *flux_sem = sem;
    if (mfpt) *mfpt = mean > 0.0 ? 1.0 / mean : INFINITY;
    return WE_OK;
}

extern "C" we_status we_events_series(we_sim *s, int32_t first, int32_t count, int64_t *out) {
    if (!s || (!out && count > 0)) return fail(WE_EINVAL, "NULL argument");
    if (first < 0 || count < 0 || first + count > s->iter) return fail(WE_EINVAL, "range out of bounds");
    we_status st = read_err(s);
    if (st != WE_OK) return st;
    std::vector<int64_t> buf((size_t)s->n_runs * s->max_iters);
    HIP_TRY(hipMemcpy(buf.data(), s->args.ev_iter, 8 * buf.size(), hipMemcpyDeviceToHost));
    for (int32_t i = 0; i < count; ++i) {
        int64_t acc = 0;
        for (int32_t r = 0; r < s->n_runs; ++r) acc += buf[(size_t)r * s->max_iters + first + i];
        out[i] = acc;
    }
    return WE_OK;
}

extern "C" we_status we_walker_events(we_sim *s, int32_t run, int32_t *n, uint32_t *out) {
    if (!s || !n || !out) return fail(WE_EINVAL, "NULL argument");
    if (run < 0 || run >= s->n_runs) return fail(WE_EINVAL, "run out of range");
    if (s->iter < 1) return fail(WE_ESTATE, "no interval propagated yet");
    we_status st = read_err(s);
    if (st != WE_OK) return st;
    const int32_t last = s->iter - 1;
    int32_t nn = 0;
    if (last < s->max_iters)
        HIP_TRY(hipMemcpy(&nn, s->args.seg_iter + (size_t)run * s->max_iters + last, 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(out, s->args.ev_walker + (size_t)run * s->cap, 4 * (size_t)s->cap, hipMemcpyDeviceToHost));
    *n = nn;
    return WE_OK;
}

extern "C" we_status we_rw_flux_matrix(we_sim *s, int32_t run, double *out) {
    if (!s || !out) return fail(WE_EINVAL, "NULL argument");
    if (!s->args.rw_F) return fail(WE_EINVAL, "reweighting is off");
    if (run < 0 || run >= s->n_runs) return fail(WE_EINVAL, "run out of range");
    we_status st = read_err(s);
    if (st != WE_OK) return st;
    const size_t nb2 = (size_t)s->NB * s->NB;
    HIP_TRY(hipMemcpy(out, s->args.rw_F + (size_t)run * nb2, 8 * nb2, hipMemcpyDeviceToHost));
    return WE_OK;
}

extern "C" we_status we_rw_counts(we_sim *s, int32_t run, int32_t *applied, int32_t *skipped) {
    if (!s) return fail(WE_EINVAL, "NULL sim");
    if (!s->args.rw_stat) return fail(WE_EINVAL, "reweighting is off");
    if (run < 0 || run >= s->n_runs) return fail(WE_EINVAL, "run out of range");
    we_status st = read_err(s);
    if (st != WE_OK) return st;
    int32_t c[2] = {0, 0};
    HIP_TRY(hipMemcpy(c, s->args.rw_stat + 2 * (size_t)run, 8, hipMemcpyDeviceToHost));
    if (applied) *applied = c[0];
    if (skipped) *skipped = c[1];
    return WE_OK;
}

extern "C" we_status we_counters(we_sim *s, int64_t *events, int64_t *segments, int32_t *iterations) {
    if (!s) return fail(WE_EINVAL, "NULL sim");
    we_status st = read_err(s);
    if (st != WE_OK) return st;
    std::vector<int64_t> buf((size_t)s->n_runs * s->max_iters);
    HIP_TRY(hipMemcpy(buf.data(), s->args.ev_iter, 8 * buf.size(), hipMemcpyDeviceToHost));
    std::vector<int32_t> seg((size_t)s->n_runs * s->max_iters);
    HIP_TRY(hipMemcpy(seg.data(), s->args.seg_iter, 4 * seg.size(), hipMemcpyDeviceToHost));
    int64_t ev = 0, sg = 0;
    for (int32_t r = 0; r < s->n_runs; ++r)
        for (int32_t i = 0; i < s->iter; ++i) {
            ev += buf[(size_t)r * s->max_iters + i];
            sg += seg[(size_t)r * s->max_iters + i];
        }
    if (events) *events = ev;
    if (segments) *segments = sg;
    if (iterations) *iterations = s->iter;
    return WE_OK;
}

extern "C" we_status we_profile(we_sim *s, int32_t enable) {
    if (!s) return fail(WE_EINVAL, "NULL sim");
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->ev_used = 0;
    s->prof_ms[0] = s->prof_ms[1] = s->prof_ms[2] = 0.0;
    s->prof_iters = 0;
    s->profiling = enable != 0;
    return WE_OK;
}

extern "C" we_status we_profile_read(we_sim *s, double *ms_propagate, double *ms_resample,
                                     double *ms_observe, int64_t *iterations) {
    if (!s) return fail(WE_EINVAL, "NULL sim");
    HIP_TRY(drain_profile(s));
    if (ms_propagate) *ms_propagate = s->prof_ms[0];
    if (ms_resample) *ms_resample = s->prof_ms[1];
    if (ms_observe) *ms_observe = s->prof_ms[2];
    if (iterations) *iterations = s->prof_iters;
    return WE_OK;
}

extern "C" const char *we_propagation_kernel(const we_sim *s) {
    if (!s) return "";
    if (s->kernel == WE_KERNEL_GROUP) return ssa_group_name(s->args, s->group_lanes);
    return s->kernel == WE_KERNEL_LANE ? ssa_lane_name(s->args) : ssa_wave_name(s->args);
}

extern "C" we_status we_set_bins(we_sim *s, const we_bins *b) {
    if (!s || !b) return fail(WE_EINVAL, "NULL argument");
    if (b->kind == WE_BINS_LEARNED) {
        if (b->grid) return fail(WE_EINVAL, "learned bins take no grid");
        const bool was = s->cm.active;
        we_status e = we_use_committor_bins(s, 1);
        if (e == WE_OK && b->qedges && (e = committor_set_edges(s, b->qedges)) != WE_OK) s->cm.active = was;
        return e;
    }
    if (b->kind != WE_BINS_GRID) return fail(WE_EINVAL, "unknown bin kind");
    if (b->qedges) return fail(WE_EINVAL, "logit edges go with learned bins");
    if (s->graph_exec) return fail(WE_ESTATE, "recapture the graph after switching bins");
    if (b->grid) {
        const we_grid *g = b->grid;
        SimConfig &cf = s->cfg;
        if (g->n_bins != cf.n_bins || (g->n_bins2 > 1 ? g->n_bins2 : 1) != (cf.n_bins2 > 1 ? cf.n_bins2 : 1))
            return fail(WE_EINVAL, "a new grid must keep the number of bins on each axis");
        if (!g->coef || !g->edges || (g->n_bins2 > 1 && (!g->coef2 || !g->edges2)))
            return fail(WE_EINVAL, "bad grid");
        for (int32_t k = 0; k < g->n_bins; ++k)
            if (!(g->edges[k] < g->edges[k + 1])) return fail(WE_EINVAL, "edges must increase strictly");
        for (int32_t k = 0; g->n_bins2 > 1 && k < g->n_bins2; ++k)
            if (!(g->edges2[k] < g->edges2[k + 1])) return fail(WE_EINVAL, "edges2 must increase strictly");
        HIP_TRY(hipStreamSynchronize(s->stream));
        cf.coef.assign(g->coef, g->coef + s->S);
        cf.edges.assign(g->edges, g->edges + g->n_bins + 1);
        if (g->n_bins2 > 1) {
            cf.coef2.assign(g->coef2, g->coef2 + s->S);
            cf.edges2.assign(g->edges2, g->edges2 + g->n_bins2 + 1);
        }
        HIP_TRY(upload_grid(s));
    }
    s->cm.active = false;
    return WE_OK;
}

extern "C" void we_destroy(we_sim *s) {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    else (void)hipDeviceSynchronize();
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    committor_free(s);
    (void)hipFree(s->rec.d_x);
    (void)hipFree(s->rec.d_origin);
    (void)hipFree(s->rec.d_rec);
    (void)hipFree(s->rec.d_n);
    if (s->capture_stream) (void)hipStreamDestroy(s->capture_stream);
    if (s->owns_ws) (void)hipFree(s->ws);
    delete s;
}

extern "C" const char *we_last_error(void) { return g_err.c_str(); }
