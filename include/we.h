/*
 * we.h -- C ABI of libwe.so, weighted-ensemble (WE) stochastic simulation of
 * chemical kinetics on AMD Instinct MI355X (gfx950).
 *
 * Method: Donovan, Sedgewick, Faeder, Zuckerman, "Efficient stochastic
 * simulation of chemical kinetics networks using a weighted ensemble of
 * trajectories" (arXiv:1303.5986).  The calls below follow the paper's
 * statement of the problem: a reaction network (Sec. II.A), a bin grid and
 * a target number of walkers per bin, the interval tau and the initial state
 * (the WE procedure of Sec. II.B), and a recycling target for steady-state
 * mean first-passage times (Sec. II.B.2, Eq. mfpt).
 *
 * Conventions for every entry point:
 *  - All pointer arguments are HOST pointers unless stated otherwise; every
 *    input array is copied before the call returns, so the caller may free
 *    it at once.  Output arrays are caller-allocated host memory.
 *  - Handles (we_network, we_sim) are opaque and owned by the library until
 *    passed to the matching destroy call.
 *  - Functions return a we_status; a negative value is an error, and
 *    we_last_error() then returns a thread-local message.  No C++ exception
 *    crosses this interface.
 *  - we_step_intervals is asynchronous on the sim's HIP stream.  Errors met
 *    on the device (a count leaving [0, WE_COUNT_MAX], a selection guard
 *    firing with no positive propensity) are latched in device memory and
 *    returned by the next synchronous call (we_synchronize and every getter).
 *  - Calls on one sim must not overlap (one host thread at a time).
 */
#ifndef WE_H
#define WE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WE_API __attribute__((visibility("default")))

/* Largest copy number of any species: keeps each reactant factor
 * prod_s C(x_s, nu_s) (reaction order <= 3) below 2^53, exact in FP64. */
#define WE_COUNT_MAX 131071

typedef struct we_network we_network;
typedef struct we_sim we_sim;

typedef enum {
    WE_OK = 0,
    WE_EINVAL = -1,     /* invalid argument or network                     */
    WE_ENOMEM = -2,     /* device or host allocation failed                */
    WE_EDEVICE = -3,    /* HIP runtime error                               */
    WE_ECAPACITY = -4,  /* more iterations or walkers than were reserved   */
    WE_EOVERFLOW = -5,  /* a copy number left [0, WE_COUNT_MAX]             */
    WE_ESTATE = -6      /* call not valid in the sim's current state       */
} we_status;

typedef enum {
    WE_KERNEL_AUTO = 0, /* lane-per-walker for small networks, else wave      */
    WE_KERNEL_LANE = 1, /* one lane per walker, full propensity recompute     */
    WE_KERNEL_WAVE = 2, /* one 64-wide wavefront per walker                   */
    WE_KERNEL_GROUP = 3 /* 64 / walkers_per_wave lanes per walker, full       */
                        /*   propensity recompute split over the group       */
} we_kernel;

/* ---------------------------------------------------------------- network
 * A mass-action reaction network (Sec. II.A), in CSR form:
 *   reactants of reaction j: reac_species[reac_ptr[j] .. reac_ptr[j+1]) with
 *     multiplicities reac_mult (1..3), each species at most once, total
 *     order <= 3;
 *   net change of reaction j: chg_species / chg_delta over chg_ptr
 *     (non-zero deltas, each species at most once; a negative delta -d needs
 *     the species among the reactants with multiplicity >= d);
 *   rate_c[j]: stochastic rate constant c_j >= 0, with constant reservoir
 *     species folded in.
 * Propensity: a_j(x) = c_j * prod_s C(x_s, nu_js)  (the combinatorial
 * mass-action convention under which the Schloegl model of Sec. III.B has
 * its wells at 82 and 563).
 * Errors: WE_EINVAL on any violation above; WE_ENOMEM / WE_EDEVICE. */
WE_API we_status we_create_network(int32_t n_species, int32_t n_reactions,
                                   const int32_t *reac_ptr, const int32_t *reac_species,
                                   const int32_t *reac_mult,
                                   const int32_t *chg_ptr, const int32_t *chg_species,
                                   const int32_t *chg_delta,
                                   const double *rate_c, we_network **out);
WE_API void we_destroy_network(we_network *net);

/* Hill-type rate (Sec. III.C): reaction `reaction`'s propensity becomes
 * c_j h_j(x) / (1 + (x_r / K)^n), r = `species`, evaluated in FP64 as
 * t = x_r / K, p = t * t * ... (n factors), a = (c_j h_j) / (1 + p).
 * 1 <= n <= 8, K > 0 finite.  Call before we_init; networks with Hill-type
 * rates run on the lane kernel only (at most 8 species and 16 reactions)
 * and not inside batches.  Errors: WE_EINVAL. */
WE_API we_status we_set_hill(we_network *net, int32_t reaction, int32_t species, int32_t n,
                             double K);

/* ---------------------------------------------------------------- bins
 * Static grid on a linear progress coordinate q(x) = sum_s coef[s] * x_s
 * (summed in species order in FP64).  Bin b is [edges[b], edges[b+1]);
 * q below edges[0] goes to bin 0 and q at or above edges[n_bins] to bin
 * n_bins-1 (the paper's grids are regular and the open-ended bin of
 * Sec. III.C is the precedent).  edges must be strictly increasing.
 * Optionally a second axis (the two-dimensional grid of Sec. III.C):
 * n_bins2 > 1 bins on q2(x) = sum_s coef2[s] x_s with edges2, binned the
 * same way; the bin is b1 + n_bins * b2, and there are n_bins * n_bins2
 * bins in all (at most 8192).  n_bins2 = 0 or 1: one axis (coef2 and
 * edges2 unused). */
typedef struct {
    int32_t n_bins;
    const double *coef;    /* [n_species] */
    const double *edges;   /* [n_bins + 1] */
    int32_t n_bins2;
    const double *coef2;   /* [n_species] */
    const double *edges2;  /* [n_bins2 + 1] */
} we_grid;

/* ---------------------------------------------------------------- run setup
 * One sim holds n_runs independent WE runs of the same network, bins and
 * tau, each with its own seed (independent replicas, as the paper uses for
 * error bars).  Each run reserves cap = m_targ * n_bins walker slots.
 * Initial ensemble: m_targ walkers at x0, weight 1/m_targ each (weights sum
 * to one, Sec. II.B), unless replaced by we_set_ensemble before the first
 * step. */
typedef struct {
    double tau;                /* WE interval, > 0                                  */
    int32_t m_targ;            /* walkers per occupied bin, >= 1                    */
    int32_t n_runs;            /* independent runs, >= 1                            */
    int32_t max_iters;         /* iterations reserved for flux / event series       */
    int32_t kernel;            /* we_kernel                                         */
    const uint64_t *seeds;     /* [n_runs] Philox keys                              */
    const int32_t *x0;         /* [n_species] initial state, 0 <= x0 <= COUNT_MAX   */
    int32_t recycle;           /* 1: steady state, walkers in B restart from A      */
    const double *tgt_coef;    /* [n_species] B = { x : sum tgt_coef_s x_s >= thr } */
    double tgt_thr;
    const int32_t *x_rec;      /* [n_species] recycling state A (NULL: x0)          */
    int32_t hist_species;      /* species whose P(x, t) is accumulated every        */
    int32_t hist_lo, hist_hi;  /*   iteration over [lo, hi] (hi < lo: none)         */
    int32_t n_joint;           /* 0..5 species in a joint histogram accumulated     */
    const int32_t *joint_species; /* every iteration over joint_bins^n_joint cells, */
    int32_t joint_bins;        /*   cell of species d = min(x / joint_width,        */
    int32_t joint_width;       /*   joint_bins - 1), first species fastest          */
    int32_t record_iters;      /* keep the resampled ensemble of this many          */
                               /*   iterations on the device (committor training)   */
    int32_t rw_period;         /* steady-state reweighting (Sec. II.B.2, Eq. ss)    */
                               /*   after every rw_period-th iteration; 0: none.    */
                               /*   Needs n_bins <= 512 and grid bins (no learned   */
                               /*   committor bins, no batches)                     */
    int32_t rw_reset;          /* 1: the flux matrix restarts after every event, so */
                               /*   each event uses only the intervals since the    */
                               /*   last one; 0: it accumulates from the start      */
    int32_t engine;            /* propagation: 0 exact direct-method SSA; 1 explicit */
                               /*   tau-leaping (Sec. IV proposes it; Gillespie     */
                               /*   2001 with the step bound of Cao, Gillespie and  */
                               /*   Petzold 2006, an exact event instead of a leap  */
                               /*   where the bound is below 10/a0, leaps halved    */
                               /*   when a count would go negative; leap uniforms   */
                               /*   from Philox(n, slot, iter, 4)).  Lane kernel,   */
                               /*   mass action, S <= 8, R <= 16, no batches        */
    double leap_eps;           /* tau-leaping error control epsilon, in (0, 1)      */
    int32_t resample_rule;     /* per-bin split/merge (Sec. II.B):                  */
                               /*   0: count-only, as the procedure is printed:     */
                               /*      n < m_targ: replicate, n > m_targ: merge the */
                               /*      two lowest weights until m_targ remain;      */
                               /*   1: weight-equalizing (the paper resamples       */
                               /*      "according to the weight" of each segment):  */
                               /*      with W the bin's weight summed in slot order */
                               /*      and w* = W / m_targ, merge the two lowest    */
                               /*      while their sum is <= w* or                  */
                               /*      sum_k max(1, ceil(w_k / (2 w*))) > m_targ,   */
                               /*      then replicate up to m_targ.  A bin of zero  */
                               /*      weight falls back to rule 0.                 */
    int32_t walkers_per_wave;  /* group kernel: walkers sharing one wave, one of    */
                               /*   2, 4, 8, 16, 32 (64 / that many lanes each,     */
                               /*   (64 / L) * S <= 4096); other kernels: ignored   */
} we_params;

/* Device bytes a sim needs (walker buffers, series, scratch). */
WE_API we_status we_workspace_size(const we_network *net, const we_grid *grid,
                                   const we_params *p, size_t *bytes);

/* Create a sim.  hip_stream: a hipStream_t (NULL = default stream) on which
 * every kernel of this sim is launched.  workspace: optional DEVICE pointer
 * of at least we_workspace_size() bytes, 256-byte aligned, owned by the
 * caller and kept alive until we_destroy (NULL: the library allocates).
 * Errors: WE_EINVAL (bad sizes, edges not increasing, x0 out of range,
 * tau <= 0, species out of range), WE_ENOMEM, WE_EDEVICE. */
WE_API we_status we_init(const we_network *net, const we_grid *grid, const we_params *p,
                         void *hip_stream, void *workspace, size_t workspace_bytes,
                         we_sim **out);

/* Name of the propagation kernel the sim's steps launch (the variant is
 * chosen from the network and the launch shape); "" for NULL.  The string is
 * static. */
WE_API const char *we_propagation_kernel(const we_sim *s);

/* Switch a sim's bins (Sec. II.B bins the state space; Sec. IV calls the
 * choice of bins open).  kind WE_BINS_GRID: grid NULL returns to the sim's
 * grid bins (after learned ones); a non-NULL grid replaces the coordinates
 * and edges, keeping the number of bins on each axis (the slot reservation
 * m_targ * n_bins depends on it).  kind WE_BINS_LEARNED: bin on the trained
 * committor (we_train_committor), grid must be NULL; qedges NULL keeps the
 * logit edges computed at training, otherwise n_bins + 1 host doubles
 * replace them (inner edges strictly increasing; a logit below the second
 * edge falls in bin 0, one at or above the last inner edge in the last bin).
 * Takes effect from the next iteration.  Synchronous.  Errors: WE_EINVAL
 * (bin counts differ, edges not increasing, qedges with grid bins),
 * WE_ESTATE (a captured graph exists: recapture after switching; learned
 * bins without a trained committor). */
typedef enum { WE_BINS_GRID = 0, WE_BINS_LEARNED = 1 } we_bins_kind;
typedef struct {
    int32_t kind;              /* we_bins_kind                                      */
    const we_grid *grid;       /* WE_BINS_GRID: new grid, or NULL                   */
    const double *qedges;      /* WE_BINS_LEARNED: [n_bins + 1] logit edges, or NULL */
} we_bins;
WE_API we_status we_set_bins(we_sim *s, const we_bins *bins);

/* ---------------------------------------------------------------- checkpoints
 * The WE procedure saves every trajectory's coordinates and weight after
 * each iteration (Sec. II.B).  A checkpoint holds the whole state of a sim at
 * an iteration boundary: every run's walkers (states, weights, bins, parent
 * slots), the iteration, the seeds, the flux, event and segment series, the
 * histogram accumulators, the reweighting flux matrix, the grid and
 * parameters the sim was built with, and a trained committor (model, Adam
 * moments, feature scaling, bin edges, whether bins are learned).  Random
 * numbers are keyed by (seed, slot, event, iteration), so no generator state
 * is needed: a sim loaded from a checkpoint continues exactly as the saved
 * one would have.  Not saved: committor training records and captured
 * graphs.  Format: a 64-byte header ("WESIMCKP", version, sizes, a
 * fingerprint of the network) followed by sections in a fixed order, host
 * byte order.
 *
 * we_save: synchronous; first reports a device fault latched by earlier
 * steps (as we_histogram does).  Errors: WE_EINVAL (NULL), WE_EDEVICE (file
 * cannot be written; device fault). */
WE_API we_status we_save(we_sim *s, const char *path);

/* Sizes recorded in a checkpoint (host-only: reads the header). */
typedef struct {
    int32_t version;
    int32_t n_species, n_reactions, n_runs, n_bins, m_targ, max_iters, iteration;
    int32_t hist_lo, hist_hi, n_joint, joint_bins, kernel;
    double tau;
    uint64_t workspace_bytes;  /* device bytes the loaded sim needs              */
} we_checkpoint_info;
WE_API we_status we_checkpoint_inspect(const char *path, we_checkpoint_info *info);

/* Build a sim from a checkpoint on network `net`, which must be the network
 * it was saved with (same species, reactions, rates, stoichiometry and Hill
 * factors; checked by fingerprint).  hip_stream, workspace and
 * workspace_bytes as for we_init (workspace_bytes >= the checkpoint's
 * workspace_bytes).  Synchronous.  Errors: WE_EINVAL (unreadable file, bad
 * magic or version, network mismatch, workspace too small), WE_ENOMEM,
 * WE_EDEVICE. */
WE_API we_status we_load(const we_network *net, const char *path, void *hip_stream, void *workspace,
                         size_t workspace_bytes, we_sim **out);

/* Replace run `run`'s ensemble before the first step: n walkers, states
 * x[n*S] (walker-major), weights w[n].  Errors: WE_ESTATE after stepping,
 * WE_ECAPACITY if n > cap, WE_EINVAL for counts out of range. */
WE_API we_status we_set_ensemble(we_sim *s, int32_t run, int32_t n, const int32_t *x,
                                 const double *w);

/* Advance every run by n WE iterations (Sec. II.B): propagate each walker
 * through tau with the Gillespie direct method, recycle walkers that reached
 * B (if enabled), bin, split/merge per bin, record observables.
 * Asynchronous.  Errors: WE_ECAPACITY past max_iters, WE_EDEVICE. */
WE_API we_status we_step_intervals(we_sim *s, int32_t n);

/* Record n iterations (n even, > 0) of the sim as one HIP graph, captured
 * on a private stream; nothing is executed by the capture.  Every kernel
 * reads the iteration number from device memory, so the graph can be
 * replayed; n even brings the double-buffered ensemble back to the buffer it
 * started from.  Replaces any earlier graph.  Errors: WE_EINVAL (n odd or
 * <= 0), WE_EDEVICE. */
WE_API we_status we_graph_capture(we_sim *s, int32_t n);

/* Launch the captured graph `times` times on the sim's stream (n*times
 * iterations, asynchronous).  Errors: WE_ESTATE (nothing captured),
 * WE_ECAPACITY past max_iters. */
WE_API we_status we_graph_replay(we_sim *s, int32_t times);

/* Wait for the sim's stream; return any latched device error. */
WE_API we_status we_synchronize(we_sim *s);

/* Copy run `run`'s current ensemble (canonical order: bins ascending,
 * parents by ascending slot, copies consecutive) to host arrays of at least
 * cap entries (x: cap*S).  Any output pointer may be NULL.  Synchronous. */
WE_API we_status we_get_walkers(we_sim *s, int32_t run, int32_t *n, int32_t *x, double *w,
                                int32_t *bin, int32_t *origin);

/* P(x_species = k, t) for k = lo..hi from run `run`'s current ensemble
 * (sum of walker weights, Sec. II.B.1); out has hi-lo+1 entries.
 * Synchronous. */
WE_API we_status we_histogram(we_sim *s, int32_t run, int32_t species, int32_t lo,
                              int32_t hi, double *out);

/* Sum over recorded iterations of P(x_hist_species = k, t) for
 * k = hist_lo..hist_hi, per run (out: n_runs*(hi-lo+1)), and the number of
 * iterations summed.  Synchronous. */
WE_API we_status we_histogram_accum(we_sim *s, double *out, int32_t *n_iters);

/* The joint histogram summed over recorded iterations, per run
 * (out: n_runs * joint_bins^n_joint doubles).  Synchronous. */
WE_API we_status we_joint_histogram(we_sim *s, double *out);

/* Weight recycled into B in iterations [first, first+count) of run `run`
 * (out: count entries).  Synchronous. */
WE_API we_status we_flux(we_sim *s, int32_t run, int32_t first, int32_t count, double *out);

/* Steady-state MFPT = 1 / flux (Eq. mfpt): per run, flux = mean recycled
 * weight per iteration after `discard` iterations divided by tau; the runs'
 * fluxes are independent samples (Sec. III.C).  flux_sem is their standard
 * error.  Synchronous. */
WE_API we_status we_mfpt(we_sim *s, int32_t discard, double *mfpt, double *flux_mean,
                         double *flux_sem);

/* Totals over all runs and iterations so far: reactions fired and
 * trajectory segments propagated (one segment = one walker over one tau).
 * Synchronous. */
WE_API we_status we_counters(we_sim *s, int64_t *events, int64_t *segments,
                             int32_t *iterations);

/* Per-iteration reactions fired, summed over runs, for iterations
 * [first, first+count).  Synchronous. */
WE_API we_status we_events_series(we_sim *s, int32_t first, int32_t count, int64_t *out);

/* Reactions fired by each walker of `run` during the last interval, in the
 * slot order that interval started with: out[cap] (host), *n = walkers
 * propagated (entries past it are stale).  Synchronous.  A diagnostic of
 * load balance: an interval lasts as long as its busiest walker. */
WE_API we_status we_walker_events(we_sim *s, int32_t run, int32_t *n, uint32_t *out);

/* ---------------------------------------------------------------- reweighting
 * Steady-state reweighting (Sec. II.B.2, Eq. ss), on when rw_period > 0.
 * Flux matrix: F[i][j] adds, every interval after the first and walker by
 * walker in slot order, the weight of each walker that started the interval
 * in bin j and ended it in bin i (after recycling).  W_j = sum_i F[i][j];
 * the rates are k_ij = F[i][j] / W_j.  After the resampling of iteration t
 * with (t + 1) % rw_period == 0, the bins that are occupied and have
 * W_j > 0 are candidates; the strongly connected component (edges j -> i
 * where F[i][j] > 0) of the candidate holding the most weight (ties: the
 * lowest bin) gets the solution pi of Eq. ss on it: its walkers are
 * rescaled so that bin a holds pi_a / sum(pi) of the component's weight.
 * The component keeps its total weight; other bins are unchanged; a
 * one-bin component changes nothing (the event counts as skipped).  With
 * rw_reset, F is cleared after every event (applied or skipped). */

/* Run `run`'s flux matrix so far: out[i * n_bins + j] = F[i][j] (n_bins^2
 * doubles).  WE_EINVAL without reweighting.  Synchronous. */
WE_API we_status we_rw_flux_matrix(we_sim *s, int32_t run, double *out);

/* Reweighting events of run `run` so far that rescaled weights (applied)
 * and that changed nothing (skipped).  Synchronous. */
WE_API we_status we_rw_counts(we_sim *s, int32_t run, int32_t *applied, int32_t *skipped);

/* ---------------------------------------------------------------- learned bins
 * A committor q(x) ~ P(reach B before A | x), learned from the sim's own
 * recorded trajectories, replaces the grid coordinate (the paper leaves the
 * choice of bins open, Sec. IV.B; WE stays unbiased for any binning).
 * Model: n_species -> 64 -> 64 -> 1 (tanh, tanh, sigmoid), FP32, inputs
 * (log1p(x_s) - mean_s)/std_s; binary cross-entropy on soft labels; Adam.
 * Parameters are one FP32 array: W1[64][S], b1[64], W2[64][64], b2[64],
 * W3[64], b3[1].  The learned bins partition the logit
 * z = log(q / (1 - q)) (which resolves q near 0): equal-count quantiles of
 * the training states, or equal widths (edge_mode below). */
typedef struct {
    int32_t steps;             /* Adam steps                                        */
    int32_t batch;             /* minibatch size, a positive multiple of 256        */
    float lr;                  /* learning rate (beta1 0.9, beta2 0.999, eps 1e-8)  */
    const double *a_coef;      /* [S] A = { x : sum a_coef_s x_s <= a_thr }          */
    double a_thr;
    uint64_t seed;             /* weight initialisation and minibatch draws         */
    int32_t edge_mode;         /* 0: n_bins equal-count quantiles of q over the     */
                               /*    training states; 1: n_bins equal widths in     */
                               /*    the logit between its 0.5% and 99.5% quantiles  */
} we_train_params;

/* Label the recorded walkers by their descendants' first outcome (B: the
 * walker's line was recycled; A: it re-entered A), train the model, and
 * compute the quantile edges.  loss_out (may be NULL) gets the mean
 * minibatch loss of every step; n_samples the training-set size.
 * Synchronous.  Errors: WE_ESTATE without records or resolved walkers. */
WE_API we_status we_train_committor(we_sim *s, const we_train_params *tp, float *loss_out,
                                    int32_t *n_samples);

/* Bin on the trained committor (enable = 1) or on the grid again (0). */
WE_API we_status we_use_committor_bins(we_sim *s, int32_t enable);

/* q(x) of n host states x[n*S] (out: q[n]).  Synchronous. */
WE_API we_status we_committor_eval(we_sim *s, int32_t n, const int32_t *x, float *q);

/* Copy the trained model: params[n_params], feat[2*S] (mean, 1/std),
 * qedges[n_bins+1] (logit edges); any pointer may be NULL.  Synchronous. */
WE_API we_status we_committor_state(we_sim *s, float *params, float *feat, double *qedges,
                                    int32_t *n_params);

/* Outcome counts of every recorded walker: counts[2*(i*n_runs*cap + slot)]
 * = (n_A, n_B).  Synchronous. */
WE_API we_status we_record_labels(we_sim *s, const double *a_coef, double a_thr,
                                  uint32_t *counts, int32_t *n_iters);

/* Recorded iteration i: walker counts per run n[n_runs], states
 * x[n_runs*cap*S], parent slots origin[n_runs*cap], recycled flags
 * recycled[n_runs*cap].  Synchronous. */
WE_API we_status we_get_record(we_sim *s, int32_t i, int32_t *n, int32_t *x, int32_t *origin,
                               uint8_t *recycled);

/* Stand-alone loss and gradient of the committor model on one host
 * minibatch (the training kernels; for checking against other
 * implementations): params[n_params(n_in)], feat[2*n_in], x[batch*n_in],
 * y[batch]; out: loss (mean BCE), grad[n_params].  Synchronous, default
 * stream. */
WE_API we_status we_mlp_loss_grad(int32_t n_in, const float *params, const float *feat,
                                  int32_t batch, const int32_t *x, const float *y, float *loss,
                                  float *grad);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training loops, harnesses that forbid hipMalloc): the loss
 * and gradient of we_mlp_loss_grad computed on caller-owned DEVICE buffers,
 * asynchronously on `hip_stream` (a stream of the current device; NULL: the
 * null stream), with no allocation of any kind.  params[n_params(n_in)],
 * feat[2*n_in], x[batch*n_in], y[batch] are read; loss (one float, the mean
 * BCE) and grad[n_params(n_in)] are written.  The per-sample activations and
 * deltas live in a fixed device array of WE_MLP_NOALLOC_FLOATS floats (5 MiB)
 * that each GPU holds until the process ends, so batch * (n_in + 258) must
 * not exceed WE_MLP_NOALLOC_FLOATS (batch 4096 at 64 inputs).  Every call on
 * a GPU shares that array; each call writes every entry it reads, so nothing
 * needs clearing, but calls that overlap in time on one GPU (different
 * streams, other threads) race and must be serialized by the caller.
 * Errors: WE_EINVAL (bad sizes or NULL pointers), WE_ECAPACITY (beyond the
 * scratch), WE_EDEVICE (symbol lookup or launch failure). */
#define WE_MLP_NOALLOC_FLOATS (4096 * (64 + 258))
#define WE_MAX_DEVICES 64
WE_API we_status we_mlp_loss_grad_noalloc(int32_t n_in, const float *params, const float *feat,
                                          int32_t batch, const int32_t *x, const float *y, float *loss,
                                          float *grad, void *hip_stream);

/* One Adam update (step t >= 1) of n host parameters in place.  Synchronous. */
WE_API we_status we_adam_step(int32_t n, float *params, float *m, float *v, const float *grad,
                              float lr, int32_t t);

/* ---------------------------------------------------------------- peaks
 * Microbenchmarks of the ceilings the kernels' rooflines are priced against,
 * measured on the current device (not part of the method): HBM bandwidth of
 * a 1 GiB device-to-device copy (read + write bytes), LDS read bandwidth
 * (conflict-free 16-byte reads), FP64 FMA rate (2 flops each) and 32-bit
 * integer lane-operation rate; each the median of five timed launches.
 * Allocates 2 GiB of device memory for the duration of the call.
 * Synchronous on hip_stream (NULL: the default stream). */
typedef struct {
    double hbm_gbs;            /* GB/s */
    double lds_tbs;            /* TB/s */
    double fp64_tflops;        /* TFLOP/s */
    double int32_tops;         /* 10^12 lane operations/s */
    int32_t compute_units;
} we_peaks;
WE_API we_status we_measure_peaks(void *hip_stream, we_peaks *out);

/* ---------------------------------------------------------------- batches
 * Many independent WE runs of DIFFERENT networks stepped together on one
 * stream (the paper runs independent replicas, Sec. IV).  Member i is an
 * ordinary sim built from nets[i], grids[i], params[i] (library-allocated
 * workspace; no reweighting, tau-leaping or Hill rates); the propagation of
 * all members is one persistent launch per kernel variant whose waves pull
 * (run, walker-tile) work items from a device counter, so uneven runs
 * balance across the chip.
 * autotune_iters > 0: for a member with params.kernel AUTO, every kernel
 * its network fits -- lane (64 walkers per wave), group (32, 16, 8, 4 or 2
 * walkers per wave), wave (1) -- is timed on one interval of a pilot sim of
 * the member's shape whose every slot holds a walker at x0 (best of
 * autotune_iters pilots) and the fastest is kept; choices are cached in the
 * JSON file cache_path (NULL: no cache).  autotune_iters = 0: lane for networks of up to 32 reactions that
 * fit it, else wave.
 * Members are owned by the batch: read them with the sim getters via
 * we_batch_sim, never step or destroy them directly.  The committor calls
 * apply to members too: a member with params.record_iters > 0 records its
 * ensembles during eager we_batch_step calls, we_train_committor trains its
 * model, and after we_use_committor_bins(member, 1) the batch bins that
 * member on its learned committor from the next iteration on (one batched
 * launch for all such members). */
typedef struct we_batch we_batch;
WE_API we_status we_batch_create(int32_t n, const we_network *const *nets, const we_grid *grids,
                                 const we_params *params, void *hip_stream,
                                 int32_t autotune_iters, const char *cache_path, we_batch **out);
/* n iterations of every member (asynchronous).  Errors: WE_ECAPACITY past
 * the smallest member max_iters. */
WE_API we_status we_batch_step(we_batch *b, int32_t n);
/* Capture n (even) batched iterations as one HIP graph / replay it.
 * Errors: WE_ESTATE while a member is still recording (capture), or when a
 * member's bins were switched or its model retrained into new buffers
 * since the capture (replay: capture again). */
WE_API we_status we_batch_graph_capture(we_batch *b, int32_t n);
WE_API we_status we_batch_graph_replay(we_batch *b, int32_t times);
/* Member i (NULL if out of range); kernels[i] gets each member's kernel and
 * walkers_per_wave[i] its walkers per wave (lane 64, group 2..32, wave 1);
 * either array may be NULL. */
WE_API we_sim *we_batch_sim(we_batch *b, int32_t i);
WE_API we_status we_batch_info(we_batch *b, int32_t *n_sims, int32_t *kernels, int32_t *walkers_per_wave);
WE_API void we_batch_destroy(we_batch *b);

/* Per-kernel timing with HIP events recorded on the sim's stream around
 * every launch.  we_profile(s, 1) clears and starts the accumulators,
 * we_profile(s, 0) stops recording.  we_profile_read waits for the stream
 * and returns the summed device time in milliseconds of the propagation
 * (SSA) kernels, the recycle/bin/resample kernels and the observable
 * kernels, and the number of iterations they cover.  Synchronous. */
WE_API we_status we_profile(we_sim *s, int32_t enable);
WE_API we_status we_profile_read(we_sim *s, double *ms_propagate, double *ms_resample,
                                 double *ms_observe, int64_t *iterations);

WE_API void we_destroy(we_sim *s);
WE_API const char *we_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WE_H */
