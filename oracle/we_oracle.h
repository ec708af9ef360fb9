/*
 * we_oracle.h -- plain, slow, sequential CPU oracle for weighted-ensemble (WE)
 * stochastic simulation of chemical kinetics (Donovan, Sedgewick, Faeder,
 * Zuckerman, arXiv:1303.5986).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product (the HIP
 * library under paper_1303_5986_amd/) never includes, links or calls it, and
 * the two share no source.
 *
 * What is computed, and where the paper defines it:
 *   - Gillespie direct-method SSA over one WE interval tau            (Sec. II.A)
 *   - mass-action propensities with combinatorial reactant factors
 *     (the reading that reproduces the Schloegl wells of Sec. III.B)  (Eqs. futile, schlogl)
 *   - steady-state recycling B -> A with flux accounting              (Sec. II.B.2, Eq. mfpt)
 *   - per-bin split / merge resampling conserving weight              (Sec. II.B, WE procedure)
 *   - Philox4x32-10 counter-based random numbers (Salmon et al., SC'11);
 *     the paper is silent on the generator.
 *
 * Every function is a direct statement of the definition; nothing is
 * blocked, fused or reordered.
 */
#ifndef WE_ORACLE_H
#define WE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Largest copy number a species may hold: keeps every combinatorial factor
 * h_j(x) (reaction order <= 3) below 2^53, so it is exact in FP64. */
#define OR_COUNT_MAX 131071
/* tau-leaping: exact events taken in a row once the step bound is below 10 / a0 */
#define OR_LEAP_SSA_RUN 100

enum { OR_OK = 0, OR_EINVAL = -1, OR_EOVERFLOW = -5 };

/* A reaction network in CSR form.
 *   reactants of reaction j: reac_species[reac_ptr[j] .. reac_ptr[j+1]) with
 *   multiplicities reac_mult (1..3, distinct species per reaction);
 *   net change of reaction j: chg_species/chg_delta over chg_ptr;
 *   rate[j]: stochastic rate constant c_j (constant reservoir species folded in);
 *   hill_species (may be NULL): reaction j's propensity is divided by the
 *   repressive Hill factor 1 + (x_r / hill_K[j])^hill_n[j], r = hill_species[j]
 *   (-1: none), the Hill-type rates of the switch of Sec. III.C. */
typedef struct {
    int32_t S, R;
    const int32_t *reac_ptr, *reac_species, *reac_mult;
    const int32_t *chg_ptr, *chg_species, *chg_delta;
    const double *rate;
    const int32_t *hill_species, *hill_n;
    const double *hill_K;
} or_net;

/* WE configuration (the arguments of the WE procedure in Sec. II.B plus the
 * steady-state recycling target of Sec. II.B.2). */
typedef struct {
    int32_t n_bins;
    const double *bin_coef;   /* [S]  progress coordinate q(x) = sum_s coef_s x_s  */
    const double *edges;      /* [n_bins+1] strictly increasing; out-of-range clamps */
    int32_t n_bins2;          /* second grid axis (0 or 1: none); bin = b1 + n_bins*b2 */
    const double *bin_coef2;  /* [S]                                               */
    const double *edges2;     /* [n_bins2+1]                                       */
    int32_t m_targ;           /* target walkers per occupied bin                  */
    double tau;               /* WE interval                                       */
    uint64_t seed;            /* Philox key                                        */
    int32_t recycle;          /* 1: walkers in B are returned to A (steady state)  */
    const double *tgt_coef;   /* [S]  B = { x : sum_s tgt_coef_s x_s >= tgt_thr }   */
    double tgt_thr;
    const int32_t *x_rec;     /* [S]  recycling state A                            */
    int32_t engine;           /* 0: exact SSA; 1: tau-leaping (or_tauleap_interval) */
    double leap_eps;          /* tau-leaping error control epsilon                  */
    int32_t resample_rule;    /* 0: count-only split/merge as printed (Sec. II.B);
                                 1: weight-equalizing (or_resample_bin)             */
} or_we_cfg;

/* Philox4x32-10: ten rounds of the Philox S-box with key schedule, per
 * Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11.  ctr = (c0,c1,c2,c3), key = (k0,k1). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* 53-bit uniform on [0,1) from two 32-bit words: ((hi>>5)*2^26 + (lo>>6)) * 2^-53. */
double or_u53(uint32_t hi, uint32_t lo);

/* Reactant combinatorial factor h_j(x) = prod_s C(x_s, nu_js), exact int64. */
int64_t or_h(const or_net *net, const int32_t *x, int32_t j);

/* Propensity a_j(x) = c_j * h_j(x)  (one FP64 rounding). */
double or_propensity(const or_net *net, const int32_t *x, int32_t j);

/* Validate a network: ids in range, 1 <= nu <= 3, order <= 3, no repeated
 * reactant species, and no change that could drive a count negative. */
int32_t or_validate(const or_net *net);

/* One WE interval of the Gillespie direct method for one walker, from local
 * time 0 to tau.  Random words for event e come from
 * Philox(ctr = (e, slot, iter, 0), key = seed).  x is updated in place.
 * Returns the number of reactions fired, or a negative status. */
int64_t or_ssa_interval(const or_net *net, int32_t *x, double tau,
                        uint64_t seed, uint32_t slot, uint32_t iter);

/* Explicit tau-leaping over one interval (Sec. IV proposes combining WE with
 * tau-leaping; the method is Gillespie's, J. Chem. Phys. 115, 1716 (2001),
 * with the step-size bound of Cao, Gillespie and Petzold, J. Chem. Phys.
 * 124, 044109 (2006)).  From t = 0, repeatedly:
 *   1. propensities a_j and a0 as in or_ssa_interval; stop if a0 = 0;
 *   2. tau' = min over reactant species i of
 *        min(b_i / |mu_i|, b_i^2 / sigma_i^2),  b_i = max(eps x_i / g_i, 1),
 *      mu_i = sum_j nu_ij a_j, sigma_i^2 = sum_j nu_ij^2 a_j (j ascending),
 *      g_i from the highest order of the reactions that consume i (CGP 2006,
 *      Eq. 27); zero denominators count as +infinity;
 *   3. if tau' < 10 / a0: OR_LEAP_SSA_RUN (100) steps of exact direct-method
 *      events, this one included, without evaluating tau' (the run of about
 *      100 SSA steps that Cao, Gillespie and Petzold recommend), with the SSA
 *      stream (counter (e, slot, iter, 0)) and the same stopping rule at tau;
 *      the run ends early with the interval;
 *   4. else leap dt = min(tau', tau - t): K_j ~ Poisson(a_j dt) for j
 *      ascending; if some count would go negative, halve tau' and draw again;
 *      otherwise x += sum_j K_j nu_j and t += dt (the leap that reaches tau
 *      ends the interval).
 * Poisson draws: inversion below a mean of 20, Hoermann's PTRS transformed
 * rejection (1993) above; uniforms (r + 0.5) 2^-32 from the words of
 * Philox(ctr = (n, slot, iter, 4), key = seed), n = 0, 1, ..., four per block.
 * Returns the number of reactions fired, or a negative status. */
int64_t or_tauleap_interval(const or_net *net, int32_t *x, double tau, double eps,
                            uint64_t seed, uint32_t slot, uint32_t iter);

/* Brute-force SSA first passage: from x (in place) run the direct method
 * for at most time T; stop at the first event after which
 * sum_s coef_s x_s >= thr.  Random words: Philox(ctr=(e_lo, e_hi, traj, 3), key=seed).
 * Returns the passage time, or -1.0 if no passage within T.  *events gets
 * the number of reactions fired. */
double or_ssa_first_passage(const or_net *net, int32_t *x, double T,
                            const double *coef, double thr,
                            uint64_t seed, uint32_t traj, int64_t *events);

/* Progress coordinate and bin of a state. */
double or_coord(int32_t S, const double *coef, const int32_t *x);
int32_t or_bin_of(int32_t n_bins, const double *edges, double q);

/* One complete WE iteration (propagate, recycle, bin, resample) on an
 * ensemble of *n walkers stored in slot order:
 *   x[k*S + s], w[k]; bin[k] and origin[k] are outputs.
 * The ensemble is replaced by the resampled one (canonical layout: bins
 * ascending; inside a bin, parents by ascending slot; copies of a parent
 * consecutive).  Arrays must hold cap = m_targ*n_bins walkers (and at least
 * the incoming *n).  flux_out gets the weight recycled this iteration;
 * events_out the reactions fired; recycled_out (may be NULL, size cap)
 * gets 1 for every incoming slot whose walker reached B and was recycled;
 * end_bin_out (may be NULL, size cap) gets the bin of every incoming slot at
 * the end of the interval, after recycling (the end bins of the inter-bin
 * fluxes used by steady-state reweighting).
 * Returns a status. */
int32_t or_we_iterate(const or_net *net, const or_we_cfg *cfg, uint32_t iter,
                      int32_t *n, int32_t *x, double *w, int32_t *bin,
                      int32_t *origin, int32_t cap,
                      double *flux_out, int64_t *events_out, int32_t *recycled_out,
                      int32_t *end_bin_out);

/* The resampling step alone, for one bin: nb walkers (parent slots, weights)
 * in ascending slot order.  Writes the surviving/replicated walkers as
 * (parent slot, weight) into out_slot/out_w in canonical order and returns
 * their number (m_targ if nb > 0, else 0).
 *   rule 0 (Sec. II.B as printed): n < M_targ: split; n > M_targ: merge the
 *     two lowest-weight walkers until M_targ remain; n = M_targ: unchanged.
 *   rule 1 (weight-equalizing): with W = sum of the bin's weights (slot
 *     order) and w* = W / M_targ, merge the two lowest-weight walkers while
 *     their sum is <= w* or sum_k max(1, ceil(w_k / (2 w*))) > M_targ; then
 *     split the survivors up to M_targ.  A bin of zero weight uses rule 0.
 * Merge draw m of (bin, iter) is Philox(ctr = (m, bin, iter, 1), key = seed). */
int32_t or_resample_bin(int32_t nb, const int32_t *slot, const double *w,
                        int32_t m_targ, int32_t rule, uint64_t seed, uint32_t bin, uint32_t iter,
                        int32_t *out_slot, double *out_w);

#ifdef __cplusplus
}
#endif
#endif
