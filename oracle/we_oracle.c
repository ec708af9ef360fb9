/*
 * we_oracle.c -- plain sequential CPU oracle for weighted-ensemble SSA.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline leg of the
 * benchmark).  Shares no code with the HIP library.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC
 * (no contraction of a*b+c into fused multiply-adds, so every FP64 operation
 * below is one IEEE-754 round-to-nearest operation in program order).
 *
 * Readings of the paper taken here (each one listed in the design notes):
 *  - propensity: a_j = c_j * prod_s C(x_s, nu_js)  -- the combinatorial
 *    mass-action convention; it is the one under which the Schloegl model of
 *    Sec. III.B has its wells at 82 and 563 and its barrier at 256.
 *  - Hill-type rates (Sec. III.C): a reaction with a repressor r divides
 *    that by 1 + (x_r / K)^n, evaluated as t = x_r / K, p = t * t * ... * t
 *    (n factors, left to right), d = 1 + p, a_j = (c_j * h_j) / d.
 *  - two-dimensional grids (Sec. III.C): bin = b1 + n_bins * b2, each axis
 *    binned like a one-dimensional grid.
 *  - interval boundary: a reaction fires iff t + dt <= tau; the state is then
 *    held to tau (memorylessness of the exponential waiting time).
 *  - split (Sec. II.B): a bin with 0 < n < M_targ walkers is filled by
 *    repeatedly giving one more copy to the parent with the largest
 *    per-copy weight w_k / c_k (ties: lowest slot); copies carry w_k / c_k.
 *    With n = 1 this is exactly the paper's w / M_targ rule.
 *  - merge (Sec. II.B): while n > M_targ, take the two lowest-weight walkers
 *    (ties: lowest slot); keep the first with probability w_i / (w_i + w_j),
 *    else the second; the survivor carries w_i + w_j.
 *  - weight-equalizing resampling (rule 1; the paper resamples "according to
 *    the weight" of each segment and ran implementations that keep the
 *    weights in a bin near W/M_targ): with W the bin's weight (summed in slot
 *    order) and w* = W / M_targ, the two lowest-weight walkers are merged as
 *    above while their sum is at most w*, or while the bin has no room to
 *    split its heavy walkers: sum_k max(1, ceil(w_k / (2 w*))) > M_targ (this
 *    also covers n > M_targ); the survivors are then split as above up to
 *    M_targ.  Rule 0 is the count-only procedure as printed.
 *  - recycling (Sec. II.B.2): checked once at the end of each interval,
 *    before binning; a walker in B adds its weight to the flux and restarts
 *    from A with its weight.
 */
#include "we_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11).                               */
/* ------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {            /* key schedule: Weyl sequence */
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double or_u53(uint32_t hi, uint32_t lo)
{
    uint64_t m = ((uint64_t)(hi >> 5) << 26) | (uint64_t)(lo >> 6);
    return (double)m * (1.0 / 9007199254740992.0);   /* 2^-53, exact */
}

static void seed_key(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
}

/* ------------------------------------------------------------------ */
/* Propensities.                                                      */
/* ------------------------------------------------------------------ */
static int64_t choose(int64_t x, int32_t nu)
{
    /* C(x, nu) for nu in {1, 2, 3}; zero when x < nu. */
    if (x < nu) return 0;
    if (nu == 1) return x;
    if (nu == 2) return x * (x - 1) / 2;
    return x * (x - 1) * (x - 2) / 6;
}

int64_t or_h(const or_net *net, const int32_t *x, int32_t j)
{
    int64_t h = 1;
    for (int32_t p = net->reac_ptr[j]; p < net->reac_ptr[j + 1]; ++p)
        h *= choose((int64_t)x[net->reac_species[p]], net->reac_mult[p]);
    return h;
}

double or_propensity(const or_net *net, const int32_t *x, int32_t j)
{
    double a = net->rate[j] * (double)or_h(net, x, j);
    if (net->hill_species && net->hill_species[j] >= 0) {
        const double t = (double)x[net->hill_species[j]] / net->hill_K[j];
        double p = t;
        for (int32_t i = 1; i < net->hill_n[j]; ++i) p = p * t;
        a = a / (1.0 + p);
    }
    return a;
}

int32_t or_validate(const or_net *net)
{
    if (net->S <= 0 || net->R <= 0) return OR_EINVAL;
    for (int32_t j = 0; j < net->R; ++j) {
        int32_t order = 0;
        if (!(net->rate[j] >= 0.0) || isinf(net->rate[j])) return OR_EINVAL;
        for (int32_t p = net->reac_ptr[j]; p < net->reac_ptr[j + 1]; ++p) {
            int32_t s = net->reac_species[p], nu = net->reac_mult[p];
            if (s < 0 || s >= net->S || nu < 1 || nu > 3) return OR_EINVAL;
            for (int32_t q = net->reac_ptr[j]; q < p; ++q)
                if (net->reac_species[q] == s) return OR_EINVAL;
            order += nu;
        }
        if (order > 3) return OR_EINVAL;
        if (net->hill_species && net->hill_species[j] >= 0) {
            if (net->hill_species[j] >= net->S || net->hill_n[j] < 1 || net->hill_n[j] > 8 ||
                !(net->hill_K[j] > 0.0) || isinf(net->hill_K[j]))
                return OR_EINVAL;
        }
        for (int32_t p = net->chg_ptr[j]; p < net->chg_ptr[j + 1]; ++p) {
            int32_t s = net->chg_species[p], d = net->chg_delta[p];
            if (s < 0 || s >= net->S || d == 0) return OR_EINVAL;
            for (int32_t q = net->chg_ptr[j]; q < p; ++q)
                if (net->chg_species[q] == s) return OR_EINVAL;
            if (d < 0) {
                /* consuming -d copies of s needs at least -d of them as reactants */
                int32_t nu = 0;
                for (int32_t q = net->reac_ptr[j]; q < net->reac_ptr[j + 1]; ++q)
                    if (net->reac_species[q] == s) nu = net->reac_mult[q];
                if (nu < -d) return OR_EINVAL;
            }
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Gillespie direct method over one interval.                         */
/* ------------------------------------------------------------------ */
/* Fire reaction j on x.  Returns OR_EOVERFLOW if a count leaves [0, COUNT_MAX]. */
static int32_t fire(const or_net *net, int32_t *x, int32_t j)
{
    int32_t st = OR_OK;
    for (int32_t p = net->chg_ptr[j]; p < net->chg_ptr[j + 1]; ++p) {
        int32_t s = net->chg_species[p];
        x[s] += net->chg_delta[p];
        if (x[s] < 0 || x[s] > OR_COUNT_MAX) st = OR_EOVERFLOW;
    }
    return st;
}

/* Reaction chosen by u2: the first j whose running sum of propensities
 * (summed sequentially from j = 0) exceeds u2 * a0.  If rounding leaves no
 * such j, the last reaction with positive propensity. */
static int32_t select_reaction(const double *a, int32_t R, double target)
{
    double cum = 0.0;
    int32_t last_pos = -1;
    for (int32_t j = 0; j < R; ++j) {
        cum = cum + a[j];
        if (a[j] > 0.0) last_pos = j;
        if (cum > target) return j;
    }
    return last_pos;
}

int64_t or_ssa_interval(const or_net *net, int32_t *x, double tau,
                        uint64_t seed, uint32_t slot, uint32_t iter)
{
    const int32_t R = net->R;
    double *a = (double *)malloc(sizeof(double) * (size_t)R);
    uint32_t key[2];
    seed_key(seed, key);
    double t = 0.0;
    int64_t fired = 0;
    uint32_t e = 0;
    for (;;) {
        /* 1. all propensities, and their total summed in reaction order */
        double a0 = 0.0;
        for (int32_t j = 0; j < R; ++j) {
            a[j] = or_propensity(net, x, j);
            a0 = a0 + a[j];
        }
        if (!(a0 > 0.0)) break;                     /* absorbing: idle to tau */
        /* 2. waiting time from the first uniform */
        uint32_t ctr[4] = {e, slot, iter, 0u}, r[4];
        or_philox4x32_10(ctr, key, r);
        e += 1;
        double u1 = or_u53(r[0], r[1]);
        double u2 = or_u53(r[2], r[3]);
        double dt = -log(1.0 - u1) / a0;
        if (t + dt > tau) break;                    /* next event lies past tau */
        t = t + dt;
        /* 3. which reaction, from the second uniform */
        int32_t j = select_reaction(a, R, u2 * a0);
        /* 4. apply its stoichiometry */
        fired += 1;
        if (fire(net, x, j) != OR_OK) { free(a); return OR_EOVERFLOW; }
    }
    free(a);
    return fired;
}

/* ---- tau-leaping */
typedef struct {
    uint32_t key[2], slot, iter, n, buf[4];
    int32_t idx;
} leap_rng;

static double leap_u(leap_rng *g)
{
    if (g->idx == 4) {
        uint32_t ctr[4] = {g->n, g->slot, g->iter, 4u};
        or_philox4x32_10(ctr, g->key, g->buf);
        g->n += 1;
        g->idx = 0;
    }
    return ((double)g->buf[g->idx++] + 0.5) * (1.0 / 4294967296.0);
}

/* Poisson(lam): inversion (sequential search) below 20; above, the PTRS
 * transformed rejection of W. Hoermann, "The transformed rejection method
 * for generating Poisson random variables", Insurance: Mathematics and
 * Economics 12 (1993). */
static int64_t leap_poisson(leap_rng *g, double lam)
{
    if (!(lam > 0.0)) return 0;
    if (lam < 20.0) {
        const double u = leap_u(g);
        double p = exp(-lam), F = p;
        int64_t k = 0;
        while (u > F && k < 1000) {
            k += 1;
            p = p * lam / (double)k;
            F = F + p;
        }
        return k;
    }
    const double slam = sqrt(lam), loglam = log(lam);
    const double b = 0.931 + 2.53 * slam, a = -0.059 + 0.02483 * b;
    const double invalpha = 1.1239 + 1.1328 / (b - 3.4), vr = 0.9277 - 3.6224 / (b - 2.0);
    for (;;) {
        const double U = leap_u(g) - 0.5, V = leap_u(g);
        const double us = 0.5 - fabs(U);
        const int64_t k = (int64_t)floor((2.0 * a / us + b) * U + lam + 0.43);
        if (us >= 0.07 && V <= vr) return k;
        if (k < 0 || (us < 0.013 && V > us)) continue;
        if (log(V) + log(invalpha) - log(a / (us * us) + b) <= -lam + (double)k * loglam - lgamma((double)k + 1.0))
            return k;
    }
}

/* g_i of CGP 2006 (Eq. 27) for a species consumed with highest order hor
 * and, in those reactions, multiplicity nu, at count x. */
static double leap_g(int32_t hor, int32_t nu, double x)
{
    if (hor <= 1) return 1.0;
    if (hor == 2) return nu == 1 ? 2.0 : 2.0 + 1.0 / (x - 1.0);
    if (nu == 1) return 3.0;
    if (nu == 2) return 1.5 * (2.0 + 1.0 / (x - 1.0));
    return 3.0 + 1.0 / (x - 1.0) + 2.0 / (x - 2.0);
}

int64_t or_tauleap_interval(const or_net *net, int32_t *x, double tau, double eps,
                            uint64_t seed, uint32_t slot, uint32_t iter)
{
    const int32_t R = net->R, S = net->S;
    double *a = (double *)malloc(sizeof(double) * (size_t)R);
    int64_t *K = (int64_t *)malloc(sizeof(int64_t) * (size_t)R);
    int64_t *xn = (int64_t *)malloc(sizeof(int64_t) * (size_t)S);
    int32_t *hor = (int32_t *)calloc((size_t)S, sizeof(int32_t));
    int32_t *hnu = (int32_t *)calloc((size_t)S, sizeof(int32_t));
    /* highest order of the reactions consuming each species, and its
     * multiplicity there (the largest, if several) */
    for (int32_t j = 0; j < R; ++j) {
        int32_t order = 0;
        for (int32_t p = net->reac_ptr[j]; p < net->reac_ptr[j + 1]; ++p) order += net->reac_mult[p];
        for (int32_t p = net->reac_ptr[j]; p < net->reac_ptr[j + 1]; ++p) {
            const int32_t sp = net->reac_species[p], nu = net->reac_mult[p];
            if (order > hor[sp] || (order == hor[sp] && nu > hnu[sp])) {
                hor[sp] = order;
                hnu[sp] = nu;
            }
        }
    }
    uint32_t key[2];
    seed_key(seed, key);
    leap_rng g;
    g.key[0] = key[0];
    g.key[1] = key[1];
    g.slot = slot;
    g.iter = iter;
    g.n = 0;
    g.idx = 4;
    double t = 0.0;
    int64_t fired = 0;
    uint32_t e = 0;
    int32_t status = OR_OK;
    int32_t ssa_left = 0;   /* exact events still to take before the bound is evaluated again */
    for (;;) {
        double a0 = 0.0;
        for (int32_t j = 0; j < R; ++j) {
            a[j] = or_propensity(net, x, j);
            a0 = a0 + a[j];
        }
        if (!(a0 > 0.0)) break;
        double tp = INFINITY;
        int exact = 0;
        if (ssa_left > 0) {
            ssa_left -= 1;
            exact = 1;
        } else {
            for (int32_t i = 0; i < S; ++i) {
                if (hor[i] == 0) continue;
                double mu = 0.0, sig = 0.0;
                for (int32_t j = 0; j < R; ++j) {
                    int32_t d = 0;
                    for (int32_t p = net->chg_ptr[j]; p < net->chg_ptr[j + 1]; ++p)
                        if (net->chg_species[p] == i) d = net->chg_delta[p];
                    mu = mu + (double)d * a[j];
                    sig = sig + (double)d * (double)d * a[j];
                }
                const double bi = fmax(eps * (double)x[i] / leap_g(hor[i], hnu[i], (double)x[i]), 1.0);
                if (mu != 0.0) tp = fmin(tp, bi / fabs(mu));
                if (sig != 0.0) tp = fmin(tp, bi * bi / sig);
            }
        }
        if (!exact && tp < 10.0 / a0) {
            /* leaping does not pay here: this and the next OR_LEAP_SSA_RUN - 1
             * steps are exact events (Cao, Gillespie and Petzold recommend a
             * run of about 100 before the bound is tried again) */
            exact = 1;
            ssa_left = OR_LEAP_SSA_RUN - 1;
        }
        if (exact) {
            /* one exact event */
            uint32_t ctr[4] = {e, slot, iter, 0u}, r[4];
            or_philox4x32_10(ctr, key, r);
            e += 1;
            const double u1 = or_u53(r[0], r[1]), u2 = or_u53(r[2], r[3]);
            const double dt = -log(1.0 - u1) / a0;
            if (t + dt > tau) break;
            t = t + dt;
            fired += 1;
            if (fire(net, x, select_reaction(a, R, u2 * a0)) != OR_OK) { status = OR_EOVERFLOW; break; }
            continue;
        }
        for (;;) {
            const double rest = tau - t;
            const int last = !(tp < rest);
            const double dt = last ? rest : tp;
            for (int32_t i = 0; i < S; ++i) xn[i] = x[i];
            for (int32_t j = 0; j < R; ++j) {
                K[j] = leap_poisson(&g, a[j] * dt);
                for (int32_t p = net->chg_ptr[j]; p < net->chg_ptr[j + 1]; ++p)
                    xn[net->chg_species[p]] += K[j] * (int64_t)net->chg_delta[p];
            }
            int neg = 0, big = 0;
            for (int32_t i = 0; i < S; ++i) {
                neg |= xn[i] < 0;
                big |= xn[i] > OR_COUNT_MAX;
            }
            if (neg) {
                tp = tp * 0.5;
                continue;
            }
            if (big) { status = OR_EOVERFLOW; break; }
            for (int32_t i = 0; i < S; ++i) x[i] = (int32_t)xn[i];
            for (int32_t j = 0; j < R; ++j) fired += K[j];
            t = last ? tau : t + dt;
            break;
        }
        if (status != OR_OK || !(t < tau)) break;
    }
    free(a); free(K); free(xn); free(hor); free(hnu);
    return status != OR_OK ? status : fired;
}

double or_ssa_first_passage(const or_net *net, int32_t *x, double T,
                            const double *coef, double thr,
                            uint64_t seed, uint32_t traj, int64_t *events)
{
    const int32_t R = net->R;
    double *a = (double *)malloc(sizeof(double) * (size_t)R);
    uint32_t key[2];
    seed_key(seed, key);
    double t = 0.0, hit = -1.0;
    uint64_t e = 0;
    int64_t fired = 0;
    for (;;) {
        double a0 = 0.0;
        for (int32_t j = 0; j < R; ++j) {
            a[j] = or_propensity(net, x, j);
            a0 = a0 + a[j];
        }
        if (!(a0 > 0.0)) break;
        uint32_t ctr[4] = {(uint32_t)e, (uint32_t)(e >> 32), traj, 3u}, r[4];
        or_philox4x32_10(ctr, key, r);
        e += 1;
        double u1 = or_u53(r[0], r[1]);
        double u2 = or_u53(r[2], r[3]);
        double dt = -log(1.0 - u1) / a0;
        if (t + dt > T) break;
        t = t + dt;
        int32_t j = select_reaction(a, R, u2 * a0);
        fired += 1;
        if (fire(net, x, j) != OR_OK) { hit = -2.0; break; }
        if (or_coord(net->S, coef, x) >= thr) { hit = t; break; }
    }
    free(a);
    if (events) *events = fired;
    return hit;
}

/* ------------------------------------------------------------------ */
/* Bins and the recycling target.                                     */
/* ------------------------------------------------------------------ */
double or_coord(int32_t S, const double *coef, const int32_t *x)
{
    double q = 0.0;
    for (int32_t s = 0; s < S; ++s) q = q + coef[s] * (double)x[s];
    return q;
}

int32_t or_bin_of(int32_t n_bins, const double *edges, double q)
{
    /* half-open bins [edges[b], edges[b+1]); values outside the grid go to
     * the first or last bin */
    int32_t b = 0;
    for (int32_t i = 1; i < n_bins; ++i)
        if (q >= edges[i]) b = i;
    return b;
}

/* ------------------------------------------------------------------ */
/* Resampling of one bin (split / merge).                             */
/* ------------------------------------------------------------------ */
/* The paper's split for a bin whose survivors number n_alive < m_targ:
 * every survivor starts with one copy; the remaining copies go one at a time
 * to the survivor with the largest per-copy weight (ties: lowest slot);
 * copies carry w_k / c_k.  Writes the copies in slot order. */
static int32_t split_survivors(int32_t nb, const int32_t *slot, const double *cw, const int32_t *alive,
                               int32_t n_alive, int32_t m_targ, int32_t *out_slot, double *out_w)
{
    int32_t *c = (int32_t *)malloc(sizeof(int32_t) * (size_t)nb);
    for (int32_t k = 0; k < nb; ++k) c[k] = alive[k] ? 1 : 0;
    for (int32_t extra = n_alive; extra < m_targ; ++extra) {
        int32_t best = -1;
        double best_share = 0.0;
        for (int32_t k = 0; k < nb; ++k) {
            if (!alive[k]) continue;
            double share = cw[k] / (double)c[k];
            if (best < 0 || share > best_share) { best = k; best_share = share; }
        }
        c[best] += 1;
    }
    int32_t o = 0;
    for (int32_t k = 0; k < nb; ++k) {
        if (!alive[k]) continue;
        double share = cw[k] / (double)c[k];
        for (int32_t copy = 0; copy < c[k]; ++copy) {
            out_slot[o] = slot[k];
            out_w[o] = share;
            ++o;
        }
    }
    free(c);
    return o;
}

/* Copies a walker of weight v needs so that none carries more than twice the
 * bin's ideal weight (at least one: every walker holds a place). */
static int32_t need_copies(double v, double two_ideal)
{
    double q = ceil(v / two_ideal);
    return q < 1.0 ? 1 : (int32_t)q;
}

int32_t or_resample_bin(int32_t nb, const int32_t *slot, const double *w,
                        int32_t m_targ, int32_t rule, uint64_t seed, uint32_t bin, uint32_t iter,
                        int32_t *out_slot, double *out_w)
{
    if (nb <= 0) return 0;
    /* the bin's weight and ideal per-walker weight (weight-equalizing rule) */
    double W = 0.0;
    for (int32_t k = 0; k < nb; ++k) W = W + w[k];
    const int equalize = (rule == 1) && (W > 0.0);
    const double ideal = W / (double)m_targ;
    const double two_ideal = ideal + ideal;

    int32_t *alive = (int32_t *)malloc(sizeof(int32_t) * (size_t)nb);
    double *cw = (double *)malloc(sizeof(double) * (size_t)nb);
    int32_t need = 0;
    for (int32_t k = 0; k < nb; ++k) {
        alive[k] = 1;
        cw[k] = w[k];
        if (equalize) need += need_copies(w[k], two_ideal);
    }
    int32_t n_alive = nb;

    /* merge: the two lowest by (weight, slot); slots ascend with k */
    uint32_t key[2];
    seed_key(seed, key);
    uint32_t m = 0;
    while (n_alive > 1) {
        int32_t i = -1, j = -1;
        for (int32_t k = 0; k < nb; ++k) {
            if (!alive[k]) continue;
            if (i < 0 || cw[k] < cw[i]) { j = i; i = k; }
            else if (j < 0 || cw[k] < cw[j]) { j = k; }
        }
        double sum = cw[i] + cw[j];
        int go = equalize ? (sum <= ideal || need > m_targ) : (n_alive > m_targ);
        if (!go) break;
        uint32_t ctr[4] = {m, bin, iter, 1u}, r[4];
        or_philox4x32_10(ctr, key, r);
        m += 1;
        double u = or_u53(r[0], r[1]);
        double p_i = cw[i] / sum;
        int32_t keep = (u < p_i) ? i : j;
        int32_t drop = (keep == i) ? j : i;
        if (equalize)
            need = need - need_copies(cw[i], two_ideal) - need_copies(cw[j], two_ideal)
                   + need_copies(sum, two_ideal);
        cw[keep] = sum;
        alive[drop] = 0;
        n_alive -= 1;
    }

    /* split: the survivors up to m_targ copies (nothing to do at m_targ) */
    int32_t o = split_survivors(nb, slot, cw, alive, n_alive, m_targ, out_slot, out_w);
    free(alive);
    free(cw);
    return o;
}

int32_t or_we_iterate(const or_net *net, const or_we_cfg *cfg, uint32_t iter,
                      int32_t *n, int32_t *x, double *w, int32_t *bin,
                      int32_t *origin, int32_t cap,
                      double *flux_out, int64_t *events_out, int32_t *recycled_out,
                      int32_t *end_bin_out)
{
    const int32_t S = net->S, N = *n, M = cfg->m_targ;
    const int32_t NB1 = cfg->n_bins, NB2 = cfg->n_bins2 > 1 ? cfg->n_bins2 : 1, NB = NB1 * NB2;
    if (N > cap || M * NB > cap) return OR_EINVAL;
    int32_t status = OR_OK;

    /* 1. propagate every walker through one interval */
    int64_t events = 0;
    for (int32_t k = 0; k < N; ++k) {
        int64_t f = cfg->engine == 1
                        ? or_tauleap_interval(net, x + (size_t)k * S, cfg->tau, cfg->leap_eps, cfg->seed,
                                              (uint32_t)k, iter)
                        : or_ssa_interval(net, x + (size_t)k * S, cfg->tau, cfg->seed, (uint32_t)k, iter);
        if (f < 0) { status = (int32_t)f; f = 0; }
        events += f;
    }

    /* 2. steady-state recycling B -> A, weight kept, flux recorded */
    double flux = 0.0;
    if (recycled_out)
        for (int32_t k = 0; k < N; ++k) recycled_out[k] = 0;
    if (cfg->recycle) {
        for (int32_t k = 0; k < N; ++k) {
            if (or_coord(S, cfg->tgt_coef, x + (size_t)k * S) >= cfg->tgt_thr) {
                if (recycled_out) recycled_out[k] = 1;
                flux = flux + w[k];
                memcpy(x + (size_t)k * S, cfg->x_rec, sizeof(int32_t) * (size_t)S);
            }
        }
    }

    /* 3. bin assignment */
    for (int32_t k = 0; k < N; ++k) {
        bin[k] = or_bin_of(NB1, cfg->edges, or_coord(S, cfg->bin_coef, x + (size_t)k * S));
        if (NB2 > 1)
            bin[k] += NB1 * or_bin_of(NB2, cfg->edges2, or_coord(S, cfg->bin_coef2, x + (size_t)k * S));
    }
    if (end_bin_out) memcpy(end_bin_out, bin, sizeof(int32_t) * (size_t)N);

    /* 4. resample bin by bin into a fresh ensemble */
    int32_t *nx = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap * (size_t)S);
    double *nw = (double *)malloc(sizeof(double) * (size_t)cap);
    int32_t *nbin = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    int32_t *norig = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    int32_t *bslot = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
    double *bw = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    int32_t *oslot = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M > N ? M : (N > 0 ? N : 1)));
    double *ow = (double *)malloc(sizeof(double) * (size_t)(M > N ? M : (N > 0 ? N : 1)));
    int32_t out = 0;
    for (int32_t b = 0; b < NB; ++b) {
        int32_t nb = 0;
        for (int32_t k = 0; k < N; ++k)
            if (bin[k] == b) { bslot[nb] = k; bw[nb] = w[k]; ++nb; }
        int32_t no = or_resample_bin(nb, bslot, bw, M, cfg->resample_rule, cfg->seed, (uint32_t)b,
                                     iter, oslot, ow);
        for (int32_t o = 0; o < no; ++o) {
            memcpy(nx + (size_t)out * S, x + (size_t)oslot[o] * S, sizeof(int32_t) * (size_t)S);
            nw[out] = ow[o];
            nbin[out] = b;
            norig[out] = oslot[o];
            ++out;
        }
    }
    memcpy(x, nx, sizeof(int32_t) * (size_t)out * S);
    memcpy(w, nw, sizeof(double) * (size_t)out);
    memcpy(bin, nbin, sizeof(int32_t) * (size_t)out);
    memcpy(origin, norig, sizeof(int32_t) * (size_t)out);
    *n = out;
    free(nx); free(nw); free(nbin); free(norig); free(bslot); free(bw); free(oslot); free(ow);

    if (flux_out) *flux_out = flux;
    if (events_out) *events_out = events;
    return status;
}
