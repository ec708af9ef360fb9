"""Exact references (closed forms and chemical-master-equation solutions) used
to pin the CPU oracle.  Independent of both the oracle and the HIP library:
each law is written from the mathematics of the model it describes.

  * birth-death 0 -> X (k), X -> 0 (gamma x): transient law from X0 is
    Binomial(X0, e^{-gamma t}) convolved with Poisson((k/gamma)(1-e^{-gamma t}));
    stationary law Poisson(k/gamma).
  * one-species birth-death chains with birth rate lambda(x), death rate mu(x):
    stationary pi(x) proportional to prod_{y<x} lambda(y)/mu(y+1); mean first
    passage a -> b (a < b) = sum_{k=a}^{b-1} (sum_{j<=k} pi_j) / (lambda_k pi_k).
  * CME transients by the matrix exponential of a truncated generator.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as la
from scipy import stats


# ---------------------------------------------------------------- birth-death
def poisson_pmf(lam: float, kmax: int) -> np.ndarray:
    return stats.poisson.pmf(np.arange(kmax + 1), lam)


def poisson_sf(lam: float, k: int) -> float:
    """P(X >= k)."""
    return float(stats.poisson.sf(k - 1, lam))


def bd_transient_pmf(x0: int, k: float, gamma: float, t: float, kmax: int) -> np.ndarray:
    """Survivors of the x0 initial copies are Binomial(x0, e^{-gamma t}); the
    copies born in (0,t] that are still alive are Poisson((k/gamma)(1-e^{-gamma t}))."""
    p = math.exp(-gamma * t)
    binom = stats.binom.pmf(np.arange(x0 + 1), x0, p)
    pois = stats.poisson.pmf(np.arange(kmax + 1), (k / gamma) * (1.0 - p))
    return np.convolve(binom, pois)[: kmax + 1]


# ---------------------------------------------------------------- Schloegl
SCHLOGL = dict(k1=3e-7, k2=1e-4, k3=1e-3, k4=3.5, A=1e5, B=2e5)


def schlogl_rates(N: int):
    """Birth and death rates of X under combinatorial mass action:
    birth = k1 A x(x-1)/2 + k3 B, death = k2 x(x-1)(x-2)/6 + k4 x."""
    p = SCHLOGL
    x = np.arange(N + 1, dtype=np.float64)
    lam = p["k1"] * p["A"] * x * (x - 1) / 2.0 + p["k3"] * p["B"]
    mu = p["k2"] * x * (x - 1) * (x - 2) / 6.0 + p["k4"] * x
    return lam, mu


def chain_stationary(lam: np.ndarray, mu: np.ndarray) -> np.ndarray:
    logpi = np.zeros(len(lam))
    for x in range(1, len(lam)):
        logpi[x] = logpi[x - 1] + math.log(lam[x - 1]) - math.log(mu[x])
    pi = np.exp(logpi - logpi.max())
    return pi / pi.sum()


def chain_mfpt(lam: np.ndarray, mu: np.ndarray, a: int, b: int) -> float:
    pi = chain_stationary(lam, mu)
    cum = np.cumsum(pi)
    return float(sum(cum[k] / (lam[k] * pi[k]) for k in range(a, b)))


def chain_transient(lam: np.ndarray, mu: np.ndarray, x0: int, t: float) -> np.ndarray:
    """p(t) = expm(Q t) e_{x0} on the chain truncated at len(lam)-1 (no birth
    out of the top state)."""
    N = len(lam) - 1
    Q = np.zeros((N + 1, N + 1))
    for k in range(N + 1):
        up = lam[k] if k < N else 0.0
        Q[k, k] -= up + mu[k]
        if k < N:
            Q[k + 1, k] += up
        if k > 0:
            Q[k - 1, k] += mu[k]
    p0 = np.zeros(N + 1)
    p0[x0] = 1.0
    return la.expm(Q * t) @ p0


# ---------------------------------------------------------------- futile cycle
def futile_states(total: int = 100):
    """States (S1, B1, B2) with S1 + S2 + B1 + B2 = total, E1 = 1 - B1,
    E2 = 1 - B2 (one enzyme of each kind)."""
    st = []
    for b1 in (0, 1):
        for b2 in (0, 1):
            for s1 in range(0, total + 1 - b1 - b2):
                st.append((s1, b1, b2))
    return st


def futile_transient(t: float, kf: float = 1.0, ks: float = 0.1, total: int = 100,
                     s1_0: int = 50):
    states = futile_states(total)
    idx = {s: i for i, s in enumerate(states)}
    n = len(states)
    Q = np.zeros((n, n))

    def move(frm, to, rate):
        if rate > 0:
            Q[idx[to], idx[frm]] += rate
            Q[idx[frm], idx[frm]] -= rate

    for (s1, b1, b2) in states:
        s2 = total - s1 - b1 - b2
        e1, e2 = 1 - b1, 1 - b2
        st = (s1, b1, b2)
        if e1 and s1:
            move(st, (s1 - 1, 1, b2), kf * s1)       # E1 + S1 -> B1
        if b1:
            move(st, (s1 + 1, 0, b2), kf)            # B1 -> E1 + S1
            move(st, (s1, 0, b2), ks)                # B1 -> E1 + S2
        if e2 and s2:
            move(st, (s1, b1, 1), kf * s2)           # E2 + S2 -> B2
        if b2:
            move(st, (s1, b1, 0), kf)                # B2 -> E2 + S2
            move(st, (s1 + 1, b1, 0), ks)            # B2 -> E2 + S1
    p0 = np.zeros(n)
    p0[idx[(s1_0, 0, 0)]] = 1.0
    return states, la.expm(Q * t) @ p0


# ---------------------------------------------------------------- two-state
def isomerization_transient(n: int, k_ab: float, k_ba: float, t: float) -> np.ndarray:
    """A <-> B with all n molecules starting as A: each molecule is an
    independent two-state chain, so #A(t) ~ Binomial(n, p(t)) with
    p(t) = k_ba/(k_ab+k_ba) + k_ab/(k_ab+k_ba) e^{-(k_ab+k_ba) t}."""
    s = k_ab + k_ba
    p = k_ba / s + (k_ab / s) * math.exp(-s * t)
    return stats.binom.pmf(np.arange(n + 1), n, p)


# ---------------------------------------------------------------- statistics
def chi2_pvalue(counts: np.ndarray, probs: np.ndarray, min_expected: float = 5.0) -> float:
    """Pearson chi-square goodness of fit; cells with small expectation are
    pooled (in order) until each pooled cell expects >= min_expected."""
    counts = np.asarray(counts, np.float64)
    probs = np.asarray(probs, np.float64)
    n = counts.sum()
    probs = probs / probs.sum()
    exp = probs * n
    obs_p, exp_p = [], []
    co, ce = 0.0, 0.0
    for o, e in zip(counts, exp):
        co += o
        ce += e
        if ce >= min_expected:
            obs_p.append(co)
            exp_p.append(ce)
            co, ce = 0.0, 0.0
    if ce > 0 or co > 0:
        if exp_p:
            obs_p[-1] += co
            exp_p[-1] += ce
        else:
            obs_p.append(co)
            exp_p.append(ce)
    obs_p = np.array(obs_p)
    exp_p = np.array(exp_p)
    chi2 = float(((obs_p - exp_p) ** 2 / exp_p).sum())
    dof = max(len(obs_p) - 1, 1)
    return float(stats.chi2.sf(chi2, dof))


# ---------------------------------------------------------------- epigenetic switch
SWITCH = dict(a1=156.0, a2=30.0, n=3, m=1, K1=1.0, K2=1.0, k0=1.0)


def switch_rates(g1: int, g2: int):
    """Birth and death rates of the switch of Sec. III.C at (g1, g2):
    g1 born at a1 / (1 + (g2/K2)^n), g2 at a2 / (1 + (g1/K1)^m), each copy
    dies at k0."""
    p = SWITCH
    b1 = p["a1"] / (1.0 + (g2 / p["K2"]) ** p["n"])
    b2 = p["a2"] / (1.0 + (g1 / p["K1"]) ** p["m"])
    return b1, p["k0"] * g1, b2, p["k0"] * g2


def _switch_generator(G1: int, G2: int, absorb_g1: int = None):
    """Sparse generator (column = from) of the switch on [0, G1] x [0, G2],
    no births out of the box; with absorb_g1, states g1 >= absorb_g1 are
    cut off (their inflow is lost: first-passage form)."""
    import scipy.sparse as sp
    top1 = G1 if absorb_g1 is None else absorb_g1 - 1
    n1, n2 = top1 + 1, G2 + 1
    idx = lambda a, b: a * n2 + b
    rows, cols, vals = [], [], []
    diag = np.zeros(n1 * n2)
    for a in range(n1):
        for b in range(n2):
            i = idx(a, b)
            b1, d1, b2, d2 = switch_rates(a, b)
            if a < G1:                      # birth of g1 (lost if it lands in the cut-off set)
                diag[i] -= b1
                if a + 1 <= top1:
                    rows.append(idx(a + 1, b)); cols.append(i); vals.append(b1)
            if a > 0:
                diag[i] -= d1
                rows.append(idx(a - 1, b)); cols.append(i); vals.append(d1)
            if b < G2:
                diag[i] -= b2
                rows.append(idx(a, b + 1)); cols.append(i); vals.append(b2)
            if b > 0:
                diag[i] -= d2
                rows.append(idx(a, b - 1)); cols.append(i); vals.append(d2)
    rows += list(range(n1 * n2)); cols += list(range(n1 * n2)); vals += list(diag)
    Q = sp.csc_matrix((vals, (rows, cols)), shape=(n1 * n2, n1 * n2))
    return Q, n1, n2


def switch_mfpt(a=(0, 30), b_g1: int = 50, G2: int = 120) -> float:
    """Mean first passage time from state a into {g1 >= b_g1}: solve
    Q_T^T m = -1 over the states below b_g1 (the backward equation)."""
    import scipy.sparse.linalg as spla
    Q, n1, n2 = _switch_generator(b_g1, G2, absorb_g1=b_g1)
    m = spla.spsolve(Q.T.tocsc(), -np.ones(n1 * n2))
    return float(m[a[0] * n2 + a[1]])


def switch_transient(x0=(0, 30), t: float = 0.5, G1: int = 60, G2: int = 80) -> np.ndarray:
    """P(g1, g2, t) from x0 on [0, G1] x [0, G2] (no births out of the box);
    array [G1 + 1, G2 + 1]."""
    import scipy.sparse.linalg as spla
    Q, n1, n2 = _switch_generator(G1, G2)
    p0 = np.zeros(n1 * n2)
    p0[x0[0] * n2 + x0[1]] = 1.0
    return spla.expm_multiply(Q * t, p0).reshape(n1, n2)
