"""Steady-state reweighting, written from the paper (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It is the plain, slow statement of the reweighting step
of Sec. II.B.2 ("Reweighting", Eq. ss) that the GPU path is checked against.

What the paper fixes:
  * w_i is the weight in bin i (the sum of its walkers' weights);
  * f_ij is the flux of weight into bin i from bin j, and f_ij = k_ij w_j
    holds whether or not the ensemble is in steady state, so measured fluxes
    and bin weights give the inter-bin rates k_ij;
  * the steady-state bin weights solve Eq. ss,
        sum_j (k_ij w_j - k_ji w_i) = 0   for every bin i,
    and the walkers of each bin are then rescaled to them.

Readings taken where the paper is silent (each listed in the design notes):
  RW1  f_ij is accumulated from the start of the run: every interval adds,
       slot by slot in ascending slot order, the weight each walker carried
       through the interval to F[i, j], j its bin at the start of the interval
       and i its bin at the end (after recycling, so a walker recycled from B
       counts as moving into the bin of A).  The rates are constants of the
       dynamics, so all intervals estimate the same k_ij.  The walkers of the
       very first interval have no bin yet (they are binned by the first
       resampling), so accumulation starts with the second interval.
       Optionally (rw_reset) F starts over after every event, so that each
       event uses only the intervals since the previous one: the rates then
       come from an ensemble that earlier events have already brought closer
       to steady state, which is how repeated application converges.
  RW2  W_j = sum_i F[i, j] (ascending i): the weight that started intervals in
       bin j; k_ij = F[i, j] / W_j for i != j.
  RW3  A reweighting event happens after the resampling of every iteration t
       with (t + 1) % period == 0.  Candidates are the bins that are occupied
       now, weigh more than zero (a bin of zero weight cannot be scaled to a
       positive target) and have W_j > 0.  Eq. ss has a unique positive solution only on a
       strongly connected set of bins (edge j -> i when F[i, j] > 0, i != j),
       and near the edge of the explored region transitions are often seen
       in one direction only.  So the event reweights the strongly connected
       component, within the candidates, of the candidate holding the most
       weight now (ties: the lowest bin), and nothing if that component is a
       single bin.
  RW4  pi solves Eq. ss on that component with sum(pi) = 1.  The component
       keeps its total weight W_A = sum_a w_a (ascending a): bin a's target is
       pi_a / Z * W_A (Z = sum of pi, ascending), and each of its walkers is
       multiplied by target / w_a.  All other bins are left as they are, so
       the total weight is conserved.

The solve here is the textbook one, done exactly: the balance equations
with one of them replaced by the normalisation, solved by Gaussian
elimination on the exact values of the measured doubles, and one rounding
of each pi_a at the end.  (Floating-point LU would do, but its error is
normwise: bins many decades below the heaviest would come out with few
correct digits.)  Written for q_b = pi_b / W_b, every coefficient is a
double or an exact sum of doubles,
    sum_b F[a, b] q_b - q_a sum_b F[b, a] = 0,   sum_b W_b q_b = 1   (b != a),
so one power-of-two scale makes the system integer, and fraction-free
(Bareiss) elimination solves it in Python integers.  That costs O(n^3)
operations on integers of O(n) words, too slow past ~64 bins; larger sets
(the two-dimensional grids of Sec. III.C) are solved instead by state
reduction in FP64 (Grassmann, Taksar and Heyman 1985), whose error is
entrywise relative (no subtractions), and which the tests pin against the
exact solver.  Strong connectivity comes from scipy's graph routine.
Neither shares code with the device.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Optional

import numpy as np


def accumulate_flux(F: np.ndarray, start_bin, end_bin, w) -> None:
    """RW1: F[end, start] += weight, walker by walker in slot order."""
    for k in range(len(w)):
        i, j = int(end_bin[k]), int(start_bin[k])
        F[i, j] = F[i, j] + float(w[k])


def start_weights(F: np.ndarray) -> np.ndarray:
    """RW2: W_j = sum_i F[i, j], i ascending."""
    nb = F.shape[0]
    W = np.zeros(nb, np.float64)
    for j in range(nb):
        acc = 0.0
        for i in range(nb):
            acc = acc + float(F[i, j])
        W[j] = acc
    return W


def bin_weights(bins, w, n_bins: int) -> np.ndarray:
    """w_i: the weights of bin i's walkers summed in slot order."""
    out = np.zeros(n_bins, np.float64)
    for k in range(len(w)):
        b = int(bins[k])
        out[b] = out[b] + float(w[k])
    return out


def component_of(F: np.ndarray, cand, pivot: int) -> list:
    """RW3: the bins of `cand` in the strongly connected component of
    `pivot` in the graph j -> i (F[i, j] > 0, i != j) restricted to `cand`,
    ascending."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    cand = list(cand)
    sub = np.asarray(F)[np.ix_(cand, cand)] > 0.0
    np.fill_diagonal(sub, False)
    # csgraph edge (r, c) means r -> c: the transpose of F's (into, from)
    _, label = connected_components(csr_matrix(sub.T.astype(np.int8)), directed=True,
                                    connection="strong")
    lp = label[cand.index(pivot)]
    return [b for b, l in zip(cand, label) if l == lp]


EXACT_MAX = 64


def steady_state_gth(F: np.ndarray, active) -> np.ndarray:
    """Eq. ss on a strongly connected set by state reduction: with
    P[i, j] = k_ji (rate from i into j), remove the last state m each step,
    P[i, j] += P[i, m] P[m, j] / s_m with s_m = sum_{j<m} P[m, j]; then
    pi_0 = 1, pi_m = sum_{i<m} pi_i P[i, m] / s_m; normalised to sum 1."""
    active = list(active)
    na = len(active)
    W = start_weights(F)
    P = np.zeros((na, na))
    for a, i in enumerate(active):
        for b, j in enumerate(active):
            if a != b:
                P[b, a] = F[i, j] / W[j]          # rate from j (index b) into i (index a)
    s = np.zeros(na)
    for m in range(na - 1, 0, -1):
        s[m] = P[m, :m].sum()
        P[:m, :m] += np.outer(P[:m, m], P[m, :m] / s[m])
    pi = np.zeros(na)
    pi[0] = 1.0
    for m in range(1, na):
        pi[m] = float(pi[:m] @ P[:m, m]) / s[m]
    return pi / pi.sum()


def steady_state(F: np.ndarray, active) -> Optional[np.ndarray]:
    """RW2, RW4: the solution of Eq. ss on a strongly connected set of bins
    (ascending) with sum 1; None for fewer than two bins.  Exact (one
    rounding per component) up to EXACT_MAX bins, state reduction beyond."""
    active = list(active)
    na = len(active)
    if na < 2:
        return None
    if na > EXACT_MAX:
        return steady_state_gth(F, active)
    W = start_weights(F)
    vals = [float(F[i, j]) for i in active for j in active] + [float(W[j]) for j in active]
    e_min = min(math.frexp(v)[1] for v in vals if v != 0.0) - 53
    def z(v):                                    # the double v times 2^-e_min, exactly
        if v == 0.0:
            return 0
        m, e = math.frexp(v)
        return int(m * (1 << 53)) << (e - 53 - e_min)
    Fz = [[z(float(F[i, j])) for j in active] for i in active]
    A = []
    for a in range(na - 1):
        row = [Fz[a][b] if b != a else 0 for b in range(na)]
        row[a] = -sum(Fz[b][a] for b in range(na) if b != a)
        A.append(row + [0])
    A.append([z(float(W[j])) for j in active] + [1 << (-e_min) if e_min <= 0 else 0])
    if e_min > 0:                                # right-hand side 1 scaled by 2^-e_min
        A[-1] = [v << e_min for v in A[-1][:na]] + [1]
    # Bareiss: every division below is exact
    prev = 1
    for k in range(na):
        if A[k][k] == 0:
            r = next(r for r in range(k + 1, na) if A[r][k] != 0)
            A[k], A[r] = A[r], A[k]
        for i in range(k + 1, na):
            for j in range(k + 1, na + 1):
                A[i][j] = (A[i][j] * A[k][k] - A[i][k] * A[k][j]) // prev
            A[i][k] = 0
        prev = A[k][k]
    q = [Fraction(0)] * na
    for a in range(na - 1, -1, -1):
        acc = Fraction(A[a][na]) - sum((A[a][b] * q[b] for b in range(a + 1, na)), Fraction(0))
        q[a] = acc / A[a][a]
    return np.array([float(q[a] * Fraction(float(W[j]))) for a, j in enumerate(active)])


def reweight(F: np.ndarray, bins, w: np.ndarray, n_bins: int) -> bool:
    """One reweighting event (RW3, RW4) on the current ensemble (bins, w in
    slot order); w is rescaled in place.  Returns True if the event applied."""
    wb = bin_weights(bins, w, n_bins)
    occupied = np.zeros(n_bins, bool)
    occupied[np.asarray(bins, np.int64)] = True
    W = start_weights(F)
    cand = [i for i in range(n_bins) if occupied[i] and wb[i] > 0.0 and W[i] > 0.0]
    if len(cand) < 2:
        return False
    pivot = cand[0]
    for i in cand:
        if wb[i] > wb[pivot]:
            pivot = i
    active = component_of(F, cand, pivot)
    pi = steady_state(F, active)
    if pi is None:
        return False
    Z = 0.0
    for v in pi:
        Z = Z + float(v)
    WA = 0.0
    for i in active:
        WA = WA + float(wb[i])
    factor = {}
    for a, i in enumerate(active):
        factor[i] = (float(pi[a]) / Z * WA) / float(wb[i])
    for k in range(len(w)):
        b = int(bins[k])
        if b in factor:
            w[k] = w[k] * factor[b]
    return True
