"""Pins of the oracle's steady-state reweighting (Sec. II.B.2, Eq. ss)
against things outside itself: detailed balance of birth-death chains (also
over 40 decades), the closed form of a one-way cycle, the Markov chain tree
theorem by brute force on small dense chains, hand-computed flux matrices,
invariants of the rescaling, and the relaxation speed-up the paper reports.
CPU only."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import closed_form as cf
from oracle import oracle as orc, reweight as rw
from paper_1303_5986_amd import workloads as wl


def _flux_from_rates(K, W):
    """F[i, j] = K[i, j] W_j off the diagonal, the rest of W_j on it (the
    weight that stayed), so that column j sums to W_j."""
    n = len(W)
    F = np.zeros((n, n))
    for j in range(n):
        out = 0.0
        for i in range(n):
            if i != j:
                F[i, j] = K[i, j] * W[j]
                out += F[i, j]
        F[j, j] = W[j] - out
        assert F[j, j] >= 0.0
    return F


def test_flux_accumulation_hand_case():
    F = np.zeros((3, 3))
    start = [0, 0, 1, 2, 1]
    end = [0, 1, 1, 0, 2]
    w = [0.25, 0.125, 0.5, 0.0625, 0.0625]
    rw.accumulate_flux(F, start, end, w)
    rw.accumulate_flux(F, [2], [0], [0.5])
    want = np.zeros((3, 3))
    want[0, 0] = 0.25
    want[1, 0] = 0.125
    want[1, 1] = 0.5
    want[0, 2] = 0.0625 + 0.5
    want[2, 1] = 0.0625
    assert np.array_equal(F, want)
    assert np.array_equal(rw.start_weights(F), [0.375, 0.5625, 0.5625])


def test_birth_death_chain_detailed_balance():
    """A 1-D chain is reversible: pi_{i+1} / pi_i = lam_i / mu_{i+1}."""
    n = 12
    lam = 0.02 + 0.03 * np.arange(n)[::-1]
    mu = 0.01 + 0.02 * np.arange(n)
    K = np.zeros((n, n))
    for i in range(n - 1):
        K[i + 1, i] = lam[i]
        K[i, i + 1] = mu[i + 1]
    rng = np.random.default_rng(1)
    F = _flux_from_rates(K, rng.uniform(0.5, 2.0, n))
    pi = rw.steady_state(F, list(range(n)))
    want = cf.chain_stationary(np.append(lam[:-1], 1.0), np.append(0.0, mu[1:]))
    assert np.allclose(pi, want, rtol=1e-12, atol=0)


def test_one_way_cycle_closed_form():
    """0 -> 1 -> 2 -> 0 with rates a, b, c: the flow around the cycle is the
    same on every edge, so pi is proportional to (1/a, 1/b, 1/c)."""
    a, b, c = 0.3, 0.05, 0.11
    K = np.zeros((3, 3))
    K[1, 0], K[2, 1], K[0, 2] = a, b, c
    F = _flux_from_rates(K, [1.0, 0.7, 1.3])
    pi = rw.steady_state(F, [0, 1, 2])
    want = np.array([1 / a, 1 / b, 1 / c])
    assert np.allclose(pi, want / want.sum(), rtol=1e-13, atol=0)


def _tree_theorem(K):
    """Markov chain tree theorem, by brute force: pi_r is proportional to the
    sum, over all spanning trees directed towards r, of the product of their
    rates (K[i][j]: rate from j into i)."""
    n = len(K)
    weight = []
    for root in range(n):
        others = [v for v in range(n) if v != root]
        total = Fraction(0)
        for succ in itertools.product(range(n), repeat=n - 1):
            nxt = dict(zip(others, succ))
            if any(nxt[v] == v for v in others):
                continue
            ok = True
            for v in others:
                u, steps = v, 0
                while u != root and steps < n:
                    u, steps = nxt[u], steps + 1
                ok = ok and u == root
            if ok:
                prod = Fraction(1)
                for v in others:
                    prod *= K[nxt[v]][v]
                total += prod
        weight.append(total)
    z = sum(weight)
    return [wt / z for wt in weight]


@pytest.mark.parametrize("n,seed", [(4, 7), (5, 8)])
def test_small_dense_chain_tree_theorem(n, seed):
    rng = np.random.default_rng(seed)
    F = rng.integers(1, 9, size=(n, n)).astype(np.float64) / 16.0
    F[rng.integers(0, n), rng.integers(0, n)] = 0.0        # one missing edge (or a diagonal)
    W = rw.start_weights(F)
    K = [[Fraction(F[i, j]) / Fraction(W[j]) for j in range(n)] for i in range(n)]
    want = np.array([float(v) for v in _tree_theorem(K)])
    pi = rw.steady_state(F, list(range(n)))
    assert np.array_equal(pi, want)              # both exact, rounded once


def test_tiny_components_keep_their_digits():
    """A birth-death chain whose stationary law spans 40 decades: every
    component comes out to a few ulps of the closed form."""
    n = 30
    lam = np.full(n, 0.01)
    mu = np.full(n, 0.25)
    K = np.zeros((n, n))
    for i in range(n - 1):
        K[i + 1, i] = lam[i]
        K[i, i + 1] = mu[i + 1]
    F = _flux_from_rates(K, np.ones(n))
    pi = rw.steady_state(F, list(range(n)))
    want = cf.chain_stationary(lam, np.append(0.0, mu[1:]))
    assert pi[-1] < 1e-40
    assert np.allclose(pi, want, rtol=1e-12, atol=0)


def test_component_selection_and_invariants():
    """Bins 0-2 form a strongly connected set holding most of the weight;
    bin 3 was only entered (seen from 2, never left); bin 4 is occupied but
    never started an interval; bin 5 started intervals but is empty now."""
    nb = 6
    F = np.zeros((nb, nb))
    for i, j, v in [(0, 0, 0.2), (1, 0, 0.1), (0, 1, 0.05), (1, 1, 0.3), (2, 1, 0.02),
                    (1, 2, 0.04), (2, 2, 0.1), (3, 2, 0.01), (3, 3, 0.02), (2, 5, 0.01)]:
        F[i, j] = v
    bins = np.array([0, 0, 1, 1, 1, 2, 3, 4])
    w = np.array([0.1, 0.1, 0.2, 0.2, 0.1, 0.15, 0.1, 0.05])
    w0 = w.copy()
    assert rw.reweight(F, bins, w, nb)
    wb = rw.bin_weights(bins, w, nb)
    assert np.array_equal(w[6:], w0[6:])                       # bins 3, 4 untouched
    assert math.isclose(wb[:3].sum(), 0.85, rel_tol=1e-14)     # component keeps its weight
    assert math.isclose(w.sum(), w0.sum(), rel_tol=1e-14)
    pi = rw.steady_state(F, [0, 1, 2])
    assert np.allclose(wb[:3] / wb[:3].sum(), pi, rtol=1e-13)
    assert math.isclose(w[0] / w[1], 1.0) and math.isclose(w[2] / w[4], 2.0)  # ratios in a bin kept


def test_fixed_point_is_unchanged():
    """An ensemble whose bin weights already solve Eq. ss is left alone."""
    rng = np.random.default_rng(3)
    n = 6
    F = rng.uniform(0.01, 0.2, size=(n, n))
    pi = rw.steady_state(F, list(range(n)))
    bins = np.repeat(np.arange(n), 3)
    w = np.repeat(pi / 3.0, 3)
    w0 = w.copy()
    assert rw.reweight(F, bins, w, n)
    assert np.allclose(w, w0, rtol=1e-13, atol=0)


def test_single_bin_component_is_skipped():
    F = np.zeros((3, 3))
    F[0, 0], F[1, 0], F[1, 1] = 0.5, 0.1, 0.4        # 0 -> 1 only: two components
    bins = np.array([0, 0, 1])
    w = np.array([0.3, 0.3, 0.4])
    w0 = w.copy()
    assert not rw.reweight(F, bins, w, 3)
    assert np.array_equal(w, w0)


def _bd_unit_bins(seed):
    net = wl.birth_death()
    return wl.WEConfig(name="bd_unit", net=net, x0=np.array([10], np.int32),
                       bin_coef=np.array([1.0]), edges=wl.uniform_edges(0.0, 100.0, 100),
                       m_targ=4, tau=1.0, n_iters=40, seeds=np.array([seed], np.uint64))


def test_flux_matrix_of_a_run_adds_up():
    """The column sums of the accumulated F equal the start-bin weights of
    every interval after the first, summed from ensemble snapshots."""
    cfg = _bd_unit_bins(11)
    o = orc.OracleWE(cfg, 11, rw_period=1000)
    want = np.zeros(cfg.n_bins)
    o.step(1)
    for _ in range(12):
        _, w, b, _ = o.walkers()
        want += np.bincount(b, weights=w, minlength=cfg.n_bins)
        o.step(1)
    assert np.allclose(rw.start_weights(o.rw_F), want, rtol=1e-12, atol=1e-15)
    assert o.rw_applied == 0 and o.rw_skipped == 0


def test_reweighting_speeds_up_relaxation():
    """Birth-death (k = 1, gamma = 0.025) in unit bins from X = 10: the
    stationary law is Poisson(40) with a relaxation time of 40 intervals.
    After 40 intervals plain WE is still far from it; reweighting every 5
    intervals is much closer (the acceleration of Sec. II.B.2 and III.B).
    Total weight is conserved throughout."""
    lam = np.full(300, 1.0)
    mu = 0.025 * np.arange(300)
    pi = cf.chain_stationary(lam, mu)[:100]
    tv = {}
    for period in (0, 5):
        tv[period] = []
        for seed in (3, 4, 5):
            o = orc.OracleWE(_bd_unit_bins(seed), seed, rw_period=period)
            o.step(40)
            _, w, b, _ = o.walkers()
            assert math.isclose(w.sum(), 1.0, rel_tol=1e-12)
            tv[period].append(0.5 * np.abs(rw.bin_weights(b, w, 100) - pi).sum())
        if period:
            assert o.rw_applied == 8 and o.rw_skipped == 0
    assert min(tv[0]) > 0.6
    assert max(tv[5]) < 0.4
    assert np.mean(tv[5]) < 0.3


@pytest.mark.parametrize("n,seed", [(20, 1), (64, 2)])
def test_state_reduction_matches_the_exact_solve(n, seed):
    """The FP64 state reduction used past EXACT_MAX bins against the exact
    solver, on sparse random chains whose rates span six decades."""
    rng = np.random.default_rng(seed)
    F = np.zeros((n, n))
    for j in range(n):
        for i in rng.choice(n, size=4, replace=False):
            F[i, j] = 10.0 ** rng.uniform(-6, 0)
        F[(j + 1) % n, j] = 10.0 ** rng.uniform(-6, 0)      # a cycle keeps it irreducible
    exact = rw.steady_state(F, list(range(n)))
    gth = rw.steady_state_gth(F, list(range(n)))
    assert np.allclose(gth, exact, rtol=1e-11, atol=0)


def test_state_reduction_keeps_tiny_components():
    n = 30
    K = np.zeros((n, n))
    for i in range(n - 1):
        K[i + 1, i] = 0.01
        K[i, i + 1] = 0.25
    F = _flux_from_rates(K, np.ones(n))
    want = cf.chain_stationary(np.full(n, 0.01), np.append(0.0, np.full(n - 1, 0.25)))
    assert np.allclose(rw.steady_state_gth(F, list(range(n))), want, rtol=1e-12, atol=0)
