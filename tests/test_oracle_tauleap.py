"""Pins of the oracle's tau-leaping engine (Sec. IV proposes combining WE
with tau-leaping; Gillespie 2001, step bound of Cao, Gillespie and Petzold
2006) against exact laws.  tau-leaping is approximate: the pins check the
parts that are exact (the Poisson samplers, the fall-back to exact events,
conservation, non-negativity) and that the approximation error is small
where leaps are taken.  CPU only."""
import math

import numpy as np
import pytest
from scipy import stats

import closed_form as cf
from oracle import oracle as orc
from paper_1303_5986_amd import workloads as wl


@pytest.mark.parametrize("mean", [5.0, 19.5, 20.5, 500.0])
def test_pure_birth_is_one_poisson_leap(mean):
    """0 -> X at a constant rate consumes nothing, so the step bound is
    infinite and the whole interval is one leap: X(tau) ~ Poisson(k tau)
    exactly.  Means on both sides of 20 pin the inversion and the PTRS
    samplers."""
    net = wl.Network.from_reactions(["X"], [({}, {"X": 1}, mean)])
    onet = orc.OracleNet(net)
    xs = np.array([orc.tauleap_interval(onet, [0], 1.0, 0.03, 3, k, 0)[0][0] for k in range(20000)])
    hi = int(mean + 12 * math.sqrt(mean) + 20)
    ref = stats.poisson.pmf(np.arange(hi + 1), mean)
    counts = np.bincount(xs, minlength=hi + 1)[:hi + 1]
    assert xs.max() <= hi
    assert cf.chi2_pvalue(counts, ref) > 0.01


def test_small_steps_fall_back_to_exact_events():
    """Where the step bound stays below 10 / a0 (birth-death at X = 40:
    a0 = 2, bound 0.5) every step is an exact event drawn from the SSA
    stream, so the result equals the SSA engine's bit for bit."""
    onet = orc.OracleNet(wl.birth_death())
    for k in range(300):
        a, ea = orc.tauleap_interval(onet, [40], 1.0, 0.03, 11, k, 2)
        b, eb = orc.ssa_interval(onet, [40], 1.0, 11, k, 2)
        assert np.array_equal(a, b) and ea == eb


def test_leaps_on_isomerization_conserve_and_stay_close():
    """A <-> B with 1000 molecules: leaps are taken; the total is conserved,
    no count goes negative, and the law of A(0.7) (Binomial, exact) is
    matched in mean and variance to within 2% and 5%."""
    net = wl.isomerization(1.0, 0.5)
    onet = orc.OracleNet(net)
    n = 1000
    xs = np.array([orc.tauleap_interval(onet, [n, 0], 0.7, 0.03, 5, k, 0)[0] for k in range(6000)])
    assert (xs.sum(axis=1) == n).all() and (xs >= 0).all()
    ref = cf.isomerization_transient(n, 1.0, 0.5, 0.7)
    m = (ref * np.arange(n + 1)).sum()
    v = (ref * np.arange(n + 1) ** 2).sum() - m * m
    assert abs(xs[:, 0].mean() / m - 1) < 0.02
    assert abs(xs[:, 0].var() / v - 1) < 0.05
    _, ev = orc.tauleap_interval(onet, [n, 0], 0.7, 0.03, 5, 0, 0)
    assert ev > 100            # reactions fired, counted through the leaps


def test_schlogl_transient_close_to_the_cme():
    """Schloegl from X = 82 over 0.5 s with eps = 0.03: chi-square against
    the exact transient law still passes at this sample size."""
    onet = orc.OracleNet(wl.schlogl())
    lam, mu = cf.schlogl_rates(700)
    ref = cf.chain_transient(lam, mu, 82, 0.5)
    xs = np.array([orc.tauleap_interval(onet, [82], 0.5, 0.03, 5, k, 3)[0][0] for k in range(8000)])
    assert cf.chi2_pvalue(np.bincount(xs, minlength=701)[:701], ref) > 0.001


def test_tauleap_we_iteration_conserves_weight():
    cfg = wl.schlogl_config(n_runs=1, n_iters=20)
    cfg.engine = "tauleap"
    o = orc.OracleWE(cfg, 7)
    o.step(20)
    _, w, _, _ = o.walkers()
    assert math.isclose(w.sum(), 1.0, rel_tol=1e-12)
