"""Pins of the oracle's Hill-type propensities and two-dimensional bins on
the epigenetic switch of Sec. III.C: the exact CME transient (matrix
exponential of the truncated generator), the exact mean first passage time
(sparse solve) against the numbers the paper prints, hand-computed
propensities and bins, and a WE estimate of the MFPT.  CPU only."""
import json
import math
import os
from fractions import Fraction

import numpy as np

import closed_form as cf
from oracle import oracle as orc
from paper_1303_5986_amd import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
PAPER = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))


def test_switch_mfpt_closed_form_matches_the_paper():
    """With A = (0, 30) and B = {g1 >= 50}, the exact MFPT lies within the
    paper's brute-force MLE (1.3e6 +- 6.5e4 s) and WE (1.3e6 +- 3e4 s) one-
    sigma intervals; the truncation of g2 does not matter."""
    m = cf.switch_mfpt(G2=120)
    assert abs(m - PAPER["switch_mle"]["mu"]) < PAPER["switch_mle"]["sigma"]
    assert abs(m - PAPER["switch_we_mfpt"]["value"]) < PAPER["switch_we_mfpt"]["err"]
    assert math.isclose(m, cf.switch_mfpt(G2=200), rel_tol=1e-9)


def test_hill_propensities_at_hand_states():
    """a = (c h) / (1 + (x_r / K)^n), each step one rounding: at (g1, g2) =
    (2, 3) the g1 birth rate is 156 / 28 and the g2 birth rate 30 / 3."""
    onet = orc.OracleNet(wl.switch())
    for g1, g2 in ((2, 3), (0, 30), (7, 0), (49, 1)):
        x = [g1, g2]
        want1 = float(Fraction(156) / (1 + Fraction(g2) ** 3))
        want3 = float(Fraction(30) / (1 + Fraction(g1)))
        assert orc.propensity(onet, x, 0) == want1
        assert orc.propensity(onet, x, 2) == want3
        assert orc.propensity(onet, x, 1) == float(g1)
        assert orc.propensity(onet, x, 3) == float(g2)


def test_ssa_interval_switch_transient():
    """One interval of length 1 from (5, 3), where both Hill factors vary,
    follows the exact CME transient (chi-square over the joint law)."""
    onet = orc.OracleNet(wl.switch())
    ref = cf.switch_transient(x0=(5, 3), t=1.0, G1=250, G2=60)
    assert ref[-1, :].sum() + ref[:, -1].sum() < 1e-9      # the box holds the law
    n = 20000
    counts = np.zeros_like(ref)
    for k in range(n):
        x, _ = orc.ssa_interval(onet, [5, 3], 1.0, 77, k, 0)
        counts[x[0], x[1]] += 1
    assert cf.chi2_pvalue(counts.ravel(), ref.ravel()) > 0.01
    # the g1 marginal alone, where the g2-dependent birth rate acts
    assert cf.chi2_pvalue(counts.sum(axis=1), ref.sum(axis=1)) > 0.01


def test_two_dimensional_bins_by_hand():
    """bin = b1 + 15 b2 on the paper's grid: g1 in unit bins on [0, 10],
    width 10 on [10, 50], then [50, inf); g2 unit on [0, 30], then [30, inf).
    A network that never fires leaves the walkers where they are, so one
    iteration only bins and resamples them."""
    frozen = wl.Network.from_reactions(["g1", "g2"], [({"g1": 1}, {}, 0.0)])
    cfg = wl.WEConfig(**{**wl.switch_config(n_runs=1).__dict__, "net": frozen, "recycle": False,
                         "m_targ": 1})
    states = [(0, 0), (9, 0), (10, 0), (19, 5), (49, 29), (50, 30), (3, 31), (1000, 1000)]
    want = [0, 9, 10, 10 + 15 * 5, 13 + 15 * 29, 14 + 15 * 30, 3 + 15 * 30, 14 + 15 * 30]
    x = np.array(states, np.int32)
    o = orc.OracleWE(cfg, 1, init_x=x, init_w=np.full(len(states), 1.0 / len(states)))
    o.step(1)
    _, _, b, origin = o.walkers()
    got = {int(orig): int(bb) for bb, orig in zip(b, origin)}
    for k, wb in enumerate(want):
        if k in got:
            assert got[k] == wb, (states[k], got[k], wb)
    assert sorted(set(b.tolist())) == sorted(set(want))


def test_switch_we_mfpt_estimate():
    """WE on the paper's grid with reweighting every 100 iterations (4 runs
    x 300 iterations, first 100 discarded): the combined MFPT estimate is
    within a factor 1.6 of the exact value (a run's estimate scatters by
    about 50% at this length)."""
    cfg = wl.switch_config(n_runs=4, n_iters=300)
    fl = []
    for s in cfg.seeds:
        o = orc.OracleWE(cfg, int(s), rw_period=100)
        o.step(300)
        fl.append(np.mean(o.flux[100:]) / cfg.tau)
        assert o.rw_applied == 3
    m = 1.0 / np.mean(fl)
    assert 1 / 1.6 < m / cf.switch_mfpt() < 1.6
