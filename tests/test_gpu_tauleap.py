"""GPU checks of the tau-leaping engine against the oracle and exact laws.

Both sides take the same steps in the same FP64 order with the same Philox
words (the leap stream (n, slot, iter, 4), exact events from the SSA
stream).  Leaps call exp, log, sqrt and lgamma, whose device and host
versions may differ in the last bit; a Poisson draw can then change when a
uniform falls within an ulp of a cumulative probability, after which that
walker's trajectory differs.  So: where every step is an exact event the
ensembles must be identical; where leaps are taken, at least 99% of walkers
must be identical after every iteration and the laws must agree."""
import math

import numpy as np
import pytest
from scipy import stats

import closed_form as cf
from oracle import oracle as orc
from paper_1303_5986_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _we():
    from paper_1303_5986_amd import we
    return we


def _say(msg):
    print(msg, flush=True)


def test_exact_fallback_is_bit_identical():
    """Birth-death at X ~ 40: every step bound is below 10 / a0, so the
    engine takes exact events only and must match the oracle bit for bit."""
    _say("case: tau-leap engine, birth-death (exact events only), 3 runs x 20 iterations")
    we = _we()
    cfg = wl.birth_death_config(n_runs=3, n_iters=20)
    cfg.engine = "tauleap"
    sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=20)
    ors = [orc.OracleWE(cfg, int(s)) for s in cfg.seeds]
    for it in range(20):
        sim.step(1)
        for r, o in enumerate(ors):
            o.step(1)
            g, h = sim.walkers(r), o.walkers()
            for u, v in zip(g, h):
                assert np.array_equal(np.asarray(u), np.asarray(v)), (it, r)


@pytest.mark.parametrize("mean", [5.0, 500.0])
def test_one_leap_pure_birth_is_poisson(mean):
    """0 -> X at rate `mean` consumes nothing: each walker's interval is one
    leap, X(1) ~ Poisson(mean) exactly (inversion below 20, PTRS above)."""
    _say(f"case: tau-leap pure birth, mean {mean}, one bin x 4096 walkers x 2 runs")
    we = _we()
    net = wl.Network.from_reactions(["X"], [({}, {"X": 1}, mean)])
    cfg = wl.WEConfig(name="birth", net=net, x0=np.array([0], np.int32), bin_coef=np.array([1.0]),
                      edges=np.array([-1.0, 1e9]), m_targ=4096, tau=1.0, n_iters=1,
                      seeds=np.array([5, 6], np.uint64), engine="tauleap")
    sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=1)
    sim.step(1)
    xs = np.concatenate([sim.walkers(r)[0][:, 0] for r in range(2)])
    hi = int(mean + 12 * math.sqrt(mean) + 20)
    assert xs.max() <= hi
    ref = stats.poisson.pmf(np.arange(hi + 1), mean)
    assert cf.chi2_pvalue(np.bincount(xs, minlength=hi + 1)[:hi + 1], ref) > 0.01


def test_schlogl_leaps_match_oracle():
    """Schloegl started in the upper well (40 walkers at X = 420 ... 615, no
    recycling), where most steps are leaps: after every iteration at least
    99% of the walkers equal the oracle's, and the weighted mean counts
    agree to 2%."""
    _say("case: tau-leap engine, Schloegl upper well, 2 runs x 8 iterations")
    we = _we()
    cfg = wl.schlogl_config(n_runs=2, seed0=41, n_iters=8, recycle=False)
    cfg.engine = "tauleap"
    x0 = np.arange(420, 620, 5, dtype=np.int32).reshape(-1, 1)
    w0 = np.full(len(x0), 1.0 / len(x0))
    sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=8)
    ors = []
    for r, s in enumerate(cfg.seeds):
        sim.set_ensemble(r, x0, w0)
        ors.append(orc.OracleWE(cfg, int(s), init_x=x0, init_w=w0))
    worst = 1.0
    for it in range(8):
        sim.step(1)
        for r, o in enumerate(ors):
            o.step(1)
            gx, gw, gb, _ = sim.walkers(r)
            ox, ow, ob, _ = o.walkers()
            same = float(np.mean((gx == ox).all(axis=1))) if len(gw) == len(ow) else 0.0
            worst = min(worst, same)
            assert same >= 0.99, (it, r, same)
            assert abs(np.dot(gw, gx[:, 0]) / np.dot(ow, ox[:, 0]) - 1.0) < 0.02
    _say(f"   smallest identical fraction {worst:.4f}")


def test_tauleap_rejected_where_unsupported():
    we = _we()
    with pytest.raises(we.WEError):
        c = wl.switch_config(n_runs=1)
        c.engine = "tauleap"
        we.sim_from_config(c, kernel=we.WE_KERNEL_LANE)
    with pytest.raises(we.WEError):
        c = wl.schlogl_config(n_runs=1)
        c.engine = "tauleap"
        we.sim_from_config(c, kernel=we.WE_KERNEL_WAVE)
    c = wl.schlogl_config(n_runs=1)
    c.engine = "tauleap"
    with pytest.raises(we.WEError):
        we.Batch([c, c], max_iters=4)
