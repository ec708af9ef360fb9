"""GPU parity of steady-state reweighting (Sec. II.B.2, Eq. ss) against the
CPU oracle.

The flux matrix is a sum of walker weights in a fixed order on both sides,
so until the first reweighting event it must be identical, and so must
every walker.  The event itself solves Eq. ss in two different ways: the
oracle exactly (rational elimination, rounded once), the device by state
reduction in FP64, whose error is entrywise relative and of order n^3 u for
n bins (O'Cinneide 1993): about 1e-11 for the 40-bin components here, and
far smaller in practice.  The rescaled weights carry that error into later
iterations (each event adds its own), so weights, fluxes and the flux matrix
are compared with rtol 1e-9 after the first event, while states, bins,
parents and the event counts must still be identical (a merge outcome would
flip only for a draw within ~1e-12 of its threshold)."""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1303_5986_amd import workloads as wl

pytestmark = pytest.mark.gpu

RTOL = 1e-9


def _we():
    from paper_1303_5986_amd import we
    return we


def _say(msg):
    print(msg, flush=True)


def _bd_unit(n_bins, seeds, x0=10):
    return wl.WEConfig(name="bd_unit", net=wl.birth_death(), x0=np.array([x0], np.int32),
                       bin_coef=np.array([1.0]), edges=wl.uniform_edges(0.0, float(n_bins), n_bins),
                       m_targ=4, tau=1.0, n_iters=40, seeds=np.asarray(seeds, np.uint64))


def _compare(it, r, g, o, exact):
    gx, gw, gb, go = g
    ox, ow, ob, oo = o
    assert len(gw) == len(ow), f"iter {it} run {r}: {len(gw)} vs {len(ow)} walkers"
    assert np.array_equal(gx, ox), f"iter {it} run {r}: states differ"
    assert np.array_equal(gb, ob), f"iter {it} run {r}: bins differ"
    assert np.array_equal(go, oo), f"iter {it} run {r}: parents differ"
    if exact:
        assert np.array_equal(gw.view(np.uint64), ow.view(np.uint64)), f"iter {it} run {r}: weights differ"
    else:
        np.testing.assert_allclose(gw, ow, rtol=RTOL, atol=0, err_msg=f"iter {it} run {r}")


def _run(cfg, period, n_iters, reset=False):
    we = _we()
    sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=n_iters, rw_period=period,
                             rw_reset=reset)
    ors = [orc.OracleWE(cfg, int(s), rw_period=period, rw_reset=reset) for s in cfg.seeds]
    for it in range(n_iters):
        sim.step(1)
        exact = it + 1 < period          # no event has happened yet
        for r, o in enumerate(ors):
            o.step(1)
            _compare(it, r, sim.walkers(r), o.walkers(), exact)
            F = sim.rw_flux_matrix(r)
            if exact:
                assert np.array_equal(F, o.rw_F), f"iter {it} run {r}: flux matrix differs"
            else:
                np.testing.assert_allclose(F, o.rw_F, rtol=RTOL, atol=0, err_msg=f"iter {it} run {r}")
            assert sim.rw_counts(r) == (o.rw_applied, o.rw_skipped), f"iter {it} run {r}"
            np.testing.assert_allclose(sim.flux(r), o.flux, rtol=RTOL, atol=0)
    return sim, ors


@pytest.mark.parametrize("n_bins,reset", [(100, False), (200, False), (100, True)])
def test_birth_death_reweighting_matches_oracle(n_bins, reset):
    """Unit bins from X = 10 (far from the stationary Poisson(40)); 100 bins
    keep the rate matrix in LDS, 200 bins put it in global memory; with
    reset, each event sees only the intervals since the previous one."""
    _say(f"case: reweighting, birth-death {n_bins} unit bins, M=4, period 5, reset {reset}, "
         "3 runs x 30 iterations")
    sim, ors = _run(_bd_unit(n_bins, [3, 4, 5]), period=5, n_iters=30, reset=reset)
    for r, o in enumerate(ors):
        assert o.rw_applied == 6 and o.rw_skipped == 0
        _, w, _, _ = sim.walkers(r)
        assert abs(w.sum() - 1.0) < 1e-12


def test_schlogl_recycling_reweighting_matches_oracle():
    """Schloegl with recycling X >= 563 -> X = 82: recycled walkers count as
    moving into the bin of X = 82.  Reweighting every 3 iterations."""
    _say("case: reweighting, Schloegl recycling, 60 bins M=4, period 3, 2 runs x 15 iterations")
    base = wl.schlogl_config(n_runs=2, seed0=21, n_iters=15)
    cfg = dataclasses.replace(base, m_targ=4)
    _run(cfg, period=3, n_iters=15)


def test_every_iteration_and_skipped_events():
    """Period 1: the event after iteration 0 has no flux yet (skipped), later
    ones apply; the counts match the oracle's."""
    _say("case: reweighting every iteration, birth-death 100 bins, 2 runs x 8 iterations")
    sim, ors = _run(_bd_unit(100, [8, 9], x0=40), period=1, n_iters=8)
    for r, o in enumerate(ors):
        assert o.rw_skipped >= 1
        assert sim.rw_counts(r) == (o.rw_applied, o.rw_skipped)


def test_graph_replay_equals_eager_with_reweighting():
    """Six iterations captured as a graph (events at iterations 1, 3, 5 with
    period 2), replayed three times with host work between replays: every
    replay leaves walkers and flux matrix identical to eager stepping."""
    _say("case: reweighting under hipGraph replay, birth-death 100 bins, period 2, 6 x 3")
    we = _we()
    cfg = _bd_unit(100, [5, 6])
    g = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=18, rw_period=2)
    e = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=18, rw_period=2)
    g.graph_capture(6)
    for rep in range(3):
        g.graph_replay(1)
        e.step(6)
        g.synchronize()
        for r in range(2):
            a, b = g.walkers(r), e.walkers(r)
            for u, v in zip(a, b):
                assert np.array_equal(np.asarray(u).view(np.uint8), np.asarray(v).view(np.uint8)), (rep, r)
            assert np.array_equal(g.rw_flux_matrix(r), e.rw_flux_matrix(r)), (rep, r)
            assert g.rw_counts(r) == e.rw_counts(r)
            assert sum(g.rw_counts(r)) == 3 * (rep + 1)


def test_reweighting_rejected_where_unsupported():
    we = _we()
    with pytest.raises(we.WEError):
        we.sim_from_config(_bd_unit(513, [1]), kernel=we.WE_KERNEL_LANE, rw_period=2)
    with pytest.raises(we.WEError):
        we.sim_from_config(_bd_unit(10, [1]), kernel=we.WE_KERNEL_LANE, rw_period=-1)
    sim = we.sim_from_config(_bd_unit(10, [1]), kernel=we.WE_KERNEL_LANE)
    with pytest.raises(we.WEError):
        sim.rw_flux_matrix(0)
