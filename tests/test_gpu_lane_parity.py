"""GPU parity of the lane-per-walker path against the CPU oracle.

The lane kernel computes the same FP64 operations in the same order as the
oracle and draws the same Philox blocks, so the integer trajectories, bins,
parent slots and weights must be IDENTICAL after every WE iteration; the
recycled-weight series too (summed in slot order on both sides).  The only
possible source of a difference is the waiting time (the kernel's own FP64
logarithm and Newton reciprocal against the host's log and division, an ulp
or two apart), which could flip an event only when t + dt lands within a few
ulps of tau; no such case is expected at these sizes and any occurrence fails
the test with the iteration and slot named.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1303_5986_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _we():
    from paper_1303_5986_amd import we
    return we


def _say(msg):
    print(msg, flush=True)


def _assert_same(it, r, sim_w, or_w):
    x, w, b, o = sim_w
    ox, ow, ob, oo = or_w
    assert len(w) == len(ow), f"iter {it} run {r}: {len(w)} walkers on GPU, {len(ow)} in oracle"
    bad = np.flatnonzero((x != ox).any(axis=1) | (w != ow) | (b != ob) | (o != oo))
    assert bad.size == 0, (
        f"iter {it} run {r}: first divergence at slot {bad[0]}: gpu x={x[bad[0]]} w={w[bad[0]]!r} "
        f"bin={b[bad[0]]} origin={o[bad[0]]}; oracle x={ox[bad[0]]} w={ow[bad[0]]!r} "
        f"bin={ob[bad[0]]} origin={oo[bad[0]]}")


def _run_parity(cfg, n_iters, check_runs, every=1, init=None, kernel=None):
    we = _we()
    kernel = we.WE_KERNEL_LANE if kernel is None else kernel
    sim = we.sim_from_config(cfg, kernel=kernel, max_iters=n_iters)
    ors = {}
    for r in check_runs:
        if init is not None:
            ix, iw = init(r)
            sim.set_ensemble(r, ix, iw)
            ors[r] = orc.OracleWE(cfg, int(cfg.seeds[r]), init_x=ix, init_w=iw)
        else:
            ors[r] = orc.OracleWE(cfg, int(cfg.seeds[r]))
    for it in range(n_iters):
        sim.step(1)
        for r in check_runs:
            ors[r].step(1)
        if (it + 1) % every == 0 or it == n_iters - 1:
            for r in check_runs:
                _assert_same(it, r, sim.walkers(r), ors[r].walkers())
    for r in check_runs:
        f = sim.flux(r)
        assert np.array_equal(f, np.array(ors[r].flux)), f"run {r}: flux series differs"
    return sim, ors


def test_birth_death_bit_identical_every_iteration():
    _say("case: birth-death, 4 runs x 60 iterations, lane kernel")
    cfg = wl.birth_death_config(n_runs=4, seed0=11, n_iters=60)
    sim, ors = _run_parity(cfg, 60, [0, 1, 2, 3])
    ev = sim.events_series()
    assert np.array_equal(ev, np.sum([o.events for o in ors.values()], axis=0))


def test_schlogl_recycling_bit_identical_every_iteration():
    _say("case: Schloegl with recycling, 3 runs x 150 iterations, lane kernel")
    cfg = wl.schlogl_config(n_runs=3, seed0=5, n_iters=150)
    _run_parity(cfg, 150, [0, 1, 2])


def test_schlogl_many_runs_sampled():
    """The launch shape of the benchmark (many runs in one launch): sampled
    runs are compared at the end of 120 iterations."""
    _say("case: Schloegl, 512 runs x 120 iterations, sampled runs 0/257/511")
    cfg = wl.schlogl_config(n_runs=512, seed0=1000, n_iters=120)
    _run_parity(cfg, 120, [0, 257, 511], every=40)


def test_futile_cycle_six_species_bit_identical():
    """Bimolecular reactions and six species (the 8-species/16-reaction
    register variant), 101 unit bins on S1 (Sec. III.A)."""
    _say("case: futile cycle, 2 runs x 40 iterations")
    net = wl.futile_cycle()
    cfg = wl.WEConfig(name="futile", net=net, x0=np.array([50, 50, 1, 1, 0, 0], np.int32),
                      bin_coef=np.array([1.0, 0, 0, 0, 0, 0]),
                      edges=np.arange(0.0, 102.0), m_targ=4, tau=1.0, n_iters=40,
                      seeds=np.array([3, 4], np.uint64))
    _run_parity(cfg, 40, [0, 1])


def test_weight_equalizing_rule_bit_identical():
    """The weight-equalizing split/merge (rule 1) on the paper's futile-cycle
    grid (101 unit bins on S1, 100 walkers per bin, bins above 64 walkers
    take the sorted-queue path) and on Schloegl with recycling (8 walkers per
    bin, one walker per lane): states, weights, bins, parents and flux equal
    the oracle's after every iteration."""
    _say("case: rule 1, futile cycle 2 runs x 30 iterations (M = 100)")
    cfg = wl.WEConfig(name="futile", net=wl.futile_cycle(),
                      x0=np.array([50, 50, 1, 1, 0, 0], np.int32),
                      bin_coef=np.array([1.0, 0, 0, 0, 0, 0]),
                      edges=np.arange(0.0, 102.0), m_targ=100, tau=1.0, n_iters=30,
                      seeds=np.array([601, 602], np.uint64), resample_rule=1)
    _run_parity(cfg, 30, [0, 1])
    _say("case: rule 1, Schloegl with recycling, 3 runs x 120 iterations")
    cfg = dataclasses.replace(wl.schlogl_config(n_runs=3, seed0=7, n_iters=120), resample_rule=1)
    _run_parity(cfg, 120, [0, 1, 2])


@pytest.mark.parametrize("S,R,seed", [(12, 30, 5), (24, 60, 6)])
def test_random_small_networks_bit_identical(S, R, seed):
    """Random mass-action networks that select the 16x32 and 32x64 register
    variants; ragged walker counts (5 bins x 3 walkers, 14 initial walkers)."""
    _say(f"case: random network S={S} R={R}")
    net = wl.random_network(seed, S, R, rate_lo=1e-2, rate_hi=1.0)
    rng = np.random.default_rng(seed)
    x0 = rng.integers(0, 30, size=S).astype(np.int32)
    coef = np.zeros(S)
    coef[0] = 1.0
    cfg = wl.WEConfig(name="rnd", net=net, x0=x0, bin_coef=coef, edges=np.array([0, 5, 10, 20, 40, 80.]),
                      m_targ=3, tau=0.2, n_iters=25, seeds=np.array([seed, seed + 1], np.uint64))

    def init(r):
        n = 14
        ix = np.tile(x0, (n, 1)) + rng.integers(0, 3, size=(n, S)).astype(np.int32)
        iw = np.full(n, 1.0 / n)
        return ix, iw

    _run_parity(cfg, 25, [0, 1], init=init)


def test_absorbing_network_goes_quiet():
    """X -> 0 only: every walker reaches the absorbing state and stops firing
    (a0 = 0 idles to tau)."""
    _say("case: absorbing decay network")
    net = wl.Network.from_reactions(["X"], [({"X": 1}, {}, 2.0)])
    cfg = wl.WEConfig(name="decay", net=net, x0=np.array([6], np.int32), bin_coef=np.array([1.0]),
                      edges=np.arange(0.0, 8.0), m_targ=2, tau=0.5, n_iters=30,
                      seeds=np.array([9], np.uint64))
    sim, ors = _run_parity(cfg, 30, [0])
    x, w, b, o = sim.walkers(0)
    assert (x == 0).all()
    assert sim.events_series()[-1] == 0


def test_histogram_and_mfpt_outputs():
    _say("case: histograms / MFPT outputs, Schloegl 4 runs x 80 iterations")
    cfg = wl.schlogl_config(n_runs=4, seed0=21, n_iters=80)
    we = _we()
    sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=80)
    ors = [orc.OracleWE(cfg, int(s)) for s in cfg.seeds]
    acc = np.zeros((4, cfg.hist_hi - cfg.hist_lo + 1))
    for it in range(80):
        sim.step(1)
        for r, o in enumerate(ors):
            o.step(1)
            acc[r] += o.histogram(0, cfg.hist_lo, cfg.hist_hi)
    h, n = sim.histogram_accum()
    assert n == 80
    np.testing.assert_allclose(h, acc, rtol=1e-12, atol=1e-300)
    for r, o in enumerate(ors):
        np.testing.assert_array_equal(sim.histogram(r, 0, 0, 800), o.histogram(0, 0, 800))
    mfpt, fm, fs = sim.mfpt(20)
    per_run = [np.mean(o.flux[20:]) / cfg.tau for o in ors]
    assert fm == pytest.approx(np.mean(per_run), rel=1e-12)
    ev, seg, its = sim.counters()
    assert its == 80
    assert ev == sum(sum(o.events) for o in ors)
    assert seg == sum(sum(o.segments) for o in ors)


def test_overflow_is_reported():
    """A pure birth process pushed past WE_COUNT_MAX: the kernel's own bounds
    check stops the walker and the next synchronous call reports it."""
    _say("case: overflow error path")
    we = _we()
    net = wl.Network.from_reactions(["X"], [({}, {"X": 1}, 1e6)])
    cfg = wl.WEConfig(name="boom", net=net, x0=np.array([130000], np.int32),
                      bin_coef=np.array([1.0]), edges=np.array([0.0, 1e9]), m_targ=1, tau=1.0,
                      n_iters=2, seeds=np.array([1], np.uint64))
    sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=2)
    sim.step(1)
    with pytest.raises(we.WEError) as ei:
        sim.synchronize()
    assert ei.value.status == we.WE_EOVERFLOW


def test_invalid_arguments_rejected():
    we = _we()
    net = we.Network(wl.schlogl())
    with pytest.raises(we.WEError):
        we.Sim(net, [1.0], [0.0, 0.0], tau=0.1, m_targ=2, seeds=[1], x0=[1], max_iters=1)
    with pytest.raises(we.WEError):
        we.Sim(net, [1.0], [0.0, 1.0], tau=-1.0, m_targ=2, seeds=[1], x0=[1], max_iters=1)
    sim = we.Sim(net, [1.0], [0.0, 1.0], tau=0.1, m_targ=2, seeds=[1], x0=[1], max_iters=1)
    sim.step(1)
    with pytest.raises(we.WEError):
        sim.step(1)                       # past max_iters


def test_graph_replay_matches_eager_and_oracle():
    """Four iterations captured as one HIP graph and replayed five times, with
    host work and synchronisation between replays: every replay leaves the
    ensemble identical to step-by-step launches and to the oracle."""
    _say("case: hipGraph replay, Schloegl 2 runs, 4 iterations x 5 replays")
    we = _we()
    cfg = wl.schlogl_config(n_runs=2, seed0=61, n_iters=20)
    g = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=20)
    e = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=20)
    ors = [orc.OracleWE(cfg, int(s)) for s in cfg.seeds]
    g.graph_capture(4)
    for rep in range(5):
        g.graph_replay(1)
        e.step(4)
        g.synchronize()
        for r in range(2):
            ors[r].step(4)
            gw = g.walkers(r)
            _assert_same(4 * rep + 3, r, gw, e.walkers(r))
            _assert_same(4 * rep + 3, r, gw, ors[r].walkers())
    for r in range(2):
        assert np.array_equal(g.flux(r), np.array(ors[r].flux))
    assert g.iterations == 20
    h1, n1 = g.histogram_accum()
    h2, n2 = e.histogram_accum()
    assert n1 == n2 == 20
    np.testing.assert_allclose(h1, h2, rtol=1e-12, atol=1e-300)


def test_joint_histogram_matches_ensembles():
    """The 3-species joint histogram accumulated on the device equals the sum
    over iterations of the oracle ensembles' weights per cell."""
    _say("case: joint histogram, futile cycle")
    we = _we()
    net = wl.futile_cycle()
    cfg = wl.WEConfig(name="futile", net=net, x0=np.array([50, 50, 1, 1, 0, 0], np.int32),
                      bin_coef=np.array([1.0, 0, 0, 0, 0, 0]), edges=np.arange(0.0, 102.0, 4.0),
                      m_targ=3, tau=1.0, n_iters=12, seeds=np.array([4], np.uint64))
    sim = we.Sim(we.Network(net), cfg.bin_coef, cfg.edges, tau=cfg.tau, m_targ=cfg.m_targ,
                 seeds=cfg.seeds, x0=cfg.x0, max_iters=12, kernel=we.WE_KERNEL_LANE,
                 joint_species=[0, 1, 4], joint_bins=8, joint_width=16)
    o = orc.OracleWE(cfg, 4)
    acc = np.zeros(8 ** 3)
    for it in range(12):
        sim.step(1)
        o.step(1)
        x, w, _, _ = o.walkers()
        for xi, wi in zip(x, w):
            c = [min(int(xi[s]) // 16, 7) for s in (0, 1, 4)]
            acc[c[0] + 8 * c[1] + 64 * c[2]] += wi
    np.testing.assert_allclose(sim.joint_histogram()[0], acc, rtol=1e-12, atol=1e-300)
