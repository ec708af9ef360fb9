"""GPU parity of the wave-per-walker path against the CPU oracle.

Three kernels implement the path: the factored-table kernel (every table in
LDS) runs when all live walkers get a wave at once, the descriptor-table
kernel otherwise, and the latter's header-table variant when a network does
not fit the factored format; each is driven below.

The wave kernel draws the same Philox blocks as the oracle but sums
propensities in chunks (two wave-level prefix scans, incremental chunk sums)
instead of sequentially, so a0 and the running sums may differ in the last
bits.  An event can only change when u2*a0 or t+dt lands within a few ulps of
a boundary, so trajectories are expected to agree walker for walker; the
tests allow a small fraction of differing walkers (and say how many) and
back this with distribution-level checks (chi-square p > 0.01, as the wave
path's agreement is statistical by construction).
"""
import numpy as np
import pytest
from scipy import stats

from oracle import oracle as orc
from paper_1303_5986_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _we():
    from paper_1303_5986_amd import we
    return we


def _say(msg):
    print(msg, flush=True)


def _compare(cfg, n_iters, runs, kernel, init=None, max_frac=0.01):
    we = _we()
    sim = we.sim_from_config(cfg, kernel=kernel, max_iters=n_iters)
    ors = {}
    for r in runs:
        if init is not None:
            ix, iw = init(r)
            sim.set_ensemble(r, ix, iw)
            ors[r] = orc.OracleWE(cfg, int(cfg.seeds[r]), init_x=ix, init_w=iw)
        else:
            ors[r] = orc.OracleWE(cfg, int(cfg.seeds[r]))
    sim.step(n_iters)
    sim.synchronize()
    total = same = 0
    for r in runs:
        ors[r].step(n_iters)
        x, w, b, o = sim.walkers(r)
        ox, ow, ob, oo = ors[r].walkers()
        assert abs(w.sum() - 1.0) < 1e-12
        if len(w) == len(ow):
            eq = (x == ox).all(axis=1) & (w == ow)
            same += int(eq.sum())
        total += len(ow)
    frac_diff = 1.0 - same / total
    _say(f"   walkers compared {total}, differing fraction {frac_diff:.4f}")
    assert frac_diff <= max_frac
    return sim, ors


def test_wave_schlogl_matches_oracle():
    _say("case: wave kernel, Schloegl 3 runs x 60 iterations")
    cfg = wl.schlogl_config(n_runs=3, seed0=40, n_iters=60)
    _compare(cfg, 60, [0, 1, 2], _we().WE_KERNEL_WAVE)


@pytest.mark.parametrize("S,R,seed", [(30, 200, 11), (100, 700, 12)])
def test_wave_random_networks_match_oracle(S, R, seed):
    """Several chunks of 64 reactions; dependency lists over one round."""
    _say(f"case: wave kernel, random network S={S} R={R}")
    net = wl.random_network(seed, S, R, rate_lo=1e-3, rate_hi=1.0)
    rng = np.random.default_rng(seed)
    x0 = rng.integers(0, 20, size=S).astype(np.int32)
    coef = np.zeros(S)
    coef[1] = 1.0
    cfg = wl.WEConfig(name="rnd", net=net, x0=x0, bin_coef=coef,
                      edges=np.array([0, 2, 4, 8, 16, 32, 64.]), m_targ=4, tau=0.05, n_iters=12,
                      seeds=np.array([seed, seed + 7], np.uint64))
    _compare(cfg, 12, [0, 1], _we().WE_KERNEL_WAVE)


def test_wave_long_dependency_lists():
    """A hub species used by 300 reactions: firing its inflow changes more
    propensities than the incremental path holds (2 x 64), which takes the
    rebuild-all-chunks path."""
    _say("case: wave kernel, hub network (dependency list of 300)")
    names = ["hub"] + [f"s{i}" for i in range(1, 301)]
    rx = [({}, {"hub": 1}, 50.0)]
    for i in range(1, 301):
        rx.append(({"hub": 1, f"s{i}": 1}, {f"s{i}": 1}, 0.01))   # hub consumed, s_i catalyst
        rx.append(({}, {f"s{i}": 1}, 0.5))
        rx.append(({f"s{i}": 1}, {}, 0.1))
    net = wl.Network.from_reactions(names, rx)
    x0 = np.full(301, 3, np.int32)
    x0[0] = 20
    coef = np.zeros(301)
    coef[0] = 1.0
    cfg = wl.WEConfig(name="hub", net=net, x0=x0, bin_coef=coef, edges=np.arange(0.0, 65.0, 8.0),
                      m_targ=3, tau=0.05, n_iters=8, seeds=np.array([5], np.uint64))
    _compare(cfg, 8, [0], _we().WE_KERNEL_WAVE)


def test_wave_large_network_relaxed_start():
    """The 354-species / 3680-reaction network (from its seed), started from a
    state with small counts so the oracle finishes in seconds."""
    _say("case: wave kernel, 354/3680 network, small-count start")
    base = wl.large_network_config()
    x0 = np.minimum(base.x0, 12).astype(np.int32)
    coef = base.bin_coef
    cfg = wl.WEConfig(name="large_small", net=base.net, x0=x0, bin_coef=coef,
                      edges=np.arange(0.0, 25.0, 2.0), m_targ=2, tau=0.01, n_iters=6,
                      seeds=np.array([77], np.uint64))
    _compare(cfg, 6, [0], _we().WE_KERNEL_WAVE)


def test_wave_agrees_with_lane_kernel():
    """Where both kernels run (R <= 64) they give the same ensembles."""
    _say("case: wave vs lane, futile cycle")
    we = _we()
    net = wl.futile_cycle()
    cfg = wl.WEConfig(name="futile", net=net, x0=np.array([50, 50, 1, 1, 0, 0], np.int32),
                      bin_coef=np.array([1.0, 0, 0, 0, 0, 0]), edges=np.arange(0.0, 102.0),
                      m_targ=4, tau=1.0, n_iters=30, seeds=np.array([8, 9], np.uint64))
    a = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=30)
    b = we.sim_from_config(cfg, kernel=we.WE_KERNEL_WAVE, max_iters=30)
    a.step(30)
    b.step(30)
    for r in range(2):
        xa, wa, _, _ = a.walkers(r)
        xb, wb, _, _ = b.walkers(r)
        assert len(wa) == len(wb)
        assert np.mean((xa == xb).all(axis=1) & (wa == wb)) >= 0.99


def test_wave_single_bin_matches_brute_force_distribution():
    """One bin holding all M walkers is M independent SSA trajectories: the
    wave kernel's histogram of a species of the large network after 5
    intervals matches the oracle's brute-force SSA ensemble (two-sample
    chi-square, p > 0.01) -- a distribution-level check that does not rely on
    shared random numbers (the oracle runs use other seeds)."""
    _say("case: wave kernel single bin vs oracle brute force, 354/3680 network")
    we = _we()
    base = wl.large_network_config()
    x0 = np.minimum(base.x0, 10).astype(np.int32)
    sp = int(np.argmax(base.bin_coef))
    M = 1024
    cfg = wl.WEConfig(name="bf", net=base.net, x0=x0, bin_coef=base.bin_coef,
                      edges=np.array([-1e9, 1e9]), m_targ=M, tau=0.01, n_iters=5,
                      seeds=np.array([123], np.uint64))
    sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_WAVE, max_iters=5)
    sim.step(5)
    x, w, _, _ = sim.walkers(0)
    gpu = x[:, sp]
    onet = orc.OracleNet(base.net)
    cpu = []
    for k in range(300):
        y = x0.copy()
        for it in range(5):
            y, _ = orc.ssa_interval(onet, y, 0.01, 999, k, it)
        cpu.append(y[sp])
    cpu = np.array(cpu)
    lo, hi = min(gpu.min(), cpu.min()), max(gpu.max(), cpu.max())
    edges = np.arange(lo, hi + 2)
    hg = np.histogram(gpu, edges)[0]
    hc = np.histogram(cpu, edges)[0]
    keep = (hg + hc) >= 5
    tab = np.vstack([np.append(hg[keep], hg[~keep].sum()), np.append(hc[keep], hc[~keep].sum())])
    tab = tab[:, tab.sum(axis=0) > 0]
    p = stats.chi2_contingency(tab)[1] if tab.shape[1] > 1 else 1.0
    _say(f"   two-sample chi-square p = {p:.3f}")
    assert p > 0.01


def test_descriptor_table_kernel_many_walkers():
    """More walkers than the factored kernel holds at once (8 runs x 1536
    slots of a 100 x 700 network), which takes the descriptor-table kernel
    with descriptors alone in LDS and the dependency lists from global
    memory (two blocks per CU)."""
    _say("case: wave kernel, 8 runs x 1536 slots, random 100x700 network (descriptor-table kernel)")
    net = wl.random_network(13, 100, 700, rate_lo=1e-3, rate_hi=1.0)
    rng = np.random.default_rng(13)
    x0 = rng.integers(0, 20, size=100).astype(np.int32)
    coef = np.zeros(100)
    coef[1] = 1.0
    cfg = wl.WEConfig(name="rnd_many", net=net, x0=x0, bin_coef=coef,
                      edges=np.array([0, 2, 4, 8, 16, 32, 64.]), m_targ=256, tau=0.05, n_iters=8,
                      seeds=np.arange(31, 39, dtype=np.uint64))
    assert cfg.cap * len(cfg.seeds) // 2 > 16 * 256
    _compare(cfg, 8, [0, 5], _we().WE_KERNEL_WAVE)


def test_header_table_kernel_for_networks_outside_the_factored_format():
    """A reaction changing five species does not fit the factored format
    (at most four changes per reaction), so this network runs on the
    descriptor-table kernel with the reaction headers in LDS."""
    _say("case: wave kernel, five-change reaction (header-table kernel)")
    names = ["A", "B", "C", "D", "E", "F"]
    rx = [({}, {"A": 1}, 3.0), ({"A": 1}, {"B": 1, "C": 1, "D": 1, "E": 1, "F": 1}, 0.5)]
    for n in names[1:]:
        rx.append(({n: 1}, {}, 0.4))
        rx.append(({n: 2}, {"A": 1}, 0.02))
    net = wl.Network.from_reactions(names, rx)
    coef = np.zeros(6)
    coef[2] = 1.0
    cfg = wl.WEConfig(name="five", net=net, x0=np.array([5, 3, 3, 3, 3, 3], np.int32), bin_coef=coef,
                      edges=np.arange(0.0, 21.0, 2.0), m_targ=6, tau=0.2, n_iters=20,
                      seeds=np.array([4, 5], np.uint64))
    _compare(cfg, 20, [0, 1], _we().WE_KERNEL_WAVE)


def test_wave_large_network_from_its_own_initial_state():
    """The large workload itself at its own start: x0 log-uniform on [0, 1000]
    (a0 about 2e7 per unit time), on a reduced budget (tau = 5e-6, four
    intervals, about 100 events per walker per interval).  Walker by walker
    the wave kernel follows the oracle (the same random numbers), and its
    histogram of the binned species over 1024 independent trajectories (one
    bin) matches an oracle brute-force ensemble on other seeds (two-sample
    chi-square p > 0.01) for two species."""
    _say("case: wave kernel, 354/3680 network from its own x0, tau 5e-6")
    we = _we()
    base = wl.large_network_config()
    cfg = wl.WEConfig(name="large_x0", net=base.net, x0=base.x0, bin_coef=base.bin_coef,
                      edges=np.array([-1e9, 1e9]), m_targ=32, tau=5e-6, n_iters=4,
                      seeds=np.array([321], np.uint64))
    _compare(cfg, 4, [0], _we().WE_KERNEL_WAVE, max_frac=0.05)
    big = wl.WEConfig(name="large_x0_bf", net=base.net, x0=base.x0, bin_coef=base.bin_coef,
                      edges=np.array([-1e9, 1e9]), m_targ=1024, tau=5e-6, n_iters=4,
                      seeds=np.array([654], np.uint64))
    sim = we.sim_from_config(big, kernel=we.WE_KERNEL_WAVE, max_iters=4)
    sim.step(4)
    x, _, _, _ = sim.walkers(0)
    onet = orc.OracleNet(base.net)
    cpu = []
    for k in range(200):
        y = base.x0.copy()
        for it in range(4):
            y, _ = orc.ssa_interval(onet, y, 5e-6, 777, k, it)
        cpu.append(y)
    cpu = np.array(cpu)
    sp = int(np.argmax(base.bin_coef))
    busiest = int(np.argmax(np.abs(x - base.x0).mean(axis=0)))   # the species that moved most
    for s in (sp, busiest):
        g, c = x[:, s], cpu[:, s]
        edges = np.arange(min(g.min(), c.min()), max(g.max(), c.max()) + 2)
        hg, hc = np.histogram(g, edges)[0], np.histogram(c, edges)[0]
        keep = (hg + hc) >= 5
        tab = np.vstack([np.append(hg[keep], hg[~keep].sum()), np.append(hc[keep], hc[~keep].sum())])
        tab = tab[:, tab.sum(axis=0) > 0]
        p = stats.chi2_contingency(tab)[1] if tab.shape[1] > 1 else 1.0
        _say(f"   species {s}: two-sample chi-square p = {p:.3f} over {tab.shape[1]} cells")
        assert p > 0.01


def _run_twice(cfg, n_iters, kernel_expected):
    we = _we()
    out = []
    for _ in range(2):
        sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_WAVE, max_iters=n_iters)
        assert sim.propagation_kernel() == kernel_expected
        sim.step(n_iters)
        sim.synchronize()
        out.append(([sim.walkers(r) for r in range(len(cfg.seeds))], sim.counters()))
    (wa, ca), (wb, cb) = out
    assert ca == cb
    for (xa, wta, ba, oa), (xb, wtb, bb, ob) in zip(wa, wb):
        assert np.array_equal(xa, xb) and np.array_equal(wta, wtb)
        assert np.array_equal(ba, bb) and np.array_equal(oa, ob)


def test_wave_kernels_repeat_bit_for_bit():
    """The chunk sums take each dependent's propensity change by an LDS
    atomic add, whose same-address lanes the LDS unit applies in a fixed
    order: two runs of the same configuration end with identical walkers,
    weights and counters, on the factored-table kernel (the 354/3680
    network from its own start) and on the descriptor-table kernel."""
    _say("case: wave kernels run twice, factored (354/3680, 12 intervals) and descriptor-table")
    base = wl.large_network_config(n_iters=12)
    _run_twice(base, 12, "ssa_wave_fact_kernel")
    net = wl.random_network(13, 100, 700, rate_lo=1e-3, rate_hi=1.0)
    rng = np.random.default_rng(13)
    x0 = rng.integers(0, 20, size=100).astype(np.int32)
    coef = np.zeros(100)
    coef[1] = 1.0
    cfg = wl.WEConfig(name="rnd_many", net=net, x0=x0, bin_coef=coef,
                      edges=np.array([0, 2, 4, 8, 16, 32, 64.]), m_targ=256, tau=0.05, n_iters=8,
                      seeds=np.arange(31, 39, dtype=np.uint64))
    _run_twice(cfg, 8, "ssa_wave_lds_kernel<false>")
