"""GPU parity of the group kernel (L lanes per walker, 64 / L walkers per
wave) against the CPU oracle, inside batches, and its place among the
autotuner's candidates.

The group kernel draws the same Philox blocks as the oracle and picks the
reaction in the same order (lane blocks follow the reactions' order); only
the summation order differs (per-lane partial sums, then a scan over the
group), so trajectories agree walker for walker except where u2 a0 or t + dt
lands within a few ulps of a boundary.  The tests allow 1% of walkers to
differ and say how many did.
"""
import json
import os
import tempfile

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


def _random_cfg(S, R, seed, m_targ=4, n_runs=2, tau=0.05, n_iters=20):
    net = wl.random_network(seed, S, R, rate_lo=1e-3, rate_hi=1.0)
    x0 = np.random.default_rng(seed).integers(0, 20, size=S).astype(np.int32)
    coef = np.zeros(S)
    coef[1] = 1.0
    return wl.WEConfig(name=f"rnd{S}x{R}", net=net, x0=x0, bin_coef=coef,
                       edges=np.array([0, 2, 4, 8, 16, 32, 64.]), m_targ=m_targ, tau=tau, n_iters=n_iters,
                       seeds=np.arange(seed, seed + n_runs, dtype=np.uint64))


def _compare(cfg, wpw, n_iters, max_frac=0.01, tables="lds"):
    """tables: 'regs' (descriptors and propensities of blocks of at most four
    reactions in registers), 'lds' (tables in LDS) or 'cache' (through the
    cache): the kernel variant the network and walkers per wave select."""
    we = _we()
    sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_GROUP, walkers_per_wave=wpw, max_iters=n_iters)
    suffix = {"regs": "true, 4", "regs8": "true, 8", "lds": "true, 0", "cache": "false, 0"}[tables]
    assert sim.propagation_kernel() == f"ssa_group_kernel<{64 // wpw}, {suffix}>"
    sim.step(n_iters)
    sim.synchronize()
    total = same = 0
    for r in range(len(cfg.seeds)):
        o = orc.OracleWE(cfg, int(cfg.seeds[r]))
        o.step(n_iters)
        x, w, b, _ = sim.walkers(r)
        ox, ow, ob, _ = o.walkers()
        assert abs(w.sum() - 1.0) < 1e-12
        assert (x >= 0).all()
        if len(w) == len(ow):
            eq = (x == ox).all(axis=1) & (w == ow)
            same += int(eq.sum())
        total += len(ow)
    frac = 1.0 - same / total
    _say(f"   walkers compared {total}, differing fraction {frac:.4f}")
    assert frac <= max_frac
    return sim


@pytest.mark.parametrize("wpw", [32, 16, 8, 4, 2])
def test_group_kernel_random_network_matches_oracle(wpw):
    _say(f"case: group kernel, {wpw} walkers per wave, random 30x200 network, 2 runs x 20 iterations")
    _compare(_random_cfg(30, 200, 17), wpw, 20, tables="regs8" if wpw == 2 else "lds")   # blocks of 7 on 32 lanes


@pytest.mark.parametrize("wpw", [8, 2])
def test_group_kernel_tables_through_the_cache_match_oracle(wpw):
    """A network whose descriptors and changes exceed the 48 KB LDS table
    budget (3200 reactions): the variant reading them through the cache."""
    _say(f"case: group kernel, {wpw} walkers per wave, random 300x3200 network (tables in global memory)")
    _compare(_random_cfg(300, 3200, 23, tau=0.002, n_iters=5), wpw, 5, tables="cache")


@pytest.mark.parametrize("wpw,tables", [(4, "regs"), (2, "regs"), (8, "regs8")])
def test_group_kernel_register_blocks_match_oracle(wpw, tables):
    """60 reactions on 16 or 32 lanes per walker (blocks of at most four
    reactions) or on 8 (blocks of 8): descriptors and propensities held in
    registers."""
    _say(f"case: group kernel, {wpw} walkers per wave, random 12x60 network (register blocks)")
    _compare(_random_cfg(12, 60, 29), wpw, 20, tables=tables)


@pytest.mark.parametrize("wpw", [32, 8])
def test_group_kernel_schlogl_with_recycling_matches_oracle(wpw):
    """Four reactions on up to 32 lanes (most lanes' blocks are empty), with
    recycling: the flux series equal the oracle's (at most two intervals of
    a run may differ, where a walker did)."""
    _say(f"case: group kernel, {wpw} walkers per wave, Schloegl with recycling, 3 runs x 40 iterations")
    cfg = wl.schlogl_config(n_runs=3, seed0=5, n_iters=40)
    sim = _compare(cfg, wpw, 40, tables="regs")
    for r in range(3):
        o = orc.OracleWE(cfg, int(cfg.seeds[r]))
        o.step(40)
        f, fo = sim.flux(r), np.array(o.flux)
        assert np.sum(f != fo) <= 2, (r, np.flatnonzero(f != fo))


def test_group_kernel_is_deterministic_and_rejects_bad_shapes():
    we = _we()
    cfg = _random_cfg(12, 60, 3)
    a = we.sim_from_config(cfg, kernel=we.WE_KERNEL_GROUP, walkers_per_wave=16, max_iters=10)
    b = we.sim_from_config(cfg, kernel=we.WE_KERNEL_GROUP, walkers_per_wave=16, max_iters=10)
    a.step(10)
    b.step(10)
    for r in range(2):
        xa, wa, _, _ = a.walkers(r)
        xb, wb, _, _ = b.walkers(r)
        assert np.array_equal(xa, xb) and np.array_equal(wa, wb)
    with pytest.raises(we.WEError):
        we.sim_from_config(cfg, kernel=we.WE_KERNEL_GROUP, walkers_per_wave=3, max_iters=10)
    big = _random_cfg(200, 400, 5)
    with pytest.raises(we.WEError):     # 32 walkers x 200 species > 4096 counts per wave
        we.sim_from_config(big, kernel=we.WE_KERNEL_GROUP, walkers_per_wave=32, max_iters=10)


def test_batch_group_members_equal_standalone_runs():
    """Group members inside a batch (8 and 32 walkers per wave) next to a lane
    member: every member equals the same configuration stepped on its own,
    bit for bit, through eager steps and a captured graph."""
    _say("case: batch with group members (8, 32 walkers per wave) and a lane member")
    we = _we()
    cfgs = [_random_cfg(30, 200, 21), _random_cfg(10, 90, 23, m_targ=6),
            wl.schlogl_config(n_runs=2, seed0=41, n_iters=40)]
    kernels = [(we.WE_KERNEL_GROUP, 8), (we.WE_KERNEL_GROUP, 32), we.WE_KERNEL_LANE]
    b = we.Batch(cfgs, max_iters=30, kernels=kernels)
    assert list(b.walkers_per_wave()) == [8, 32, 64]
    b.step(10)
    b.graph_capture(10)
    b.graph_replay(2)
    b.synchronize()
    for c, k, m in zip(cfgs, kernels, b.members):
        kern, wpw = k if isinstance(k, tuple) else (k, 0)
        s = we.sim_from_config(c, kernel=kern, walkers_per_wave=wpw, max_iters=30)
        s.step(30)
        s.synchronize()
        for r in range(len(c.seeds)):
            xa, wa, ba, oa = m.walkers(r)
            xb, wb, bb, ob = s.walkers(r)
            assert np.array_equal(xa, xb) and np.array_equal(wa, wb)
            assert np.array_equal(ba, bb) and np.array_equal(oa, ob)
            assert np.array_equal(m.flux(r), s.flux(r))


def test_autotuner_times_group_variants():
    """The autotuner's candidates for a 40 x 400 network are the five group
    variants and the wave kernel (no lane kernel: too many reactions); its
    choice is cached as kernel + 16 x walkers per wave and reused."""
    _say("case: autotune over group and wave variants, random 40x400 network")
    we = _we()
    cfgs = [_random_cfg(40, 400, 31, m_targ=16)]
    path = os.path.join(tempfile.mkdtemp(prefix="we_tune_"), "tune.json")
    b = we.Batch(cfgs, max_iters=10, autotune_iters=2, cache_path=path)
    k, w = int(b.kernels()[0]), int(b.walkers_per_wave()[0])
    cache = json.load(open(path))
    (val,) = cache.values()
    assert k in (we.WE_KERNEL_GROUP, we.WE_KERNEL_WAVE)
    assert val == k + 16 * (w if k == we.WE_KERNEL_GROUP else 0)
    _say(f"   chose kernel {k}, {w} walkers per wave")
    b.step(4)
    b.synchronize()
    b2 = we.Batch(cfgs, max_iters=10, autotune_iters=2, cache_path=path)
    assert int(b2.kernels()[0]) == k and int(b2.walkers_per_wave()[0]) == w


def test_autotune_helper_and_walker_events():
    """we.autotune returns a kernel the configuration runs on; the per-walker
    event counts of an interval sum to the interval's events (run 0) and
    cover every walker propagated."""
    we = _we()
    cfg = wl.toggle_config(n_runs=2, n_bins=16, m_targ=8, n_iters=10)
    k, w = we.autotune(cfg, iters=2)
    assert k in (we.WE_KERNEL_LANE, we.WE_KERNEL_GROUP, we.WE_KERNEL_WAVE)
    assert (w in (2, 4, 8, 16, 32)) if k == we.WE_KERNEL_GROUP else w == 0
    sim = we.sim_from_config(cfg, kernel=k, walkers_per_wave=w, max_iters=10)
    sim.step(3)
    sim.synchronize()
    n_prev = len(sim.walkers(0)[1])
    sim.step(1)
    sim.synchronize()
    ev = sim.walker_events(0)
    assert len(ev) == n_prev
    per_run = sim.counters()[0]
    total = sum(int(sim.walker_events(r).sum()) for r in range(2))
    assert total == int(sim.events_series(3, 1)[0])
    assert per_run >= total


def test_measured_peaks_are_plausible():
    """The ceilings measured on the device lie within a factor of two of the
    datasheet figures the rooflines use (HBM 8 TB/s, LDS 78.6 TB/s, FP64
    78.6 TFLOP/s, int32 lane operations 39.3e12/s at 2.4 GHz)."""
    we = _we()
    pk = we.measure_peaks()
    _say(f"   measured {pk}")
    assert pk["compute_units"] >= 1
    assert 1000 < pk["hbm_gbs"] < 16000
    assert 39 < pk["lds_tbs"] < 160
    assert 39 < pk["fp64_tflops"] < 160
    assert 19 < pk["int32_tops"] < 80
