"""Batched runs of different networks: each member of a batch evolves exactly
as the same run stepped on its own (the persistent launch only changes which
wave carries which walker, never the arithmetic or the random numbers)."""
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


def _mixed_configs():
    sch = wl.schlogl_config(n_runs=2, seed0=31, n_iters=40)
    fut = wl.WEConfig(name="futile", net=wl.futile_cycle(), x0=np.array([50, 50, 1, 1, 0, 0], np.int32),
                      bin_coef=np.array([1.0, 0, 0, 0, 0, 0]), edges=np.arange(0.0, 102.0, 5.0),
                      m_targ=3, tau=1.0, n_iters=40, seeds=np.array([5], np.uint64))
    net = wl.random_network(11, 30, 200, rate_lo=1e-3, rate_hi=1.0)
    x0 = np.random.default_rng(11).integers(0, 20, size=30).astype(np.int32)
    coef = np.zeros(30)
    coef[1] = 1.0
    rnd = wl.WEConfig(name="rnd", net=net, x0=x0, bin_coef=coef,
                      edges=np.array([0, 2, 4, 8, 16, 32, 64.]), m_targ=4, tau=0.05, n_iters=40,
                      seeds=np.array([12, 19], np.uint64))
    return [sch, fut, rnd]


def _same(a, b):
    for r in range(a.n_runs):
        xa, wa, ba, oa = a.walkers(r)
        xb, wb, bb, ob = b.walkers(r)
        assert len(wa) == len(wb)
        assert np.array_equal(xa, xb) and np.array_equal(wa, wb)
        assert np.array_equal(ba, bb) and np.array_equal(oa, ob)
        assert np.array_equal(a.flux(r), b.flux(r))


def test_batch_members_equal_standalone_runs():
    print("case: batch of Schloegl (lane), futile (lane), random 30x200 (wave)", flush=True)
    we = _we()
    cfgs = _mixed_configs()
    kernels = [we.WE_KERNEL_LANE, we.WE_KERNEL_LANE, we.WE_KERNEL_WAVE]
    b = we.Batch(cfgs, max_iters=40, kernels=kernels)
    assert list(b.kernels()) == kernels
    b.step(25)
    for i, (c, k) in enumerate(zip(cfgs, kernels)):
        s = we.sim_from_config(c, kernel=k, max_iters=40)
        s.step(25)
        _same(b.members[i], s)
    # the lane members are also the oracle's runs
    o = orc.OracleWE(cfgs[0], int(cfgs[0].seeds[1]))
    o.step(25)
    x, w, _, _ = b.members[0].walkers(1)
    ox, ow, _, _ = o.walkers()
    assert np.array_equal(x, ox) and np.array_equal(w, ow)


def test_batch_graph_replay_equals_eager():
    print("case: batch hipGraph replay", flush=True)
    we = _we()
    cfgs = _mixed_configs()
    kernels = [we.WE_KERNEL_LANE, we.WE_KERNEL_LANE, we.WE_KERNEL_WAVE]
    g = we.Batch(cfgs, max_iters=40, kernels=kernels)
    e = we.Batch(cfgs, max_iters=40, kernels=kernels)
    g.graph_capture(6)
    for rep in range(4):
        g.graph_replay(1)
        e.step(6)
        g.synchronize()
        for i in range(3):
            _same(g.members[i], e.members[i])


def test_batch_autotune_writes_and_reuses_cache():
    print("case: batch autotune", flush=True)
    we = _we()
    cfgs = _mixed_configs()[:2]
    path = os.path.join(tempfile.mkdtemp(prefix="we_tune_"), "tune.json")
    b1 = we.Batch(cfgs, max_iters=10, autotune_iters=3, cache_path=path)
    k1 = b1.kernels()
    assert os.path.exists(path)
    text = open(path).read()
    assert "S1_R4" in text and "S6_R6" in text
    b2 = we.Batch(cfgs, max_iters=10, autotune_iters=3, cache_path=path)
    assert list(b2.kernels()) == list(k1)
    assert list(b2.walkers_per_wave()) == list(b1.walkers_per_wave())
    assert all(k in (we.WE_KERNEL_LANE, we.WE_KERNEL_GROUP, we.WE_KERNEL_WAVE) for k in k1)
    b2.step(4)
    b2.synchronize()


def test_uneven_batch_runs():
    """A 16-run slice of the uneven batch workload (8 to 3680 reactions,
    256 to 8192 walker slots) steps through a captured graph.  Every member's
    weights still sum to one, and every member the autotuner put on the lane
    kernel equals the oracle's run of the same configuration and seed, bit
    for bit (states, weights, bins, parents, flux)."""
    print("case: uneven batch, 16 runs", flush=True)
    we = _we()
    cfgs = wl.batch_configs(n_runs=16, n_iters=20)
    b = we.Batch(cfgs, max_iters=20)
    b.graph_capture(10)
    b.graph_replay(2)
    b.synchronize()
    kernels = list(b.kernels())
    n_lane = 0
    for c, m, k in zip(cfgs, b.members, kernels):
        x, w, bb, oo = m.walkers(0)
        assert abs(w.sum() - 1.0) < 1e-12
        assert (x >= 0).all()
        if k != we.WE_KERNEL_LANE:
            continue
        n_lane += 1
        o = orc.OracleWE(c, int(c.seeds[0]))
        o.step(20)
        ox, ow, ob, oo_ = o.walkers()
        print(f"   {c.name}: S={c.net.S} R={c.net.R}, {len(w)} walkers vs oracle", flush=True)
        assert len(w) == len(ow)
        assert np.array_equal(x, ox) and np.array_equal(w, ow)
        assert np.array_equal(bb, ob) and np.array_equal(oo, oo_)
        assert np.array_equal(m.flux(0), np.array(o.flux))
    assert n_lane >= 2


def test_batch_learned_bins_equal_standalone_runs():
    """Records and learned bins inside a batch.  Two toggle members (lane and
    wave kernel) record 30 eager iterations; their recorded ensembles equal
    a standalone run's.  Each member then trains its committor and switches
    to learned bins, and its checkpoint is loaded into a standalone sim.  The
    batch continues 10 eager iterations and 20 through a captured graph (the
    batched committor-bin launch), the standalone sims the same 30 on their
    own: states, weights, bins, parents and flux are equal bit for bit."""
    print("case: batch with records and learned bins (toggle lane + wave members)", flush=True)
    we = _we()
    base = wl.toggle_config(n_runs=2, n_bins=16, m_targ=4, n_iters=80)
    cfgs = [base, wl.toggle_config(seed0=100, n_runs=1, n_bins=16, m_targ=6, n_iters=80)]
    cfgs[1].seeds = np.array([77], np.uint64)
    kernels = [we.WE_KERNEL_LANE, we.WE_KERNEL_WAVE]
    b = we.Batch(cfgs, max_iters=80, kernels=kernels, record_iters=30)
    b.step(30)
    b.synchronize()
    s0 = we.sim_from_config(cfgs[0], kernel=kernels[0], max_iters=80, record_iters=30)
    s0.step(30)
    for it in (0, 17, 29):
        gn, gx, go, grc = b.members[0].record(it)
        sn, sx, so, src = s0.record(it)
        assert np.array_equal(gn, sn)
        for r in range(len(gn)):
            k = gn[r]
            assert np.array_equal(gx[r, :k], sx[r, :k]) and np.array_equal(go[r, :k], so[r, :k])
            assert np.array_equal(grc[r, :k], src[r, :k])
    tmp = tempfile.mkdtemp(prefix="we_bcm_")
    solo = []
    for i, (c, m) in enumerate(zip(cfgs, b.members)):
        loss, n = m.train_committor(c.bin_coef, c.a_thr, steps=120, batch=512, lr=2e-3, seed=4 + i,
                                    edge_mode=1)
        assert n > 0
        m.use_committor_bins(True)
        path = os.path.join(tmp, f"m{i}.ckpt")
        m.save(path)
        solo.append(we.Sim.load(b.networks[i], path))
    b.step(10)
    b.graph_capture(10)
    b.graph_replay(2)
    b.synchronize()
    for i, s in enumerate(solo):
        s.step(30)
        s.synchronize()
        _same(b.members[i], s)
        x, w, bb, _ = b.members[i].walkers(0)
        assert abs(w.sum() - 1.0) < 1e-12
    print(f"   members equal their standalone learned-bin runs after 30 iterations", flush=True)
