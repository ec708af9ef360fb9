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
    assert all(k in (we.WE_KERNEL_LANE, we.WE_KERNEL_WAVE) for k in k1)
    b2.step(4)
    b2.synchronize()


def test_uneven_batch_runs():
    """A 16-run slice of the uneven batch workload (8 to 3680 reactions,
    256 to 8192 walker slots) steps through a captured graph; every member's
    weights still sum to one."""
    print("case: uneven batch, 16 runs", flush=True)
    we = _we()
    cfgs = wl.batch_configs(n_runs=16, n_iters=20)
    b = we.Batch(cfgs, max_iters=20)
    b.graph_capture(10)
    b.graph_replay(2)
    b.synchronize()
    for m in b.members:
        x, w, _, _ = m.walkers(0)
        assert abs(w.sum() - 1.0) < 1e-12
        assert (x >= 0).all()
