"""Checkpoints and bin switching through the C ABI (we_save / we_load /
we_set_bins).

* save -> load -> continue equals the uninterrupted run bit for bit: the lane
  kernel with recycling, steady-state reweighting and the weight-equalizing
  rule; the wave kernel; and learned committor bins (model, Adam moments,
  features and edges restored).
* a checkpoint refuses a different network, and its header reports the sizes.
* we_set_bins with a new grid continues exactly as the oracle does when it
  is handed the same ensemble and the new grid at that iteration, and with
  no grid returns from learned to grid bins.
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


def _same_sims(a, b, runs):
    for r in range(runs):
        for u, v in zip(a.walkers(r), b.walkers(r)):
            assert np.array_equal(u, v), r
        assert np.array_equal(a.flux(r), b.flux(r)), r
    assert a.counters() == b.counters()
    assert np.array_equal(a.events_series(), b.events_series())


def test_lane_checkpoint_resumes_bit_identically(tmp_path):
    we = _we()
    _say("case: checkpoint, Schloegl with recycling, RW-5, rule 1, 3 runs, save at 17 of 30")
    cfg = dataclasses.replace(wl.schlogl_config(n_runs=3, seed0=21, n_iters=30), resample_rule=1)
    a = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=30, rw_period=5)
    ref = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=30, rw_period=5)
    a.step(17)
    path = str(tmp_path / "schlogl.ckpt")
    a.save(path)
    info = we.checkpoint_info(path)
    assert (info.iteration, info.n_runs, info.n_bins, info.m_targ) == (17, 3, cfg.n_bins, cfg.m_targ)
    a.step(5)                                  # the saved sim moves on; the file does not
    b = we.Sim.load(we.Network(cfg.net), path)
    b.step(13)
    ref.step(30)
    _same_sims(b, ref, 3)
    for r in range(3):
        assert np.array_equal(b.rw_flux_matrix(r), ref.rw_flux_matrix(r))
    # and the loaded run still equals the oracle
    o = orc.OracleWE(cfg, int(cfg.seeds[1]), rw_period=5)
    o.step(30)
    ox, ow, ob, oo = o.walkers()
    bx, bw, bb, bo = b.walkers(1)
    assert np.array_equal(bx, ox) and np.array_equal(bb, ob) and np.array_equal(bo, oo)
    assert np.allclose(bw, ow, rtol=1e-9, atol=0)


def test_wave_checkpoint_resumes_bit_identically(tmp_path):
    we = _we()
    _say("case: checkpoint, wave kernel, random 40 x 300 network, save at 6 of 12")
    net = wl.random_network(77, 40, 300, rate_lo=1e-3, rate_hi=1.0)
    x0 = np.random.default_rng(77).integers(0, 20, size=40).astype(np.int32)
    coef = np.zeros(40)
    coef[1] = 1.0
    cfg = wl.WEConfig(name="rnd", net=net, x0=x0, bin_coef=coef,
                      edges=np.array([0, 2, 4, 8, 16, 32, 64.]), m_targ=4, tau=0.05, n_iters=12,
                      seeds=np.array([77, 84], np.uint64))
    a = we.sim_from_config(cfg, kernel=we.WE_KERNEL_WAVE, max_iters=12)
    ref = we.sim_from_config(cfg, kernel=we.WE_KERNEL_WAVE, max_iters=12)
    a.step(6)
    path = str(tmp_path / "wave.ckpt")
    a.save(path)
    b = we.Sim.load(we.Network(cfg.net), path)
    b.step(6)
    ref.step(12)
    _same_sims(b, ref, 2)


def test_learned_bins_checkpoint_resumes_bit_identically(tmp_path):
    we = _we()
    _say("case: checkpoint with a trained committor and learned bins (toggle)")
    cfg = wl.toggle_config(n_runs=2, n_iters=80)
    a = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=80, record_iters=40)
    a.step(40)
    a.train_committor(cfg.bin_coef, cfg.a_thr, steps=200, batch=1024, lr=2e-3, seed=5)
    a.use_committor_bins(True)
    a.step(10)
    path = str(tmp_path / "toggle.ckpt")
    a.save(path)
    b = we.Sim.load(we.Network(cfg.net), path)
    pa, fa, ea = a.committor_state()
    pb, fb, eb = b.committor_state()
    assert np.array_equal(pa, pb) and np.array_equal(fa, fb) and np.array_equal(ea, eb)
    a.step(20)
    b.step(20)
    _same_sims(a, b, 2)


def test_checkpoint_refuses_another_network(tmp_path):
    we = _we()
    cfg = wl.birth_death_config(n_runs=1, n_iters=5)
    a = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=5)
    a.step(2)
    path = str(tmp_path / "bd.ckpt")
    a.save(path)
    other = wl.birth_death(k=1.5)
    with pytest.raises(we.WEError) as e:
        we.Sim.load(we.Network(other), path)
    assert e.value.status == we.WE_EINVAL
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(b"not a checkpoint" * 8)
    with pytest.raises(we.WEError):
        we.checkpoint_info(str(bad))


def test_set_bins_new_grid_follows_the_oracle():
    we = _we()
    _say("case: we_set_bins, Schloegl 60 -> 60 bins on a shifted grid at iteration 12")
    cfg = wl.schlogl_config(n_runs=2, seed0=31, n_iters=30)
    cfg2 = dataclasses.replace(cfg, edges=wl.uniform_edges(-7.0, 793.0, cfg.n_bins))
    sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=30)
    sim.step(12)
    snap = [sim.walkers(r) for r in range(2)]
    sim.set_grid_bins(cfg2.bin_coef, cfg2.edges)
    sim.step(10)
    for r in range(2):
        x, w, b, o = snap[r]
        ora = orc.OracleWE(cfg2, int(cfg.seeds[r]), init_x=x, init_w=w)
        ora.iter = 12
        ora.step(10)
        for u, v in zip(sim.walkers(r), ora.walkers()):
            assert np.array_equal(u, v), r
    with pytest.raises(we.WEError):
        sim.set_grid_bins(cfg.bin_coef, wl.uniform_edges(0.0, 800.0, cfg.n_bins + 1))
    with pytest.raises(we.WEError):
        sim.set_learned_bins()                 # no trained committor
