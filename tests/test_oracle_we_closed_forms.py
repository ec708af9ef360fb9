"""Whole-WE estimates of the oracle against closed forms (-m "not gpu").

WE is an unbiased estimator, not an exact algorithm (Sec. II.B), so these
pins run independent replicas (the paper's practice, Sec. III) and compare
their mean with the exact law, in units of the standard error over
replicas.  All use the weight-equalizing split/merge (resample_rule 1):

* birth-death (0 -> X at 1, X -> 0 at 0.025 X; stationary Poisson(40)):
  the bulk of P(X, t = 200) on the 20-bin, 4-walker grid against the exact
  transient law, and the tail P(X >= 100) = 1.2e-15 on unit bins against
  Poisson(40) at 10%.  On the 20-bin grid, whose bins are 6 copies wide,
  four walkers per bin reach the bins beyond X ~ 80 too rarely for a tail
  estimate (one replica in 2048 carries the mean of P(X >= 96)); unit bins
  are the paper's own grid for tails (Secs. III.A, III.B).
* Schloegl (Sec. III.B, Eq. schlogl): the MFPT from the low to the high
  well, tau / mean recycled weight (Eq. mfpt), against the exact chain
  formula 5.03e4 s (the paper: about 5e4); and, without recycling and
  started from the two wells with their exact weights, the time-averaged
  stationary law against pi across 14 decades.
"""
import dataclasses
import multiprocessing as mp

import numpy as np

import closed_form as cf
from oracle import oracle as orc
from paper_1303_5986_amd import workloads as wl


def _pool_map(fn, items):
    ctx = mp.get_context("fork")
    with ctx.Pool(min(8, len(items))) as p:
        return p.map(fn, items)


def _bd_unit_tail(seed):
    cfg = dataclasses.replace(wl.birth_death_config(n_runs=1, seed0=seed, n_iters=600),
                              edges=np.arange(0.0, 122.0), m_targ=16, resample_rule=1)
    o = orc.OracleWE(cfg, seed)
    acc = 0.0
    for it in range(600):
        o.step(1)
        if it >= 200:                       # P(X >= 100, t) is 0.998 of stationary at t = 200
            x, w, _, _ = o.walkers()
            acc += w[x[:, 0] >= 100].sum()
    return acc / 400


def test_birth_death_we_tail_matches_poisson():
    exact = cf.poisson_sf(40.0, 100)
    assert abs(exact / 1.2063e-15 - 1) < 1e-3
    est = np.array(_pool_map(_bd_unit_tail, list(range(1, 33))))
    mean, sem = est.mean(), est.std(ddof=1) / np.sqrt(len(est))
    print(f"P(X>=100): WE {mean:.4e} +- {sem:.1e}, Poisson(40) {exact:.4e}")
    assert abs(mean - exact) < 3 * sem
    assert abs(mean / exact - 1) < 0.10


def _bd_grid_bins(seed):
    cfg = dataclasses.replace(wl.birth_death_config(n_runs=1, seed0=seed, n_iters=200), resample_rule=1)
    o = orc.OracleWE(cfg, seed)
    o.step(200)
    x, w, b, _ = o.walkers()
    return np.bincount(b, weights=w, minlength=20)


def test_birth_death_we_bulk_on_the_twenty_bin_grid():
    H = np.array(_pool_map(_bd_grid_bins, list(range(1, 513))))
    tr = cf.bd_transient_pmf(40, 1.0, 0.025, 200.0, 200)
    exact = np.array([tr[6 * k:6 * k + 6].sum() for k in range(20)])
    mean, sem = H.mean(0), H.std(0, ddof=1) / np.sqrt(len(H))
    bulk = exact > 1e-3
    assert bulk.sum() >= 7
    z = (mean[bulk] - exact[bulk]) / sem[bulk]
    assert np.all(np.abs(z) < 4), z
    core = exact > 1e-2                     # where 512 replicas resolve a bin to a few per cent
    assert np.all(np.abs(mean[core] / exact[core] - 1) < 0.10)


def _schlogl_flux(seed):
    cfg = dataclasses.replace(wl.schlogl_config(n_runs=1, seed0=seed, n_iters=1000), resample_rule=1)
    o = orc.OracleWE(cfg, seed)
    o.step(1000)
    return np.mean(o.flux[200:]) / cfg.tau


def test_schlogl_we_mfpt_matches_chain_formula():
    lam, mu = cf.schlogl_rates(1000)
    exact = cf.chain_mfpt(lam, mu, 82, 563)
    assert abs(exact / 5.0308e4 - 1) < 1e-3
    f = np.array(_pool_map(_schlogl_flux, list(range(1, 17))))
    mfpt = 1.0 / f.mean()
    se = f.std(ddof=1) / np.sqrt(len(f)) / f.mean() * mfpt      # delta method
    print(f"MFPT: WE {mfpt:.4e} +- {se:.1e}, exact {exact:.4e}")
    assert abs(mfpt - exact) < 2 * se
    assert se / mfpt < 0.08


def _schlogl_stationary(seed):
    lam, mu = cf.schlogl_rates(1200)
    pi = cf.chain_stationary(lam, mu)
    p_low = pi[:256].sum()
    cfg = dataclasses.replace(wl.schlogl_config(n_runs=1, seed0=seed, n_iters=400, recycle=False),
                              resample_rule=1)
    M = cfg.m_targ
    ix = np.array([[82]] * M + [[563]] * M, np.int32)
    iw = np.array([p_low / M] * M + [(1 - p_low) / M] * M)
    o = orc.OracleWE(cfg, seed, init_x=ix, init_w=iw)
    acc = np.zeros(cfg.n_bins)
    for it in range(400):
        o.step(1)
        if it >= 100:
            _, w, b, _ = o.walkers()
            acc += np.bincount(b, weights=w, minlength=cfg.n_bins)
    return acc / 300


def test_schlogl_we_stationary_law_matches_pi():
    lam, mu = cf.schlogl_rates(1200)
    pi = cf.chain_stationary(lam, mu)
    edges = wl.uniform_edges(0.0, 800.0, 60)
    exact = np.zeros(60)
    for xv, p in enumerate(pi):
        exact[min(int(np.searchsorted(edges, xv, side="right")) - 1, 59)] += p
    H = np.array(_pool_map(_schlogl_stationary, list(range(1, 9))))
    mean, sem = H.mean(0), H.std(0, ddof=1) / np.sqrt(len(H))
    sel = exact > 1e-6                      # 14 decades, both wells and the barrier
    assert sel.sum() >= 45
    z = (mean[sel] - exact[sel]) / sem[sel]
    assert np.all(np.abs(z) < 4.5), z
    core = exact > 1e-4                     # resolved to a few per cent by 8 replicas
    assert np.all(np.abs(mean[core] / exact[core] - 1) < 0.10)
    assert abs(mean[:19].sum() / pi[:256].sum() - 1) < 0.05   # the low well's weight, X < 253
