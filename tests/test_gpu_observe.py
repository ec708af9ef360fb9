"""GPU checks of the observables step through the C ABI: the per-run
histogram of one species accumulated over iterations, on both of its device
paths, against the oracle's ensembles.

Up to 6144 histogram bins the counts are summed per block in LDS (1024
walkers per block, so a run with more slots spans several blocks) and the
same kernel advances the iteration counter; above that, one FP64 atomic per
walker and a separate advance.  The ensembles are the oracle's bit for bit
(lane path), so the accumulated histograms agree up to the order of the FP64
additions (rtol 1e-12), and the iteration counter must have advanced once per
iteration on either path."""
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


@pytest.mark.parametrize("m_targ,hist_hi", [(24, 800), (8, 7000)])
def test_histogram_paths_match_oracle(m_targ, hist_hi):
    """(24, 800): 1440 slots per run, two LDS blocks per run.  (8, 7000):
    7001 bins, the atomic path and the separate advance kernel."""
    _say(f"case: Schloegl histogram, M = {m_targ}, bins 0..{hist_hi}, 3 runs x 30 iterations")
    we = _we()
    cfg = dataclasses.replace(wl.schlogl_config(n_runs=3, seed0=5, n_iters=30), m_targ=m_targ,
                              hist_lo=0, hist_hi=hist_hi)
    assert cfg.cap > 1024 or hist_hi + 1 > 6144
    sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=30)
    ors = [orc.OracleWE(cfg, int(s)) for s in cfg.seeds]
    acc = np.zeros((3, hist_hi + 1))
    for it in range(30):
        sim.step(1)
        for r, o in enumerate(ors):
            o.step(1)
            acc[r] += o.histogram(0, 0, hist_hi)
    h, n = sim.histogram_accum()
    assert n == 30
    assert acc.sum() > 0 and np.count_nonzero(acc) > 50
    np.testing.assert_allclose(h, acc, rtol=1e-12, atol=1e-300)
    _, _, its = sim.counters()
    assert its == 30
    for r, o in enumerate(ors):
        g, w_or = sim.walkers(r), o.walkers()
        assert np.array_equal(g[0], w_or[0]) and np.array_equal(g[1], w_or[1])
