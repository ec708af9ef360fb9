"""GPU parity of the split/merge step on hand-built ensembles (Sec. II.B).

A network whose only reaction has rate zero never fires, so one WE
iteration is resampling alone: the ensembles below are built to stress the
split/merge code -- bins far above M with many equal weights (the merge
order hinges on the slot tie-break), bins far below M with equal shares
(the split order hinges on the same tie-break), zero weights, bins on both
sides of 64, 128, 256 and 512 walkers (a merging bin of up to 256 and a
splitting bin of up to 128 is held one to four walkers per lane), and sizes
on both sides of the LDS limit of the per-run working arrays.  Walkers, weights,
bins, parents and the recycled-weight record must equal the oracle's
bit for bit.  Every case runs under both split/merge rules: count-only as
printed (rule 0) and weight-equalizing (rule 1), whose merges also run in
bins at or below M and whose split then follows the merges."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1303_5986_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _frozen_config(n_bins, m_targ, n_runs, rule):
    net = wl.Network.from_reactions(["X", "Y"], [({"X": 1}, {"X": 1, "Y": 1}, 0.0)])
    return wl.WEConfig(name="frozen", net=net, x0=np.array([0, 0], np.int32),
                       bin_coef=np.array([1.0, 0.0]),
                       edges=wl.uniform_edges(0.0, float(n_bins), n_bins), m_targ=m_targ,
                       tau=1.0, n_iters=4, seeds=np.arange(11, 11 + n_runs, dtype=np.uint64),
                       resample_rule=rule)


def _ensemble(rng, counts, weight_kind):
    """counts[b] walkers with X = b (so bin b), interleaved in slot order."""
    xs, ws = [], []
    for b, c in enumerate(counts):
        if c == 0:
            continue
        x = np.zeros((c, 2), np.int32)
        x[:, 0] = b
        x[:, 1] = rng.integers(0, 50, c)      # a passenger species, copied with the parent
        if weight_kind == "equal":
            w = np.full(c, 1.0 / 64.0)
        elif weight_kind == "dyadic":
            w = 2.0 ** -rng.integers(3, 9, c).astype(np.float64)
        elif weight_kind == "zeros":
            w = rng.choice([0.0, 1.0 / 32.0, 1.0 / 128.0], c)
        else:
            w = rng.uniform(0.0, 1.0, c) / c
        xs.append(x)
        ws.append(w)
    x = np.concatenate(xs)
    w = np.concatenate(ws)
    perm = rng.permutation(len(w))
    return x[perm], w[perm]


CASES = [
    # (n_bins, m_targ, per-run bin counts, weight kind)
    (8, 16, [[1, 0, 0, 97, 0, 20, 0, 7], [0, 3, 16, 16, 40, 0, 1, 2]], "equal"),
    (8, 16, [[1, 0, 0, 97, 0, 20, 0, 7], [0, 3, 16, 16, 40, 0, 1, 2]], "dyadic"),
    (8, 16, [[5, 30, 0, 1, 0, 64, 0, 3], [12, 12, 12, 12, 12, 12, 12, 11]], "zeros"),
    # bins on both sides of 64 walkers (one walker per lane up to 64)
    (64, 4, [[64, 65, 63, 1, 33, 2], [4, 5, 64, 3, 0, 60]], "equal"),
    (64, 4, [[64, 65, 63, 1, 33, 2], [4, 5, 64, 3, 0, 60]], "dyadic"),
    (4, 100, [[1, 64, 65, 99], [63, 2, 100, 101]], "dyadic"),
    # bins held four walkers per lane (129-256), and past them
    (4, 480, [[300, 511, 512, 513], [257, 0, 700, 401]], "dyadic"),
    (4, 480, [[300, 511, 512, 513], [257, 0, 700, 401]], "equal"),
    (8, 128, [[128, 129, 200, 256, 257, 1, 0, 3], [130, 0, 255, 64, 65, 9, 8, 7]], "equal"),
    (8, 128, [[128, 129, 200, 256, 257, 1, 0, 3], [130, 0, 255, 64, 65, 9, 8, 7]], "dyadic"),
    (8, 128, [[128, 129, 200, 256, 257, 1, 0, 3], [130, 0, 255, 64, 65, 9, 8, 7]], "uniform"),
    (4, 3000, [[1, 9000, 2500, 499], [0, 3000, 5999, 3001]], "equal"),
    (4, 3000, [[1, 9000, 2500, 499], [700, 0, 11000, 300]], "uniform"),
]


@pytest.mark.parametrize("rule", [0, 1])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_resample_matches_oracle_on_stress_ensembles(case, rule):
    we = __import__("paper_1303_5986_amd.we", fromlist=["we"])
    n_bins, m_targ, counts, kind = CASES[case]
    _say(f"case: resample stress {case} rule {rule}: bins={n_bins} M={m_targ} counts={counts} weights={kind}")
    rng = np.random.default_rng(100 + case)
    cfg = _frozen_config(n_bins, m_targ, len(counts), rule)
    sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=4)
    ors = []
    for r, cnt in enumerate(counts):
        x, w = _ensemble(rng, cnt, kind)
        assert len(w) <= cfg.cap
        sim.set_ensemble(r, x, w)
        ors.append(orc.OracleWE(cfg, int(cfg.seeds[r]), init_x=x, init_w=w))
    for it in range(2):
        sim.step(1)
        for r, o in enumerate(ors):
            o.step(1)
            gx, gw, gb, go = sim.walkers(r)
            ox, ow, ob, oo = o.walkers()
            assert len(gw) == len(ow), (it, r)
            assert np.array_equal(gx, ox), (it, r)
            assert np.array_equal(gw.view(np.uint64), ow.view(np.uint64)), (it, r)
            assert np.array_equal(gb, ob), (it, r)
            assert np.array_equal(go, oo), (it, r)
            assert sim.flux(r, it, 1)[0] == o.flux[it]
    _say(f"   {len(counts)} runs x 2 iterations identical; n after = {[len(o.walkers()[1]) for o in ors]}")
