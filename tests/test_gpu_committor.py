"""GPU parity of the learned-committor pieces: FP32 gradient and Adam kernels
against the FP64 reference, lineage labels against the oracle's, training and
binning on the toggle model."""
import numpy as np
import pytest
from scipy import stats

from oracle import lineage, mlp
from oracle import oracle as orc
from paper_1303_5986_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _we():
    from paper_1303_5986_amd import we
    return we


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("n_in,B", [(8, 1024), (354, 256)])
def test_gradient_matches_fp64_reference(n_in, B):
    """One minibatch through the training kernels (FP32) against the FP64
    chain rule: loss to 1e-5 relative, gradient to 1e-4 of its norm."""
    _say(f"case: MLP loss/grad n_in={n_in} B={B}")
    we = _we()
    rng = np.random.default_rng(n_in)
    npar = we.n_params(n_in)
    p = rng.normal(0, 0.15, npar).astype(np.float32)
    feat = np.concatenate([rng.uniform(0.5, 3.0, n_in), rng.uniform(0.3, 1.5, n_in)]).astype(np.float32)
    x = rng.integers(0, 80, size=(B, n_in)).astype(np.int32)
    y = rng.uniform(0, 1, B).astype(np.float32)
    L, g = we.mlp_loss_grad(n_in, p, feat, x, y)
    Lr, gr = mlp.loss_grad(p.astype(np.float64), feat.astype(np.float64), x, y.astype(np.float64), n_in)
    assert abs(L - Lr) <= 1e-5 * abs(Lr)
    err = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    _say(f"   loss {L:.6f} vs {Lr:.6f}; gradient relative error {err:.2e}")
    assert err <= 1e-4
    assert np.all(np.abs(g - gr) <= 1e-4 * np.abs(gr).max() + 1e-3 * np.abs(gr))


def test_adam_matches_fp64_reference():
    we = _we()
    rng = np.random.default_rng(9)
    n = 5000
    p = rng.normal(size=n).astype(np.float32)
    m = (rng.normal(size=n) * 1e-2).astype(np.float32)
    v = (rng.uniform(size=n) * 1e-4).astype(np.float32)
    g = (rng.normal(size=n) * 1e-2).astype(np.float32)
    q, mq, vq = we.adam_step(p, m, v, g, 1e-3, 5)
    qr, mr, vr = mlp.adam(p.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                          g.astype(np.float64), 1e-3, 5)
    assert np.allclose(mq, mr, rtol=1e-5, atol=1e-9)
    assert np.allclose(vq, vr, rtol=1e-5, atol=1e-12)
    assert np.allclose(q, qr, rtol=1e-5, atol=1e-6)


def _toggle_small(n_runs=2, n_bins=16, m_targ=4, n_iters=40):
    cfg = wl.toggle_config(n_runs=n_runs, n_bins=n_bins, m_targ=m_targ, n_iters=n_iters)
    return cfg


def test_lineage_labels_match_oracle():
    """Records of a lane-path run equal the oracle's ensembles, and the
    device's reverse-pass outcome counts equal the oracle lineage labels
    computed from the oracle's own ensembles."""
    _say("case: lineage labels, toggle 2 runs x 40 iterations")
    we = _we()
    cfg = _toggle_small()
    T = 40
    sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=T, record_iters=T)
    ors = [orc.OracleWE(cfg, int(s)) for s in cfg.seeds]
    recs = []
    S, cap, R = cfg.net.S, cfg.cap, len(cfg.seeds)
    for it in range(T):
        sim.step(1)
        n = np.zeros(R, np.int32)
        x = np.zeros((R, cap, S), np.int32)
        o = np.zeros((R, cap), np.int32)
        rc = np.zeros((R, cap), np.uint8)
        for r, orr in enumerate(ors):
            orr.step(1)
            ox, ow, ob, oo = orr.walkers()
            n[r] = len(ow)
            x[r, :n[r]] = ox
            o[r, :n[r]] = oo
            rc[r, :n[r]] = orr.child_recycled()
        recs.append((n, x, o, rc))
        gn, gx, go, grc = sim.record(it)
        assert np.array_equal(gn, n)
        for r in range(R):
            k = n[r]
            assert np.array_equal(gx[r, :k], x[r, :k])
            assert np.array_equal(go[r, :k], o[r, :k])
            assert np.array_equal(grc[r, :k], rc[r, :k])
    ref = lineage.label_counts(recs, cfg.bin_coef, cfg.a_thr)
    got = sim.record_labels(cfg.bin_coef, cfg.a_thr, T)
    for i in range(T):
        for r in range(R):
            k = recs[i][0][r]
            assert np.array_equal(got[i, r, :k], ref[i, r, :k]), (i, r)
    assert ref.sum() > 0


def test_training_learns_a_committor_and_bins_on_it():
    """Train on 120 recorded iterations of the toggle (4 runs x 64 bins x 16):
    the loss falls, q rises with the hand-chosen coordinate Delta (Spearman >
    0.6), the quantile edges increase, and WE keeps running on learned bins
    with the total weight of every run equal to one."""
    _say("case: committor training on the toggle")
    we = _we()
    cfg = wl.toggle_config(n_runs=4, n_iters=200)
    sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=200, record_iters=120)
    sim.step(120)
    loss, n = sim.train_committor(cfg.bin_coef, cfg.a_thr, steps=600, batch=1024, lr=2e-3, seed=5)
    _say(f"   {n} training states; loss {loss[:10].mean():.4f} -> {loss[-50:].mean():.4f}")
    assert n > 1000
    assert loss[-50:].mean() < 0.9 * loss[:10].mean()
    p, feat, edges = sim.committor_state()
    assert np.all(np.diff(edges) > 0)
    rng = np.random.default_rng(0)
    xs = []
    for r in range(4):
        x, w, b, o = sim.walkers(r)
        xs.append(x)
    X = np.concatenate(xs)
    q = sim.committor(X)
    delta = X @ cfg.bin_coef
    rho = stats.spearmanr(q, delta).correlation
    _say(f"   Spearman(q, Delta) = {rho:.3f}")
    assert rho > 0.6
    sim.use_committor_bins(True)
    sim.step(40)
    for r in range(4):
        x, w, b, o = sim.walkers(r)
        assert abs(w.sum() - 1.0) < 1e-12
        assert b.min() >= 0 and b.max() < cfg.n_bins


def test_learned_bins_gain_over_a_product_count_coordinate():
    """What the trained network gains: with bins on a single product count
    (P1 + 2 D1) the 16 replicas' MFPT estimates of the toggle stay far from
    the brute-force reference after 2000 iterations; binning the same runs on
    the committor learned from their own first 400 iterations brings the RMS
    relative error down by at least a factor of 1.5."""
    _say("case: learned vs plain (product-count) bins, toggle MFPT")
    import dataclasses
    we = _we()
    T, burn = 2000, 100
    base = wl.toggle_config(n_runs=16, n_iters=T)
    delta = np.array([0, 0, 0, 0, 1, -1, 2, -2.0])
    weak = dataclasses.replace(base, bin_coef=np.array([0, 0, 0, 0, 1, 0, 2, 0.0]),
                               edges=wl.uniform_edges(-0.5, 48.0, base.n_bins))
    bf = dataclasses.replace(base, edges=np.array([-1e9, 1e9]), m_targ=1024,
                             seeds=np.arange(1001, 1065, dtype=np.uint64))
    sb = we.sim_from_config(bf, kernel=we.WE_KERNEL_LANE, max_iters=T)
    sb.graph_capture(20)
    sb.graph_replay(T // 20)
    ref, _, _ = sb.mfpt(200)

    def rel_err(sim):
        f = np.stack([sim.flux(r, burn, T - burn) for r in range(16)])
        m = base.tau / f.mean(axis=1)
        return float(np.sqrt(np.mean((m / ref - 1.0) ** 2)))

    plain = we.sim_from_config(weak, kernel=we.WE_KERNEL_LANE, max_iters=T)
    plain.graph_capture(20)
    plain.graph_replay(T // 20)
    learned = we.sim_from_config(weak, kernel=we.WE_KERNEL_LANE, max_iters=T, record_iters=400)
    learned.step(400)
    learned.train_committor(delta, -base.tgt_thr, steps=1500, batch=1024, lr=2e-3, seed=7,
                            edge_mode=1)
    learned.use_committor_bins(True)
    learned.graph_capture(20)
    learned.graph_replay((T - 400) // 20)
    ep, el = rel_err(plain), rel_err(learned)
    _say(f"   reference MFPT {ref:.0f}; RMS relative error plain {ep:.3f}, learned {el:.3f}")
    assert el * 1.5 < ep


@pytest.mark.parametrize("edge_mode", [0, 1])
def test_inference_and_learned_bins_match_oracle_forward(edge_mode):
    """Device inference against the FP64 forward pass on the trained
    parameters: q(x) of the live walkers and of seeded states spanning the
    count range to 2e-5 absolute (the logit to 1e-3 where |z| < 8), and the
    learned bin of every live walker after a step on committor bins equal to
    the oracle's bin of the FP64 logit on the same edges -- except within
    1e-3 of an edge, where the FP32 and FP64 logits may fall either side and
    either neighbouring bin is accepted.  Equal-count edges are quantiles of
    the training states' own FP32 logits, so walkers sitting in those states
    lie on an edge by construction; equal-width edges are not data points,
    and there such walkers must be rare.  Walkers in the same state always
    share a bin."""
    _say(f"case: committor inference + learned bins vs oracle forward, edge_mode={edge_mode}")
    we = _we()
    cfg = wl.toggle_config(n_runs=4, n_iters=80)
    sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=80, record_iters=60)
    sim.step(60)
    sim.train_committor(cfg.bin_coef, cfg.a_thr, steps=300, batch=1024, lr=2e-3, seed=3,
                        edge_mode=edge_mode)
    sim.use_committor_bins(True)
    sim.step(2)
    sim.synchronize()
    p, feat, edges = sim.committor_state()
    S = cfg.net.S
    assert len(edges) == cfg.n_bins + 1 and np.all(np.diff(edges[1:-1]) > 0)
    xs, bs = [], []
    for r in range(len(cfg.seeds)):
        x, w, b, _ = sim.walkers(r)
        xs.append(x)
        bs.append(b)
    X = np.concatenate(xs)
    B = np.concatenate(bs)
    rng = np.random.default_rng(11)
    extra = np.floor(np.exp(rng.uniform(0, np.log(1001), size=(512, S))) - 1).astype(np.int32)
    allx = np.concatenate([X, extra])
    q_dev = sim.committor(allx).astype(np.float64)
    _, _, _, z = mlp.forward(p.astype(np.float64), feat.astype(np.float64), allx, S)
    q_ref = 1.0 / (1.0 + np.exp(-z))
    err_q = np.abs(q_dev - q_ref)
    _say(f"   {len(X)} walkers + {len(extra)} seeded states; max |q - q_ref| {err_q.max():.2e}; "
         f"z range [{z.min():.1f}, {z.max():.1f}]")
    assert err_q.max() <= 2e-5
    mid = np.abs(z) < 8
    z_dev = np.log(q_dev[mid] / (1.0 - q_dev[mid]))
    assert np.abs(z_dev - z[mid]).max() <= 1e-3
    zw = z[:len(X)]
    ref_bins = np.array([orc.bin_of(edges, float(v)) for v in zw])
    inner = edges[1:-1]
    near = np.min(np.abs(zw[:, None] - inner[None, :]), axis=1) <= 1e-3
    assert np.array_equal(B[~near], ref_bins[~near])
    assert np.all(np.abs(B[near] - ref_bins[near]) <= 1)
    _say(f"   bins equal on {np.sum(~near)} walkers; {np.sum(near)} within 1e-3 of an edge")
    if edge_mode == 1:
        assert np.sum(near) <= max(2, len(X) // 100)
    _, inv = np.unique(X, axis=0, return_inverse=True)
    inv = inv.ravel()
    for g in np.unique(inv[near]):
        assert np.unique(B[inv == g]).size == 1


def test_caller_logit_edges_replace_the_trained_ones():
    """we_set_bins with WE_BINS_LEARNED and caller edges: the sim keeps those
    edges, and after a step every live walker sits in the oracle's bin of
    its FP64 logit on them (either neighbour within 1e-3 of an edge);
    non-increasing inner edges, and edges with grid bins, are refused and
    leave the edges unchanged."""
    _say("case: caller-given logit edges for learned bins")
    we = _we()
    cfg = wl.toggle_config(n_runs=4, n_iters=40)
    sim = we.sim_from_config(cfg, kernel=we.WE_KERNEL_LANE, max_iters=40, record_iters=30)
    sim.step(30)
    sim.train_committor(cfg.bin_coef, cfg.a_thr, steps=200, batch=1024, lr=2e-3, seed=5, edge_mode=1)
    p, feat, e_trained = sim.committor_state()
    nb = cfg.n_bins
    e = np.linspace(-6.0, 3.0, nb + 1)
    sim.set_learned_bins(e)
    _, _, got = sim.committor_state()
    assert np.array_equal(got, e)
    bad = e.copy()
    bad[5] = bad[4]
    with pytest.raises(we.WEError):
        sim.set_learned_bins(bad)
    _, _, got = sim.committor_state()
    assert np.array_equal(got, e)
    import ctypes
    st = we.load_library().we_set_bins(sim.handle, ctypes.byref(we._Bins(we.WE_BINS_GRID, None,
                                                                          e.ctypes.data)))
    assert st != 0                           # logit edges go with learned bins only
    sim.step(2)
    sim.synchronize()
    S = cfg.net.S
    for r in range(len(cfg.seeds)):
        x, w, b, _ = sim.walkers(r)
        _, _, _, z = mlp.forward(p.astype(np.float64), feat.astype(np.float64), x, S)
        ref = np.array([orc.bin_of(e, float(v)) for v in z])
        near = np.min(np.abs(z[:, None] - e[None, 1:-1]), axis=1) <= 1e-3
        assert np.array_equal(b[~near], ref[~near])
        assert np.all(np.abs(b[near] - ref[near]) <= 1)
        assert abs(w.sum() - 1.0) < 1e-12
    _say(f"   {nb} caller edges on [-6, 3] kept; bins equal the oracle's")
