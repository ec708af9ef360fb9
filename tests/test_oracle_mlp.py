"""Pins of the FP64 committor-model reference and the lineage labels.

The gradient is checked against central finite differences of the loss (an
independent route through the same mathematics); Adam against its closed
form after one step; the labels against a hand-worked genealogy.
"""
import numpy as np

from oracle import lineage, mlp


def _problem(n_in=8, B=16, seed=0):
    rng = np.random.default_rng(seed)
    npar = mlp.H * n_in + mlp.H + mlp.H * mlp.H + mlp.H + mlp.H + 1
    p = rng.normal(0, 0.3, npar)
    feat = np.concatenate([rng.uniform(0.5, 2.0, n_in), rng.uniform(0.5, 1.5, n_in)])
    x = rng.integers(0, 60, size=(B, n_in))
    y = rng.uniform(0, 1, B)
    return p, feat, x, y


def test_gradient_matches_finite_differences():
    n_in = 8
    p, feat, x, y = _problem(n_in)
    L, g = mlp.loss_grad(p, feat, x, y, n_in)
    rng = np.random.default_rng(1)
    idx = rng.choice(len(p), 60, replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss(pp, feat, x, y, n_in) - mlp.loss(pm, feat, x, y, n_in)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_loss_is_cross_entropy():
    """The stable form equals -(y log q + (1-y) log(1-q))."""
    n_in = 3
    p, feat, x, y = _problem(n_in, B=8)
    _, _, _, z = mlp.forward(p, feat, x, n_in)
    q = 1 / (1 + np.exp(-z))
    ref = np.mean(-(y * np.log(q) + (1 - y) * np.log(1 - q)))
    assert abs(mlp.loss(p, feat, x, y, n_in) - ref) < 1e-12


def test_adam_first_step_closed_form():
    """At t = 1 the bias-corrected moments are g and g^2, so every parameter
    moves by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    q, m, v = mlp.adam(p, np.zeros(50), np.zeros(50), g, 1e-3, 1)
    assert np.allclose(q, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_adam_two_steps_hand_computed():
    """A scalar parameter, gradients g1 = 1 then g2 = -2 (beta 0.9 / 0.999):
    m1 = 0.1, v1 = 0.001, so m1/(1-0.9) = 1, v1/(1-0.999) = 1 and the first
    step is lr/(1+eps); m2 = 0.09 - 0.2 = -0.11, v2 = 0.000999 + 0.004 =
    0.004999, bias-corrected -0.11/0.19 and 0.004999/0.001999, so the second
    step is lr * 0.5789474 / 1.5813763 = 0.3661035 lr upwards.  A slip in the
    bias correction (beta instead of beta^t) moves step 2 by ~11%."""
    lr = 1e-2
    p0 = np.array([0.5])
    p1, m1, v1 = mlp.adam(p0, np.zeros(1), np.zeros(1), np.array([1.0]), lr, 1)
    assert abs(m1[0] - 0.1) < 1e-15 and abs(v1[0] - 0.001) < 1e-16
    assert abs(p1[0] - (0.5 - lr / (1 + 1e-8))) < 1e-15
    p2, m2, v2 = mlp.adam(p1, m1, v1, np.array([-2.0]), lr, 2)
    assert abs(m2[0] + 0.11) < 1e-15 and abs(v2[0] - 0.004999) < 1e-16
    step = (0.11 / 0.19) / (np.sqrt(0.004999 / 0.001999) + 1e-8)
    assert abs(step - 0.3661035) < 1e-6
    assert abs(p2[0] - (p1[0] + lr * step)) < 1e-14


def test_adam_constant_gradient_takes_equal_steps():
    """With a constant gradient the bias-corrected moments are exactly g and
    g^2 at every t, so every step is lr g / (|g| + eps) (t = 1..6)."""
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 7):
        q, m, v = mlp.adam(p, m, v, g, 1e-3, t)
        assert np.allclose(p - q, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        p = q


def test_lineage_labels_hand_worked():
    """Two iterations, one run, three slots.  Iteration 1 (children):
    slot 0 from parent 0, flagged recycled (B); slot 1 from parent 0, in A;
    slot 2 from parent 1, neither.  Iteration 0 parents then have counts
    (1,1) for slot 0 and the (still unresolved) child's (0,0) for slot 1."""
    S = 1
    a_coef, a_thr = [1.0], 5.0
    n = np.array([3])
    x0 = np.array([[[10], [20], [30]]])
    x1 = np.array([[[7], [3], [40]]])
    rec0 = (n, x0, np.array([[0, 1, 2]]), np.array([[0, 0, 0]]))
    rec1 = (n, x1, np.array([[0, 0, 1]]), np.array([[1, 0, 0]]))
    cnt = lineage.label_counts([rec0, rec1], a_coef, a_thr)
    assert cnt[0, 0, 0].tolist() == [1, 1]
    assert cnt[0, 0, 1].tolist() == [0, 0]
    assert cnt[0, 0, 2].tolist() == [0, 0]
    assert cnt[1].sum() == 0
