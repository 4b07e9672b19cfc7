"""Pins for the FP64 width cost-model reference: its back-propagated
gradient against central finite differences of the loss, the Adam step
against its closed form on one step, a hand-wired network with a known
output, and the sizes."""
import numpy as np

from oracle import mlp_oracle as M


def test_parameter_count():
    assert M.NPARAM == 4609


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = M.init(seed=1) + 0.05 * rng.normal(size=M.NPARAM)
    x = rng.normal(size=(17, 5))
    t = rng.normal(size=17)
    loss, g = M.loss_and_grad(p, x, t)
    idx = np.r_[rng.integers(0, M.NPARAM, 300), np.arange(M.NPARAM - 70, M.NPARAM)]
    h = 1e-6
    for i in idx:
        e = np.zeros(M.NPARAM)
        e[i] = h
        fd = (M.loss_and_grad(p + e, x, t)[0] - M.loss_and_grad(p - e, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_first_step_is_sign_times_lr():
    # after one step from m = v = 0 with bias correction, the update is
    # lr * g / (|g| + eps), i.e. lr * sign(g) for |g| >> eps
    g = np.array([3.0, -2.0, 1e-3, 0.0])
    p, m, v = M.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), step=1, lr=0.01, eps=1e-12)
    assert np.allclose(p[:3], -0.01 * np.sign(g[:3]), rtol=1e-9)
    assert p[3] == 0.0


def test_training_reduces_the_loss():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(64, 5))
    t = np.sin(x[:, 0]) + 0.5 * x[:, 1] * x[:, 2]
    p = M.init(seed=3)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = M.loss_and_grad(p, x, t)[0]
    for k in range(1, 301):
        loss, g = M.loss_and_grad(p, x, t)
        p, m, v = M.adam(p, g, m, v, k, lr=3e-3)
    assert M.loss_and_grad(p, x, t)[0] < 0.2 * l0


def test_hand_wired_network_computes_abs():
    # W1 rows 0/1 take +-(x0 - 2 x3); W2 copies hidden units 0 and 1 into
    # units 5 and 9; W3 sums those and b3 adds 0.5, so y = |x0 - 2 x3| + 0.5.
    # A transposed weight matrix or a swapped layer would break this.
    d = {k: np.zeros(s) for k, s in M.SIZES.items()}
    d["W1"][0, 0], d["W1"][0, 3] = 1.0, -2.0
    d["W1"][1, 0], d["W1"][1, 3] = -1.0, 2.0
    d["W2"][5, 0] = 1.0
    d["W2"][9, 1] = 1.0
    d["W3"][5] = d["W3"][9] = 1.0
    d["b3"][0] = 0.5
    p = M.pack(d)
    x = np.random.default_rng(4).normal(size=(50, 5))
    y, h1, h2 = M.forward(p, x)
    assert np.array_equal(y, np.abs(x[:, 0] - 2 * x[:, 3]) + 0.5)
    assert np.count_nonzero(h2[:, [i for i in range(64) if i not in (5, 9)]]) == 0
