"""The width cost model's HIP kernels (FP32) against the FP64 reference:
forward, MSE gradient, back-propagation, Adam, and a short training run."""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_2210_06438_amd import learned

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return "cuda:0"


def _setup(seed=0, rows=300):
    rng = np.random.default_rng(seed)
    p = (M.init(seed=seed + 1) + 0.05 * rng.normal(size=M.NPARAM)).astype(np.float32)
    x = rng.normal(size=(rows, 5)).astype(np.float32)
    t = rng.normal(size=rows).astype(np.float32)
    return p, x, t


def test_forward_matches_reference(dev):
    p, x, _ = _setup()
    mlp = learned.MLP(params=p, device=dev)
    y = mlp.predict(x)
    ref, _, _ = M.forward(p.astype(np.float64), x.astype(np.float64))
    assert np.max(np.abs(y - ref)) <= 1e-4 * np.max(np.abs(ref))


@pytest.mark.parametrize("rows", [1, 37, 300, 1000])
def test_gradient_matches_reference(dev, rows):
    p, x, t = _setup(seed=rows, rows=rows)
    mlp = learned.MLP(params=p, device=dev)
    loss, g = mlp.gradient(x, t)
    rl, rg = M.loss_and_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    assert abs(float(loss.item()) - rl) <= 1e-5 * rl
    g = g.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(g - rg)) <= 1e-4 * np.max(np.abs(rg))


def test_adam_matches_reference(dev):
    p, x, t = _setup(seed=3)
    mlp = learned.MLP(params=p, device=dev)
    pr = p.astype(np.float64)
    mr = np.zeros_like(pr)
    vr = np.zeros_like(pr)
    for k in range(1, 6):
        _, g = mlp.gradient(x, t)
        gref = g.cpu().numpy().astype(np.float64)
        mlp.adam(lr=1e-3)
        pr, mr, vr = M.adam(pr, gref, mr, vr, k, lr=1e-3)
        got = mlp.params().astype(np.float64)
        assert np.max(np.abs(got - pr)) <= 1e-6 * max(1.0, np.max(np.abs(pr)))


def test_training_decreases_loss(dev):
    rng = np.random.default_rng(9)
    x = rng.normal(size=(256, 5)).astype(np.float32)
    t = (np.sin(x[:, 0]) + 0.5 * x[:, 1] * x[:, 2]).astype(np.float32)
    mlp = learned.MLP(seed=4, device=dev)
    curve = mlp.fit(x, t, epochs=600, lr=3e-3)
    assert curve[-1] < 0.2 * curve[0]
    assert all(np.isfinite(curve))
