"""The kernels' own reciprocal and square root (Newton-Raphson reciprocal;
Goldschmidt square root with an FMA residual correction) against correctly
rounded IEEE division and sqrt, over the range of arguments the step meets:
densities and pressures of the 1e-10 atmosphere (p ~ 2e-17) up to ~1e3."""
import numpy as np
import pytest

from paper_2210_06438_amd import hydroagg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MAX_ULP = 1.0


def _ulps(got, exact):
    return np.abs(got - exact) / np.spacing(np.abs(exact))


def test_recip_and_sqrt_within_one_ulp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(7)
    x = np.concatenate([
        np.logspace(-17, 3, 200001),
        10.0 ** rng.uniform(-17, 3, 200000),
        2.0 ** np.arange(-56, 10, dtype=np.float64),            # powers of two
        np.nextafter(2.0 ** np.arange(-56, 10, dtype=np.float64), 0),
        np.array([1.0, 5 / 3, 1e-10, (5 / 3) * 2.154e-17 / 1e-10]),
    ])
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(x).to(dev)
    r = torch.empty_like(xt)
    q = torch.empty_like(xt)
    hydroagg.math_check(xt, r, q)
    torch.cuda.synchronize()
    r = r.cpu().numpy()
    q = q.cpu().numpy()
    ur = _ulps(r, 1.0 / x)
    uq = _ulps(q, np.sqrt(x))
    print(f"recip: max {ur.max():.3f} ulp, {np.mean(ur > 0.5):.2e} of results not correctly rounded; "
          f"sqrt: max {uq.max():.3f} ulp, {np.mean(uq > 0.5):.2e} not correctly rounded", flush=True)
    assert ur.max() <= MAX_ULP, x[np.argmax(ur)]
    assert uq.max() <= MAX_ULP, x[np.argmax(uq)]


def test_recip_commutes_with_power_of_two_scaling():
    """recip(x 2^k) = recip(x) 2^-k exactly (the bitwise scaling pin of the
    step relies on it)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(8)
    x = 10.0 ** rng.uniform(-12, 2, 4096)
    k = np.array([-8.0, -2.0, -1.0, 1.0, 2.0, 8.0])
    xs = np.concatenate([x] + [x * 2.0 ** e for e in k])
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(xs).to(dev)
    r = torch.empty_like(xt)
    q = torch.empty_like(xt)
    hydroagg.math_check(xt, r, q)
    torch.cuda.synchronize()
    r = r.cpu().numpy().reshape(len(k) + 1, -1)
    for j, e in enumerate(k):
        assert np.array_equal(r[j + 1], r[0] * 2.0 ** (-e)), e
