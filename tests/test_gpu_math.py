"""The kernels' own reciprocal and reciprocal square root (each a hardware
estimate refined by two Newton-Raphson steps) against correctly rounded IEEE
division and against 1/sqrt taken in extended precision, over the range of
arguments the step meets: densities and pressures of the 1e-10 atmosphere
(p ~ 2e-17) and the products gamma p rho the sound speed takes its
reciprocal square root of (down to ~4e-27), up to ~1e3."""
import numpy as np
import pytest

from paper_2210_06438_amd import hydroagg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MAX_ULP = 1.0


def _ulps(got, exact):
    return np.abs(got - exact) / np.spacing(np.abs(exact))


def test_recip_and_rsqrt_within_one_ulp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(7)
    x = np.concatenate([
        np.logspace(-27, 3, 200001),
        10.0 ** rng.uniform(-27, 3, 200000),
        2.0 ** np.arange(-90, 10, dtype=np.float64),            # powers of two
        np.nextafter(2.0 ** np.arange(-90, 10, dtype=np.float64), 0),
        # atmosphere: rho, gamma p / rho, and gamma p rho (the sound speed's argument)
        np.array([1.0, 5 / 3, 1e-10, (5 / 3) * 2.154e-17 / 1e-10, (5 / 3) * 2.154e-17 * 1e-10]),
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
    # 1/sqrt(x) in extended precision (64-bit significand), error measured
    # there against the double ulp of the exact value
    xl = x.astype(np.longdouble)
    exact = 1 / np.sqrt(xl)
    uq = np.asarray(np.abs(q.astype(np.longdouble) - exact) /
                    np.spacing(exact.astype(np.float64)).astype(np.longdouble), dtype=np.float64)
    print(f"recip: max {ur.max():.3f} ulp, {np.mean(ur > 0.5):.2e} of results not correctly rounded; "
          f"rsqrt: max {uq.max():.3f} ulp, {np.mean(uq > 0.5):.2e} not correctly rounded", flush=True)
    assert ur.max() <= MAX_ULP, x[np.argmax(ur)]
    assert uq.max() <= MAX_ULP, x[np.argmax(uq)]


def test_recip_and_rsqrt_commute_with_power_of_two_scaling():
    """recip(x 2^k) = recip(x) 2^-k and rsq(x 4^k) = rsq(x) 2^-k exactly
    (the bitwise scaling pin of the step relies on both)."""
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
    xs = np.concatenate([x] + [x * 4.0 ** e for e in k])
    xt = torch.from_numpy(xs).to(dev)
    r = torch.empty_like(xt)
    q = torch.empty_like(xt)
    hydroagg.math_check(xt, r, q)
    torch.cuda.synchronize()
    q = q.cpu().numpy().reshape(len(k) + 1, -1)
    for j, e in enumerate(k):
        assert np.array_equal(q[j + 1], q[0] * 2.0 ** (-e)), e
