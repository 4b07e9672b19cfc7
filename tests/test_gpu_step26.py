"""The 26-point step on the GPU (hydro_step26: 9 central-upwind flux points
per face, Simpson's rule over each face) against the 26-point oracle:
per sub-grid and per field, max |U_gpu - U_oracle| / max |U_oracle| <= 1e-12
over the interior, amax <= 1e-13 relative, in both output layouts, on the
random smooth state (every sub-grid of the 4096-sub-grid batch), the
periodic brick and the 8^3 sub-grids of the polytrope (atmosphere included);
a uniform state is a fixed point bitwise; the stored layout's ghosts are
never written."""
import numpy as np
import pytest

from paper_2210_06438_amd import hydroagg, workloads
from tests.gpu_util import interior, normwise, normwise_each, oracle_threads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL_AMAX = 1e-13


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _run(dev, U, dt, dx, levels=None, compact=False):
    count, nf = U.shape[0], U.shape[1]
    u_in = torch.from_numpy(U).to(dev)
    u_out = torch.full((count, nf, 8, 8, 8) if compact else U.shape, float("nan"),
                       dtype=torch.float64, device=dev)
    amax = torch.full((count,), float("nan"), dtype=torch.float64, device=dev)
    hydroagg.hydro_step26(hydroagg.subgrids(u_in, u_out, levels=levels), dt, dx, amax)
    torch.cuda.synchronize()
    return u_out.cpu().numpy(), amax.cpu().numpy()


def _check(tag, U, out, amax, ref, ref_amax, compact):
    got = out if compact else interior(out, 8)
    each = normwise_each(got, interior(ref, 8))
    worst = np.unravel_index(np.argmax(each), each.shape)
    print(f"{tag}: worst per-sub-grid normwise {each.max():.2e} at {worst}; amax rel "
          f"{np.max(np.abs(amax - ref_amax) / ref_amax):.2e}", flush=True)
    assert np.all(each <= TOL), (tag, worst, each.max())
    assert np.all(normwise(got, interior(ref, 8)) <= TOL)
    assert np.all(np.abs(amax - ref_amax) <= TOL_AMAX * ref_amax)
    if not compact:
        g = out.copy()
        g[..., 3:11, 3:11, 3:11] = np.nan
        assert np.all(np.isnan(g)), f"{tag}: ghost cells written"


@pytest.mark.parametrize("compact", [False, True])
@pytest.mark.parametrize("nf", [6, 11])
def test_random_smooth_matches_the_26_point_oracle(dev, oracle_mod, nf, compact):
    U = workloads.random_smooth(40, n=8, nfields=nf, seed=900 + nf)
    levels = [i % 4 for i in range(40)]
    dt, dx = 0.002, 0.05
    ref, ref_amax = oracle_mod.step26(U, dt, dx, levels=levels, nthreads=oracle_threads())
    out, amax = _run(dev, U, dt, dx, levels=levels, compact=compact)
    _check(f"random nf={nf} compact={compact}", U, out, amax, ref, ref_amax, compact)


def test_periodic_brick_matches_the_26_point_oracle(dev, oracle_mod):
    U = workloads.brick(seed=1)
    dx = 1.0 / 64
    _, a0 = oracle_mod.step26(U, 0.0, dx)
    dt = 0.4 * dx / float(a0.max())
    ref, ref_amax = oracle_mod.step26(U, dt, dx)
    out, amax = _run(dev, U, dt, dx)
    _check("brick", U, out, amax, ref, ref_amax, False)


def test_polytrope_8cubed_matches_the_26_point_oracle(dev, oracle_mod):
    groups = workloads.polytrope(count=300, seed=3)
    N, levels, U, _ = next(g for g in groups if g[0] == 8)
    U = np.ascontiguousarray(U[:120])
    levels = levels[:120]
    dx = 0.5
    _, a0 = oracle_mod.step26(U, 0.0, dx, levels=levels, nthreads=oracle_threads())
    dt = 0.4 * float(np.min(dx * 2.0 ** (-np.asarray(levels, dtype=np.float64)) / a0))
    ref, ref_amax = oracle_mod.step26(U, dt, dx, levels=levels, nthreads=oracle_threads())
    out, amax = _run(dev, U, dt, dx, levels=levels, compact=True)
    atm = int(np.sum(np.all(U[:, 0] <= workloads.ATMOSPHERE, axis=(1, 2, 3))))
    print(f"polytrope 8^3: {atm} of {U.shape[0]} sub-grids are atmosphere only", flush=True)
    _check("polytrope", U, out, amax, ref, ref_amax, True)


def test_every_subgrid_of_the_4096_batch(dev, oracle_mod):
    count, dx = 4096, 1.0 / 64
    print("26-point: 4096 x 8^3 x 11 fields against the oracle", flush=True)
    U = workloads.random_smooth(count, n=8, nfields=11, seed=2)
    dt = 4.0e-3
    out, amax = _run(dev, U, dt, dx, compact=True)
    ref, ref_amax = oracle_mod.step26(U, dt, dx, nthreads=oracle_threads())
    _check("4096 batch", U, out, amax, ref, ref_amax, True)


def test_uniform_state_is_a_fixed_point(dev):
    U = workloads.random_smooth(3, n=8, nfields=11, seed=905)
    U[:] = U[:, :, :1, :1, :1]
    out, _ = _run(dev, U, 0.01, 0.1)
    assert np.array_equal(interior(out, 8), interior(U, 8))


def test_other_edges_are_refused(dev):
    U = workloads.random_smooth(1, n=12, nfields=6, seed=906)
    u = torch.from_numpy(U).to(dev)
    with pytest.raises(hydroagg.HydroError):
        hydroagg.hydro_step26(hydroagg.subgrids(u, u.clone()), 0.01, 0.1)
